"""Pins of the oracle's front end H -> G J G^* (Bunch-Parlett factorization
with complete pivoting and the diagonalisation of its 2x2 blocks; paper,
Section 2.2, eq. 2.5) and of the rectangular solve (singular H of rank r,
G of n x r), each against facts independent of the oracle: the definition of
the factorization (G J G^* = H), Sylvester's inertia, closed-form 2x2
eigenvalues, the pivot rule's threshold, exact diagonal cases, LAPACK's
eigenvalues of well-conditioned H, mpmath at 50 digits, and the rank of a
singular H built exactly.  Planted mistakes in the front end must each fail
one of these pins.  CPU only."""
import os
import shutil

import mpmath
import numpy as np
import pytest

import jjgen
import oracle

EPS = 2.0 ** -53
ALPHA = (1 + np.sqrt(17.0)) / 8


def _herm(n, cplx, seed, lo=0.1, hi=10.0):
    """Hermitian H = Q diag(lam) Q^* with |lam| log-uniform in [lo, hi] (the
    seeded generator's G J G^*, formed in double)."""
    G, J, lam = jjgen.make(n, cplx, n // 2, lo, hi, seed=seed)
    H = G @ (J.astype(float)[:, None] * G.conj().T)
    H = (H + H.conj().T) / 2
    return H, lam


def _recon(r):
    G, J = r["G"], r["J"].astype(float)
    return G @ (J[:, None] * G.conj().T)


def bp_battery(factor, solve_rect):
    """Run every front-end pin; return the names of those that fail."""
    fails = []

    def check(name, ok):
        if not ok:
            fails.append(name)

    # P-F1 definition: G J G^* = H to a few n eps of max|h_ij|, and inertia
    for cplx in (False, True):
        for n in (3, 7, 40):
            H, lam = _herm(n, cplx, seed=71 + n + 100 * cplx)
            r = factor(H)
            ok = r["status"] == 0 and r["rank"] == n
            R = _recon(r) if ok else H * np.nan
            check("reconstruct n=%d cplx=%d" % (n, cplx),
                  ok and np.max(np.abs(R - H)) <= 8 * n * EPS * np.max(np.abs(H)))
            check("inertia n=%d cplx=%d" % (n, cplx), ok and np.sum(r["J"] > 0) == np.sum(lam > 0))
            # lower block triangular after the row permutation, blocks of order 1 or 2
            if ok:
                Gp = r["G"][r["perm"], :]
                piv = r["pivsize"]
                start = np.zeros(n, dtype=int)
                c = 0
                while c < n:
                    start[c:c + piv[c]] = c
                    c += max(piv[c], 1)
                tri = all(np.all(Gp[:start[c], c] == 0) for c in range(n))
                check("block triangular n=%d cplx=%d" % (n, cplx), tri and set(piv.tolist()) <= {1, 2})
    # P-F2 closed-form 2x2: a 2x2 pivot yields orthogonal columns whose
    # j ||g||^2 are the eigenvalues ((a+c) +- sqrt((a-c)^2 + 4|b|^2)) / 2
    for a, b, c in ((0.3, 2.0, -0.5), (1.0, 1.5 - 2.0j, 0.25), (0.0, 1.0, 0.0)):
        H = np.array([[a, np.conj(b)], [b, c]], dtype=np.complex128 if isinstance(b, complex) else np.float64)
        r = factor(H)
        G, J = r["G"], r["J"].astype(float)
        ev = np.sort([((a + c) + np.sqrt((a - c) ** 2 + 4 * abs(b) ** 2)) / 2,
                      ((a + c) - np.sqrt((a - c) ** 2 + 4 * abs(b) ** 2)) / 2])
        ok = r["rank"] == 2 and list(r["pivsize"]) == [2, 2]
        got = np.sort(J * np.sum(np.abs(G) ** 2, axis=0)) if ok else np.full(2, np.nan)
        check("2x2 pivot eigenvalues %s" % (b,), ok and np.max(np.abs(got - ev) / np.abs(ev)) <= 8 * EPS)
        check("2x2 pivot orthogonal %s" % (b,), ok and abs(np.vdot(G[:, 0], G[:, 1])) <= 8 * EPS * np.max(np.abs(ev)))
    # P-F3 the pivot rule's threshold alpha = (1 + sqrt 17) / 8 on [[x, 1], [1, 0]]
    for x, want in ((ALPHA * 1.0001, [1, 1]), (ALPHA * 0.9999, [2, 2])):
        r = factor(np.array([[x, 1.0], [1.0, 0.0]]))
        check("pivot rule x=%.6f" % x, list(r["pivsize"]) == want)
    # P-F4 diagonal H: G = diag(sqrt|h|) in H's row order, J = sign(h), columns by decreasing |h|
    h = np.array([0.5, -3.0, 2.0, -0.25, 7.0, 1e-3])
    r = factor(np.diag(h))
    order = np.argsort(-np.abs(h), kind="stable")
    Gd = np.zeros((6, 6))
    for c, i in enumerate(order):
        Gd[i, c] = np.sqrt(abs(h[i]))
    check("diagonal exact", r["rank"] == 6 and np.array_equal(r["G"], Gd) and
          np.array_equal(r["J"], np.sign(h[order]).astype(np.int8)))
    # P-F5 singular H = B J0 B^T, B integer n x r: the rank found is r and the
    # rectangular solve returns H's nonzero eigenvalues
    rng = np.random.default_rng(5)
    for cplx in (False, True):
        n, rk = 9, 5
        B = rng.integers(-3, 4, size=(n, rk)).astype(float)
        if cplx:
            B = B + 1j * rng.integers(-3, 4, size=(n, rk))
        J0 = np.array([1, -1, 1, 1, -1])
        H = B @ (J0[:, None] * B.conj().T)
        r = factor(H)
        check("singular rank cplx=%d" % cplx, r["rank"] == rk and np.sum(r["J"] > 0) == 3)
        if r["rank"] == rk:
            s = solve_rect(r["G"], r["J"])
            ev = np.linalg.eigvalsh(H)
            nz = np.sort(ev[np.argsort(-np.abs(ev))[:rk]])[::-1]
            check("singular eigenvalues cplx=%d" % cplx,
                  s["status"] == 0 and np.max(np.abs(s["lam"] - nz) / np.abs(nz)) <= 1e-12)
            check("singular eigenvectors cplx=%d" % cplx,
                  s["status"] == 0 and np.linalg.norm(H @ s["V"] - s["V"] * s["lam"][None, :]) <=
                  64 * n * EPS * np.linalg.norm(H))
    # P-F6 end to end against mpmath at 50 digits (n = 12) and LAPACK (n = 60,
    # eigenvalues within [0.1, 10], where its absolute accuracy is relative)
    for cplx in (False, True):
        H, _ = _herm(12, cplx, seed=400 + cplx)
        r = factor(H)
        s = solve_rect(r["G"], r["J"])
        mpmath.mp.dps = 50
        M = mpmath.matrix(H.tolist())
        ev = mpmath.eighe(M, eigvals_only=True) if cplx else mpmath.eigsy(M, eigvals_only=True)
        ref = np.sort(np.array([float(x) for x in ev]))[::-1]
        check("mpmath cplx=%d" % cplx, s["status"] == 0 and np.max(np.abs(s["lam"] - ref) / np.abs(ref)) <= 1e-13)
        H, _ = _herm(60, cplx, seed=500 + cplx)
        r = factor(H)
        s = solve_rect(r["G"], r["J"])
        ref = np.sort(np.linalg.eigvalsh(H))[::-1]
        check("lapack cplx=%d" % cplx, s["status"] == 0 and np.max(np.abs(s["lam"] - ref) / np.abs(ref)) <= 1e-12)
    return fails


def null_battery(nullspace, factor, solve_rect):
    """Pins of the null-space completion: orthonormal columns orthogonal to U,
    the projector identity Z Z^* + U U^* = I, and H Z = 0 for a singular H."""
    fails = []
    rng = np.random.default_rng(17)
    for cplx in (False, True):
        for n, r in ((30, 11), (9, 1), (12, 11)):
            X = rng.standard_normal((n, r)) + (1j * rng.standard_normal((n, r)) if cplx else 0)
            U, _ = np.linalg.qr(X)
            Z = nullspace(U)
            ok = Z.shape == (n, n - r)
            tag = "n=%d r=%d cplx=%d" % (n, r, cplx)
            if not ok:
                fails.append("shape " + tag)
                continue
            if np.max(np.abs(Z.conj().T @ Z - np.eye(n - r))) > 16 * n * EPS:
                fails.append("orthonormal " + tag)
            if np.max(np.abs(U.conj().T @ Z)) > 16 * n * EPS:
                fails.append("orthogonal to U " + tag)
            if np.max(np.abs(Z @ Z.conj().T + U @ U.conj().T - np.eye(n))) > 16 * n * EPS:
                fails.append("projector " + tag)
    # the null space of a singular H through the front end and the rectangular solve
    for cplx in (False, True):
        n, rk = 11, 6
        B = rng.integers(-3, 4, size=(n, rk)).astype(float)
        if cplx:
            B = B + 1j * rng.integers(-3, 4, size=(n, rk))
        H = B @ (np.array([1, -1, 1, -1, 1, 1])[:, None] * B.conj().T)
        f = factor(H)
        sv = solve_rect(f["G"], f["J"])
        Z = nullspace(sv["V"])
        if Z.shape != (n, n - rk) or np.linalg.norm(H @ Z) > 64 * n * EPS * np.linalg.norm(H):
            fails.append("H Z = 0 cplx=%d" % cplx)
    return fails


def test_nullspace_battery():
    assert null_battery(oracle.nullspace, _factor(), _solve_rect()) == []
    # r = 0: Q = I;  r = n: nothing to complete
    assert np.array_equal(oracle.nullspace(np.zeros((5, 0))), np.eye(5))
    assert oracle.nullspace(np.eye(4)).shape == (4, 0)


NULL_MUTATIONS = {
    "reflectors_forward_order": ("for (int k = r - 1; k >= 0; k--) {", "for (int k = 0; k < r; k++) {"),
    "dot_without_conj_e": ("for (int i = k; i < n; i++) s += FN(bp_conj)(v[i]) * e[i];",
                           "for (int i = k; i < n; i++) s += v[i] * e[i];"),
    "reflector_factor_one": ("const ST f = s * ((RT)2 / beta[k]);", "const ST f = s * ((RT)1 / beta[k]);"),
    "identity_rows_from_top": ("for (int c = 0; c < n - r; c++) E[(size_t)c * n + r + c] = 1;",
                               "for (int c = 0; c < n - r; c++) E[(size_t)c * n + c] = 1;"),
    "last_column_not_updated": ("for (int j = k; j < r; j++) {", "for (int j = k; j < r - 1; j++) {"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(NULL_MUTATIONS))
def test_nullspace_mutation_is_caught(name, tmp_path):
    old, new = NULL_MUTATIONS[name]
    src = os.path.dirname(oracle.__file__)
    for f in ("jj_oracle.c", "jj_oracle_body.inc", "jj_bp_body.inc"):
        shutil.copy(os.path.join(src, f), tmp_path / f)
    body = (tmp_path / "jj_bp_body.inc").read_text()
    assert body.count(old) >= 1, "mutation target not found in the source"
    (tmp_path / "jj_bp_body.inc").write_text(body.replace(old, new))
    so = str(tmp_path / "libmut.so")
    oracle.build(out=so, src_dir=str(tmp_path))
    lib = oracle.load(so)
    with np.errstate(all="ignore"):
        try:
            fails = null_battery(lambda U: oracle.nullspace(U, lib=lib), _factor(lib), _solve_rect(lib))
        except (np.linalg.LinAlgError, ValueError):
            fails = ["exception"]
    assert fails, "planted mistake %r was not caught by any pin" % name


def _factor(lib=None, precision="double"):
    return lambda H: oracle.bp_factor(H, precision=precision, lib=lib)


def _solve_rect(lib=None):
    return lambda G, J: oracle.solve(G, J, lib=lib)


def test_front_end_battery():
    assert bp_battery(_factor(), _solve_rect()) == []


def test_front_end_long_double_agrees():
    # the same factorization in long double: eigenvalues through the long-double
    # solve agree with the double pipeline to the input's conditioning
    H, _ = _herm(50, True, seed=77, lo=1e-3, hi=1.0)
    rd = oracle.bp_factor(H)
    rl = oracle.bp_factor(H, precision="long")
    assert rd["rank"] == rl["rank"] == 50
    ld = oracle.solve(rd["G"], rd["J"], vectors=False)["lam"]
    ll = oracle.solve(rl["G"], rl["J"], precision="long", vectors=False)["lam"].astype(float)
    assert np.max(np.abs(ld - ll) / np.abs(ll)) <= 1e-10


def test_rectangular_solve_matches_square():
    # G = Q_r Gs (n x r, Q_r with orthonormal columns) has the nonzero
    # eigenvalues of Gs J Gs^T: the rectangular solve against the square one
    rng = np.random.default_rng(9)
    n, r = 40, 23
    Gs, J, _ = jjgen.make(r, False, 10, 1e-4, 1.0, seed=31)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    G = Q[:, :r] @ Gs
    a = oracle.solve(G, J, vectors=False)
    b = oracle.solve(Gs, J, vectors=False)
    assert a["status"] == 0 and b["status"] == 0
    assert np.max(np.abs(a["lam"] - b["lam"]) / np.abs(b["lam"])) <= 1e-11


def test_front_end_empty_and_zero():
    r = oracle.bp_factor(np.zeros((0, 0)))
    assert r["status"] == 0 and r["rank"] == 0
    r = oracle.bp_factor(np.zeros((4, 4)))
    assert r["status"] == 0 and r["rank"] == 0
    Hb = np.eye(3)
    Hb[2, 0] = np.nan
    assert oracle.bp_factor(Hb)["status"] == 3


BP_MUTATIONS = {
    "alpha_half": ("const RT alpha = (1 + R_SQRT((RT)17)) / 8;", "const RT alpha = (RT)0.5;"),
    "schur_sign_1x1": ("ST v = A[(size_t)j * n + i] - L[(size_t)k * n + i] * FN(bp_conj)(A[(size_t)k * n + j]);",
                       "ST v = A[(size_t)j * n + i] + L[(size_t)k * n + i] * FN(bp_conj)(A[(size_t)k * n + j]);"),
    "schur_missing_conj_1x1": (
        "ST v = A[(size_t)j * n + i] - L[(size_t)k * n + i] * FN(bp_conj)(A[(size_t)k * n + j]);",
        "ST v = A[(size_t)j * n + i] - L[(size_t)k * n + i] * (A[(size_t)k * n + j]);"),
    "inverse_2x2_wrong_entry": ("L[(size_t)k * n + i] = (x * e22 - y * b) / det;",
                                "L[(size_t)k * n + i] = (x * e22 - y * FN(bp_conj)(b)) / det;"),
    "inverse_2x2_swapped_diag": ("L[(size_t)k * n + i] = (x * e22 - y * b) / det;",
                                 "L[(size_t)k * n + i] = (x * e11 - y * b) / det;"),
    "rotation_sign_2x2": ("gp[i] = (l1 * cs - l2 * (sn * ph)) * s1;", "gp[i] = (l1 * cs + l2 * (sn * ph)) * s1;"),
    "phase_conj_2x2": ("gp[n + i] = (l1 * sn + l2 * (cs * ph)) * s2;",
                       "gp[n + i] = (l1 * sn + l2 * (cs * FN(bp_conj)(ph))) * s2;"),
    "eigen_2x2_sign": ("const RT mu1 = a - t * ab, mu2 = e + t * ab;", "const RT mu1 = a + t * ab, mu2 = e - t * ab;"),
    "rows_not_unpermuted": ("Gout[(size_t)c * n + perm[i]] = (double)gp[i];", "Gout[(size_t)c * n + i] = (double)gp[i];"),
    "second_swap_wrong_index": ("FN(bp_swap)(A, L, perm, n, k + 1, p0);", "FN(bp_swap)(A, L, perm, n, k + 1, q0);"),
    "no_rank_stop": ("if (!(mu0 > tol * hmax)) break;", "if (!(mu0 > 0)) break;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(BP_MUTATIONS))
def test_front_end_mutation_is_caught(name, tmp_path):
    old, new = BP_MUTATIONS[name]
    src = os.path.dirname(oracle.__file__)
    for f in ("jj_oracle.c", "jj_oracle_body.inc", "jj_bp_body.inc"):
        shutil.copy(os.path.join(src, f), tmp_path / f)
    body = (tmp_path / "jj_bp_body.inc").read_text()
    assert body.count(old) >= 1, "mutation target not found in the front-end source"
    (tmp_path / "jj_bp_body.inc").write_text(body.replace(old, new))
    so = str(tmp_path / "libmut.so")
    oracle.build(out=so, src_dir=str(tmp_path))
    lib = oracle.load(so)
    with np.errstate(all="ignore"):
        try:
            fails = bp_battery(_factor(lib), _solve_rect(lib))
        except (np.linalg.LinAlgError, ValueError, ZeroDivisionError):
            fails = ["exception"]
    assert fails, "planted mistake %r was not caught by any pin" % name
