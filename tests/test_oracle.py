"""Pins of the CPU oracle to facts that do not come from the oracle itself.

Closed-form 2x2 pencils (tests/golden/two_by_two.txt), inputs with a prescribed
spectrum, exact high-precision spectra (mpmath), Sylvester inertia, trace and
determinant invariants, special cases that reduce to an SVD, residuals and
orthogonality, status paths, and the long-double instantiation as adjudicator."""
import numpy as np
import pytest

import jjgen
import oracle
from _pins import EPS, kappa_s, rel_err, residuals, spectrum_mp, two_by_two_G, two_by_two_cases


@pytest.mark.parametrize("case", range(len(two_by_two_cases())))
@pytest.mark.parametrize("precision", ["double", "long"])
def test_two_by_two_closed_form(case, precision):
    a, J, expect = two_by_two_cases()[case]
    G = two_by_two_G(a)
    r = oracle.solve(G, J, precision=precision, final_G=True)
    assert r["status"] == 0
    assert r["rotations"] == 1  # one rotation diagonalises a 2x2 pencil
    assert rel_err(r["lam"], expect) <= 4 * EPS
    # the final columns are orthogonal and H = G J G^* is preserved
    Gf = np.asarray(r["G"], dtype=np.complex128)
    assert abs(np.vdot(Gf[:, 0], Gf[:, 1])) <= 8 * EPS * np.linalg.norm(Gf[:, 0]) * np.linalg.norm(Gf[:, 1])
    H0 = G @ np.diag(J.astype(float)) @ G.conj().T
    H1 = Gf @ np.diag(J.astype(float)) @ Gf.conj().T
    assert np.max(np.abs(H1 - H0)) <= 16 * EPS * np.max(np.abs(H0))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,lo,hi", [(8, 1e-3, 1e3), (32, 1e-6, 1.0), (64, 1e-3, 1e3), (96, 1e-12, 1.0)])
def test_known_spectrum(cplx, n, lo, hi):
    G, J, lam = jjgen.make(n, cplx, n // 3, lo, hi, seed=100 + n)
    r = oracle.solve(G, J)
    assert r["status"] == 0
    ref = np.sort(lam)[::-1]
    # the stored G is a rounding of the exact construction: its spectrum differs
    # from the prescribed one by about eps * kappa(G_s) relatively
    assert rel_err(r["lam"], ref) <= 16 * EPS * kappa_s(G)


def test_config1_known_spectrum():
    G, J, lam = jjgen.config(1)
    r = oracle.solve(G, J)
    assert r["status"] == 0
    assert rel_err(r["lam"], np.sort(lam)[::-1]) <= 16 * EPS * kappa_s(G)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_exact_spectrum_mpmath(cplx, seed):
    n = 10
    G, J, _ = jjgen.make(n, cplx, 4, 1e-4, 1e2, seed=200 + seed)
    exact = spectrum_mp(G, J)
    exact_f = np.array([float(x) for x in exact])
    k = kappa_s(G)
    rd = oracle.solve(G, J)
    assert rd["status"] == 0
    assert rel_err(rd["lam"], exact_f) <= 16 * EPS * k
    rl = oracle.solve(G, J, precision="long")
    import mpmath
    with mpmath.workdps(50):
        err_l = max(abs((mpmath.mpf(str(rl["lam"][i])) - exact[i]) / exact[i]) for i in range(n))
    assert float(err_l) <= 16 * 2.0 ** -64 * k


@pytest.mark.parametrize("cplx", [False, True])
def test_inertia_trace_logdet(cplx):
    n = 48
    G, J, _ = jjgen.make(n, cplx, 17, 1e-4, 1e4, seed=7)
    r = oracle.solve(G, J)
    lam = r["lam"]
    # Sylvester: the inertia of H equals the sign counts of J
    assert np.sum(lam > 0) == np.sum(J > 0) and np.sum(lam < 0) == np.sum(J < 0)
    # trace(H) = sum_i j_i ||g_i||^2 of the input columns
    tr = np.sum(J.astype(float) * np.sum(np.abs(G) ** 2, axis=0))
    assert abs(np.sum(lam) - tr) <= 8 * n * EPS * np.sum(np.abs(lam))
    # |det H| = |det G|^2
    _, logdet = np.linalg.slogdet(G)
    assert abs(np.sum(np.log(np.abs(lam))) - 2 * logdet) <= 8 * n * EPS * kappa_s(G)


@pytest.mark.parametrize("cplx", [False, True])
def test_residual_and_orthogonality(cplx):
    n = 64
    G, J, _ = jjgen.make(n, cplx, 20, 1e-3, 1e3, seed=9)
    r = oracle.solve(G, J)
    res, orth = residuals(G, J, r["lam"], r["V"])
    assert res <= 64 * n * EPS * kappa_s(G)
    assert orth <= 8 * n * EPS


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("cplx", [False, True])
def test_definite_reduces_to_svd(sign, cplx):
    # J = +-I: H = +-G G^*, eigenvalues +-sigma_i(G)^2 (LAPACK SVD; a well
    # conditioned G so that its absolute accuracy is also relative)
    n = 40
    G, _, _ = jjgen.make(n, cplx, n, 1.0, 10.0, seed=21)
    J = np.full(n, sign, dtype=np.int8)
    r = oracle.solve(G, J)
    s = np.linalg.svd(G, compute_uv=False)
    ref = np.sort(sign * s ** 2)[::-1]
    assert r["status"] == 0
    assert rel_err(r["lam"], ref) <= 8 * n * EPS


def test_diagonal_and_orthogonal_columns_need_no_rotation():
    d = np.array([3.0, -0.5, 2.0, 1e-3, 7.0, 0.25])
    J = np.array([1, -1, -1, 1, 1, -1], dtype=np.int8)
    r = oracle.solve(np.diag(d), J)
    assert r["status"] == 0 and r["rotations"] == 0 and r["sweeps"] == 1
    assert np.array_equal(r["lam"], np.sort(J * d ** 2)[::-1])
    # Sylvester-Hadamard matrix: exactly orthogonal columns
    H2 = np.array([[1.0, 1.0], [1.0, -1.0]])
    Hd = H2
    for _ in range(3):
        Hd = np.kron(Hd, H2)
    Jh = np.array([1, -1] * 8, dtype=np.int8)
    r = oracle.solve(Hd * np.arange(1, 17), Jh)
    assert r["rotations"] == 0
    assert np.array_equal(r["lam"], np.sort(Jh * 16.0 * np.arange(1, 17) ** 2)[::-1])


def test_tiny_orders():
    r = oracle.solve(np.array([[-3.0]]), np.array([-1], dtype=np.int8))
    assert r["status"] == 0 and r["lam"][0] == -9.0 and r["V"][0, 0] == -1.0
    r = oracle.solve(np.zeros((0, 0)), np.zeros(0, dtype=np.int8))
    assert r["status"] == 0 and r["lam"].size == 0


def test_status_paths():
    G, J, _ = jjgen.config(1)
    assert oracle.solve(G, J, max_sweeps=1)["status"] == 1
    Gb = G.copy()
    Gb[3, 5] = np.nan
    assert oracle.solve(Gb, J)["status"] == 3
    Jb = J.copy()
    Jb[0] = 0
    assert oracle.solve(G, Jb)["status"] == -2
    # two equal columns with opposite signs: G^* G is singular and the
    # hyperbolic rotation does not exist (|theta| = 1)
    Gd = G.copy()
    Gd[:, 1] = Gd[:, 0]
    Jd = J.copy()
    Jd[0], Jd[1] = 1, -1
    assert oracle.solve(Gd, Jd)["status"] == 2


@pytest.mark.parametrize("cplx", [False, True])
def test_long_double_adjudicator_agrees(cplx):
    G, J, _ = jjgen.make(64, cplx, 30, 1e-6, 1.0, seed=33)
    rd = oracle.solve(G, J)
    rl = oracle.solve(G, J, precision="long")
    assert rd["status"] == rl["status"] == 0
    assert rel_err(rd["lam"], rl["lam"].astype(np.float64)) <= 8 * EPS * kappa_s(G)


def test_resume_from_intermediate_factor():
    # the whole state between sweeps is the current G: solving again from the
    # G after two sweeps gives the same eigenproblem
    G, J, _ = jjgen.make(48, False, 20, 1e-4, 1.0, seed=44)
    full = oracle.solve(G, J)
    part = oracle.solve(G, J, max_sweeps=2, final_G=True)
    assert part["status"] == 1
    again = oracle.solve(part["G"], J)
    assert rel_err(again["lam"], full["lam"]) <= 16 * EPS * kappa_s(G)


def test_sort_order_and_vectors_follow_eigenvalues():
    G, J, _ = jjgen.make(20, True, 9, 1e-2, 1e2, seed=55)
    r = oracle.solve(G, J)
    lam = r["lam"]
    assert np.all(np.diff(lam) <= 0)
    # each V column is the eigenvector of its lambda: H v = lambda v
    Jd = J.astype(float)
    for k in range(20):
        v = r["V"][:, k]
        Hv = G @ (Jd * (G.conj().T @ v))
        assert np.linalg.norm(Hv - lam[k] * v) <= 1e3 * EPS * np.max(np.abs(lam)) * kappa_s(G)
