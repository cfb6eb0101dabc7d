"""Checks that pin an eigen-solver's output to facts independent of it.

Used by the oracle pin tests and the mutation tests (which rebuild the oracle
with a planted mistake and require that one of these checks fails)."""
import os

import mpmath
import numpy as np

EPS = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kappa_s(G):
    """Condition number of G with columns scaled to unit norm."""
    Gs = G / np.linalg.norm(G, axis=0)
    s = np.linalg.svd(Gs, compute_uv=False)
    return s[0] / s[-1]


def two_by_two_cases():
    rows = []
    with open(os.path.join(GOLDEN, "two_by_two.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = line.split()
            a11 = float(v[0])
            a = complex(float(v[1]), float(v[2]))
            J = np.array([int(v[3]), int(v[4])], dtype=np.int8)
            rows.append(((a11, a), J, np.array([float(v[5]), float(v[6])])))
    return rows


def two_by_two_G(entries):
    """Upper-triangular G with G^* G = [[a11, a], [conj(a), 1]]."""
    a11, a = entries
    cplx = a.imag != 0
    if cplx:
        A = np.array([[a11, a], [np.conj(a), 1.0]], dtype=np.complex128)
    else:
        A = np.array([[a11, a.real], [a.real, 1.0]], dtype=np.float64)
    L = np.linalg.cholesky(A)  # A = L L^*
    return L.conj().T


def spectrum_mp(G, J, dps=50):
    """Eigenvalues (descending) of H = G J G^* formed exactly from the stored G
    at `dps` digits, by mpmath."""
    n = G.shape[0]
    with mpmath.workdps(dps):
        if np.iscomplexobj(G):
            Gm = mpmath.matrix([[mpmath.mpc(complex(G[i, j]).real, complex(G[i, j]).imag) for j in range(n)]
                                for i in range(n)])
            H = Gm * mpmath.diag([int(x) for x in J]) * Gm.transpose_conj()
            ev = mpmath.eighe(H, eigvals_only=True)
        else:
            Gm = mpmath.matrix([[float(G[i, j]) for j in range(n)] for i in range(n)])
            H = Gm * mpmath.diag([int(x) for x in J]) * Gm.T
            ev = mpmath.eigsy(H, eigvals_only=True)
        vals = sorted([ev[i] for i in range(n)], reverse=True)
        return vals


def rel_err(lam, ref):
    lam = np.asarray(lam, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.max(np.abs(lam - ref) / np.abs(ref))


def residuals(G, J, lam, V):
    """(||H V - V diag(lam)||_F / ||lam||_2, max |V^* V - I|), H V formed as G (J (G^* V))."""
    Jd = np.asarray(J, dtype=np.float64)
    HV = G @ (Jd[:, None] * (G.conj().T @ V))
    res = np.linalg.norm(HV - V * np.asarray(lam, dtype=np.float64)[None, :]) / np.linalg.norm(
        np.asarray(lam, dtype=np.float64))
    orth = np.max(np.abs(V.conj().T @ V - np.eye(V.shape[1])))
    return res, orth


def battery(solve):
    """Run a quick set of pins against `solve(G, J) -> dict(lam, V, status)`.
    Returns a list of failure descriptions (empty when every pin holds)."""
    import jjgen
    fails = []
    for a, J, expect in two_by_two_cases():
        G = two_by_two_G(a)
        r = solve(G, J)
        if r["status"] != 0 or rel_err(r["lam"], expect) > 8 * EPS:
            fails.append("2x2 a=%s J=%s got %s" % (a, J.tolist(), np.asarray(r["lam"], float).tolist()))
        # the annihilating rotation diagonalises a 2x2 pencil in one step
        if r.get("rotations", 1) != 1:
            fails.append("2x2 a=%s J=%s needed %d rotations" % (a, J.tolist(), r["rotations"]))
    for cplx in (False, True):
        for seed in (11, 12):
            G, J, lam = jjgen.make(12, cplx, 5, 1e-2, 1e2, seed=seed)
            r = solve(G, J)
            ref = np.sort(lam)[::-1]
            k = kappa_s(G)
            if r["status"] != 0:
                fails.append("known spectrum cplx=%s status %d" % (cplx, r["status"]))
                continue
            if rel_err(r["lam"], ref) > 16 * EPS * k:
                fails.append("known spectrum cplx=%s err %.2e" % (cplx, rel_err(r["lam"], ref)))
            if int(np.sum(np.asarray(r["lam"], float) > 0)) != int(np.sum(J > 0)):
                fails.append("inertia cplx=%s" % cplx)
            res, orth = residuals(G, J, r["lam"], r["V"])
            if res > 1e3 * EPS * k or orth > 1e3 * EPS:
                fails.append("residual cplx=%s res %.2e orth %.2e" % (cplx, res, orth))
    return fails
