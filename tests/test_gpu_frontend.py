"""Front end and rectangular solve on the GPU (libjjacobi.so through its C
ABI) against the CPU oracle: the factorization H = G J G^* (Bunch-Parlett with
complete pivoting and the diagonalisation of D's 2x2 blocks; paper, Section
2.2, eq. 2.5), the eigenpairs of an explicit H through the front end and the
one-sided J-Jacobi solve, and the n x r factor of a singular H."""
import numpy as np
import pytest

import jjgen
import oracle
from _pins import EPS, rel_err
from test_gpu_parity import check_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _jj():
    import paper_1008_4166_amd as jj
    jj._lib.load()
    return jj


def _herm(n, cplx, seed, lo=0.1, hi=10.0):
    G, J, lam = jjgen.make(n, cplx, n // 2, lo, hi, seed=seed)
    H = G @ (J.astype(float)[:, None] * G.conj().T)
    return (H + H.conj().T) / 2, lam


def gpu_factor(H, tol=0.0):
    jj = _jj()
    G, J, st = jj.factor(torch.from_numpy(np.ascontiguousarray(H)).cuda(), tol=tol)
    torch.cuda.synchronize()
    return G.cpu().numpy(), J, st


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [1, 2, 7, 64, 130, 300])
def test_factor_against_oracle(cplx, n):
    H, _ = _herm(n, cplx, seed=1700 + n + 10000 * cplx)
    G, J, st = gpu_factor(H)
    r = oracle.bp_factor(H)
    assert st == 0 and r["status"] == 0
    assert G.shape[1] == r["rank"] == n
    # the same pivots (same signs) and the same factor: the kernels follow the
    # oracle's operations in the same order (no contraction)
    assert np.array_equal(J, r["J"])
    scale = np.max(np.abs(r["G"]))
    assert np.max(np.abs(G - r["G"])) <= 16 * n * EPS * scale, np.max(np.abs(G - r["G"])) / scale
    R = G @ (J.astype(float)[:, None] * G.conj().T)
    assert np.max(np.abs(R - H)) <= 8 * n * EPS * np.max(np.abs(H))


@pytest.mark.parametrize("cplx", [False, True])
def test_factor_real_bitwise(cplx):
    # real: every operation of the kernels is a correctly rounded IEEE operation
    # in the oracle's order, so the factor is bitwise the oracle's; complex
    # moduli go through hypot, whose last bit may differ
    H, _ = _herm(96, cplx, seed=4711)
    G, J, st = gpu_factor(H)
    r = oracle.bp_factor(H)
    if not cplx:
        assert np.array_equal(G, r["G"])
    else:
        assert np.max(np.abs(G - r["G"])) <= 64 * EPS * np.max(np.abs(r["G"]))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [5, 100, 257])
def test_eigh_against_oracle_pipeline(cplx, n):
    jj = _jj()
    H, lam = _herm(n, cplx, seed=2900 + n + 10000 * cplx, lo=1e-4, hi=10.0)
    lg, V, info = jj.eigh(torch.from_numpy(np.ascontiguousarray(H)).cuda())
    torch.cuda.synchronize()
    lg, V = lg.cpu().numpy(), V.cpu().numpy()
    assert info["status"] == 0 and info["rank"] == n, info
    r = oracle.bp_factor(H)
    check_parity(r["G"], r["J"], lg, "eigh n=%d cplx=%d" % (n, cplx))
    res = np.linalg.norm(H @ V - V * lg[None, :]) / np.linalg.norm(H)
    assert res <= 64 * n * EPS
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) <= 16 * n * EPS


@pytest.mark.parametrize("cplx", [False, True])
def test_singular_H(cplx):
    # H = B J0 B^* with integer B (n x r): rank r, the r nonzero eigenvalues
    jj = _jj()
    rng = np.random.default_rng(11 + cplx)
    n, rk = 40, 17
    B = rng.integers(-3, 4, size=(n, rk)).astype(float)
    if cplx:
        B = B + 1j * rng.integers(-3, 4, size=(n, rk))
    J0 = np.where(np.arange(rk) % 3 == 0, -1, 1)
    H = B @ (J0[:, None] * B.conj().T)
    G, J, st = gpu_factor(H)
    r = oracle.bp_factor(H)
    assert G.shape[1] == r["rank"] == rk and np.array_equal(J, r["J"])
    lg, V, info = jj.eigh(torch.from_numpy(np.ascontiguousarray(H)).cuda())
    torch.cuda.synchronize()
    lg, V = lg.cpu().numpy(), V.cpu().numpy()
    assert info["status"] == 0 and info["rank"] == rk
    ro = oracle.solve(r["G"], r["J"])
    assert rel_err(lg[:rk], ro["lam"]) <= 1e-12
    assert np.all(lg[rk:] == 0)
    # the null space (Householder QR of U~): a basis is not unique, its
    # projector is; against the oracle's completion of the oracle's U~
    Z = V[:, rk:]
    assert np.max(np.abs(Z.conj().T @ Z - np.eye(n - rk))) <= 16 * n * EPS
    assert np.max(np.abs(V[:, :rk].conj().T @ Z)) <= 16 * n * EPS
    assert np.linalg.norm(H @ Z) <= 64 * n * EPS * np.linalg.norm(H)
    Zo = oracle.nullspace(ro["V"])
    assert np.max(np.abs(Z @ Z.conj().T - Zo @ Zo.conj().T)) <= 1e-12
    ev = np.linalg.eigvalsh(H)
    nz = np.sort(ev[np.argsort(-np.abs(ev))[:rk]])[::-1]
    assert rel_err(lg[:rk], nz) <= 1e-10
    Vr = V[:, :rk]
    assert np.linalg.norm(H @ Vr - Vr * lg[None, :rk]) <= 64 * n * EPS * np.linalg.norm(H)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("m,n", [(40, 23), (300, 130), (513, 500)])
def test_rect_solve_against_oracle(cplx, m, n):
    # G = Q_r Gs (m x n, orthonormal Q_r columns): full column rank, rows > columns
    jj = _jj()
    Gs, J, _ = jjgen.make(n, cplx, n // 3, 1e-5, 1.0, seed=3100 + m)
    rng = np.random.default_rng(m + n)
    X = rng.standard_normal((m, n)) + (1j * rng.standard_normal((m, n)) if cplx else 0)
    Q, _ = np.linalg.qr(X)
    G = Q @ Gs
    lg, V, info = jj.solve_rect(torch.from_numpy(np.ascontiguousarray(G)).cuda(), J)
    torch.cuda.synchronize()
    lg, V = lg.cpu().numpy(), V.cpu().numpy()
    assert info["status"] == 0, info
    assert V.shape == (m, n)
    ro = oracle.solve(G, J, vectors=False)
    e = rel_err(lg, ro["lam"])
    if e > 1e-12:
        rl = oracle.solve(G, J, precision="long", vectors=False)["lam"].astype(float)
        assert rel_err(ro["lam"], rl) > 2.5e-13 and rel_err(lg, rl) <= 4 * rel_err(ro["lam"], rl)
    HV = G @ (J.astype(float)[:, None] * (G.conj().T @ V))
    assert np.linalg.norm(HV - V * lg[None, :]) / np.linalg.norm(lg) <= 1e-10
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) <= 16 * m * EPS


def test_eigh_zero_matrix():
    # H = 0: rank 0, every eigenvalue zero, V = I
    jj = _jj()
    lg, V, info = jj.eigh(torch.zeros((6, 6), dtype=torch.complex128, device="cuda"))
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["rank"] == 0
    assert np.all(lg.cpu().numpy() == 0) and np.array_equal(V.cpu().numpy(), np.eye(6))


def test_factor_status_paths():
    jj = _jj()
    Hb = np.eye(4)
    Hb[3, 1] = np.inf
    G, J, st = gpu_factor(Hb)
    assert st == 3
    G, J, st = gpu_factor(np.zeros((5, 5)))
    assert st == 0 and G.shape[1] == 0
    st, J, r = jj.jjacobi_factor(0, 0, 0, 1, 0, 1)
    assert st == 0 and r == 0
    assert jj.jjacobi_factor(0, 16, 4, 2, 16, 4)[0] == -4
