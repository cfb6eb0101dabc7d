"""GPU path (libjjacobi.so through its C ABI) against the CPU oracle.

Eigenvalues are compared element by element (both sorted descending).  The bar
is a relative error of 1e-12 per eigenvalue wherever the double oracle itself
agrees with the long-double oracle to 2.5e-13; where the input's scaled
condition number makes two correct double computations differ by more, the GPU
must be within 4x of the double oracle's own distance to the long-double one,
or within eps kappa_s(G) of the long-double result (kappa_s: condition number
of G with unit columns; the relative perturbation bound of the paper's
Introduction, eps n kappa(A_s) with kappa(A_s) = kappa_s(G)^2 for A = G^* G,
is far looser).  Orderings of the same correct arithmetic spread by several
times on such inputs, so one oracle run is not a sharp bar alone."""
import os

import numpy as np
import pytest

import jjgen
import oracle
from _pins import EPS, kappa_s, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    import paper_1008_4166_amd as jj
    jj._lib.load()
    return jj


def gpu_solve(G, J, **kw):
    jj = _lib()
    Gt = torch.from_numpy(np.ascontiguousarray(G)).to("cuda")
    lam, V, info = jj.solve(Gt, J, **kw)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), V.cpu().numpy(), info


def check_parity(G, J, lam_gpu, tag=""):
    rd = oracle.solve(G, J, vectors=False)
    assert rd["status"] == 0
    e_gpu = rel_err(lam_gpu, rd["lam"])
    if e_gpu <= 1e-12:
        return e_gpu
    rl = oracle.solve(G, J, precision="long", vectors=False)
    ref = rl["lam"].astype(np.float64)
    e_ora = rel_err(rd["lam"], ref)
    e_gl = rel_err(lam_gpu, ref)
    assert e_ora > 2.5e-13, "%s: GPU vs oracle %.3e > 1e-12 with a well-conditioned oracle" % (tag, e_gpu)
    # the relative perturbation bound of the Introduction is eps n kappa(A_s)
    # for A = G^* G, kappa(A_s) = kappa_s(G)^2; eps kappa_s(G) lies well inside it
    ks = kappa_s(G)
    bound = max(4 * e_ora, EPS * ks)
    assert e_gl <= bound, "%s: GPU vs long double %.3e > max(4 x oracle's %.3e, eps kappa_s = %.3e)" % (
        tag, e_gl, e_ora, EPS * ks)
    return e_gpu


def check_vectors(G, J, lam, V, tol_scale=1.0):
    Jd = J.astype(float)
    HV = G @ (Jd[:, None] * (G.conj().T @ V))
    res = np.linalg.norm(HV - V * lam[None, :]) / np.linalg.norm(lam)
    orth = np.max(np.abs(V.conj().T @ V - np.eye(V.shape[1])))
    n = G.shape[0]
    assert res <= tol_scale * 64 * n * EPS * kappa_s(G), res
    assert orth <= tol_scale * 16 * n * EPS, orth


def test_config1_parity():
    G, J, lam = jjgen.config(1)
    lg, V, info = gpu_solve(G, J)
    assert info["status"] == 0
    e = check_parity(G, J, lg, "config1")
    assert e <= 1e-12
    check_vectors(G, J, lg, V)
    # prescribed spectrum, within the conditioning of the stored input
    assert rel_err(lg, np.sort(lam)[::-1]) <= 16 * EPS * kappa_s(G)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [2, 3, 4, 8, 16, 17, 32, 33, 63, 64, 65, 100, 127, 130, 200])
def test_ragged_sizes(cplx, n):
    G, J, lam = jjgen.make(n, cplx, (2 * n) // 5, 1e-4, 1e2, seed=300 + n + (1000 if cplx else 0))
    lg, V, info = gpu_solve(G, J)
    assert info["status"] == 0
    check_parity(G, J, lg, "n=%d cplx=%s" % (n, cplx))
    check_vectors(G, J, lg, V)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("bw", [4, 8, 16, 32])
def test_block_widths(cplx, bw):
    n = 150
    G, J, lam = jjgen.make(n, cplx, 70, 1e-5, 1.0, seed=77 + bw)
    lg, V, info = gpu_solve(G, J, block_width=bw)
    assert info["status"] == 0
    check_parity(G, J, lg, "bw=%d" % bw)
    check_vectors(G, J, lg, V)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("variant", [dict(inner_mode=1), dict(diag_pass=1), dict(diag_pass=2),
                                     dict(strategy=1), dict(inner_mode=1, strategy=1, diag_pass=2)])
def test_variants(cplx, variant):
    n = 260
    G, J, lam = jjgen.make(n, cplx, 100, 1e-6, 1.0, seed=91)
    lg, V, info = gpu_solve(G, J, **variant)
    assert info["status"] == 0, info
    check_parity(G, J, lg, str(variant))
    check_vectors(G, J, lg, V)


@pytest.mark.parametrize("cplx", [False, True])
def test_definite_and_diagonal(cplx):
    # J = I: the eigenvalues are the squared singular values of G (LAPACK's
    # SVD, accurate to a fraction of n eps here: sigma_max / sigma_min ~ 3.2).
    # Measured: 2.2 n eps real, 1.9 n eps complex (the plain oracle: 2.7 n eps)
    n = 96
    G, _, _ = jjgen.make(n, cplx, n, 1.0, 10.0, seed=5)
    J = np.ones(n, dtype=np.int8)
    lg, V, info = gpu_solve(G, J)
    assert info["status"] == 0, info
    s = np.linalg.svd(G, compute_uv=False)
    assert rel_err(lg, np.sort(s ** 2)[::-1]) <= 8 * n * EPS
    if cplx:
        return
    d = np.linspace(0.5, 3.0, 40)
    Jd = np.where(np.arange(40) % 3 == 0, 1, -1).astype(np.int8)
    lg, V, info = gpu_solve(np.diag(d), Jd)
    assert info["status"] == 0 and info["pivots_rotated"] == 0 and info["sweeps"] == 1
    assert np.array_equal(lg, np.sort(Jd * d ** 2)[::-1])


def test_tiny_and_empty():
    lg, V, info = gpu_solve(np.array([[-3.0]]), np.array([-1], dtype=np.int8))
    assert info["status"] == 0 and lg[0] == -9.0 and V[0, 0] == -1.0
    jj = _lib()
    assert jj.jjacobi_solve(0, np.zeros(0, np.int8), 0, 1, 0, 0, 0.0, 0) == 0


def test_status_paths():
    jj = _lib()
    G, J, _ = jjgen.config(1)
    lg, V, info = gpu_solve(G, J, max_sweeps=1)
    assert info["status"] == 1
    Gb = G.copy()
    Gb[3, 5] = np.inf
    Gt = torch.from_numpy(np.ascontiguousarray(Gb)).cuda()
    lam, V, info = jj.solve(Gt, J)
    assert info["status"] == 3
    Gd = G.copy()
    Gd[:, 1] = Gd[:, 0]
    Jd = J.copy()
    Jd[0], Jd[1] = 1, -1
    lg, V, info = gpu_solve(Gd, Jd)
    assert info["status"] == 2
    Jb = J.copy()
    Jb[7] = 0
    with pytest.raises(RuntimeError):
        jj.solve(torch.from_numpy(np.ascontiguousarray(G)).cuda(), Jb)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [40, 200])
def test_rank_deficient_G_is_a_breakdown(cplx, n):
    # Two equal columns of the same sign: G has rank n - 1 (the method needs
    # full column rank, Section 2).  Both columns fall in the first block after
    # sign ordering, so the first pivot holding them (n = 200: a blocked step;
    # n = 40: the full-rank test of the direct path) cannot factor its Gram
    # block.  They are the unit vector e_0, so that the Gram entries are 1 and
    # the second Cholesky pivot is exactly 1 - 1 = 0, whatever the rounding of
    # a square root.  The oracle reports status 2 for the same input (its first
    # rotation zeroes one of the two columns).
    G, J, _ = jjgen.make(n, cplx, n // 2, 1e-6, 1.0, seed=77)
    G = G.copy()
    G[:, 0] = 0.0
    G[0, 0] = 1.0
    G[:, 1] = G[:, 0]
    J = J.copy()
    J[0] = J[1] = 1
    assert oracle.solve(G, J, vectors=False)["status"] == 2
    lg, V, info = gpu_solve(G, J)
    assert info["status"] == 2, info


def test_deterministic():
    G, J, _ = jjgen.make(300, True, 120, 1e-6, 1.0, seed=1234)
    a, Va, _ = gpu_solve(G, J)
    b, Vb, _ = gpu_solve(G, J)
    assert np.array_equal(a, b) and np.array_equal(Va, Vb)


def test_config2_downsized_parity():
    G, J, lam = jjgen.config(2, n=256)
    lg, V, info = gpu_solve(G, J)
    assert info["status"] == 0
    check_parity(G, J, lg, "config2 n=256")
    check_vectors(G, J, lg, V)


def _golden(tag, prec):
    """Stored oracle eigenvalues (tests/golden/make_golden.py).  A missing file
    is a failure: these inputs are adjudicated only by the stored values."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "%s_lambda_%s.txt" % (tag, prec))
    assert os.path.exists(path), "stored oracle eigenvalues %s are missing" % path
    return np.loadtxt(path, dtype=np.longdouble if prec == "long" else np.float64)


def check_stored_parity(lg, tag):
    """The parity bar against stored double and long-double oracle eigenvalues:
    1e-12 per eigenvalue against the double oracle, or, where the double oracle
    itself is more than 2.5e-13 from the long-double one, at most 4x the double
    oracle's own distance to the long-double result."""
    ref = _golden(tag, "double")
    ldf = _golden(tag, "long").astype(np.float64)
    e = rel_err(lg, ref)
    if e > 1e-12:
        e_ora = rel_err(ref, ldf)
        assert e_ora > 2.5e-13, "%s: GPU vs oracle %.3e > 1e-12 with a well-conditioned oracle" % (tag, e)
        assert rel_err(lg, ldf) <= 4 * e_ora, "%s: GPU vs long double %.3e > 4 x oracle's %.3e" % (
            tag, rel_err(lg, ldf), e_ora)
    return e


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("k", [2, 3])
def test_full_size_against_stored_oracle(k, precision):
    # workloads 2 (n = 1024 complex) and 3 (n = 4096 real, graded [1e-12, 1]) in
    # plain FP64 and in the mixed form (FP32-MFMA Gram pre-sweeps, FP64 finish)
    G, J, lam = jjgen.config(k)
    lg, V, info = gpu_solve(G, J, precision=precision)
    assert info["status"] == 0, info
    if precision == 1:
        assert info["mixed_sweeps"] >= 1, info
    assert np.sum(lg > 0) == np.sum(J > 0)  # Sylvester inertia
    check_stored_parity(lg, "config%d" % k)


@pytest.mark.parametrize("precision", [0, 1])
def test_config4_law_downsized_against_stored_oracle(precision):
    # workload 4's law (complex, p = n/2, |lambda| log-uniform in [1e-8, 1e2])
    # at n = 1024, where the double and long-double oracles finish in minutes
    # (stored by make_golden.py): the blocked path with 32 blocks per sweep,
    # plain complex128 and mixed
    G, J, lam = jjgen.config(4, n=1024)
    lg, V, info = gpu_solve(G, J, precision=precision)
    assert info["status"] == 0, info
    if precision == 1:
        assert info["mixed_sweeps"] >= 1, info
    assert np.sum(lg > 0) == np.sum(J > 0)
    check_stored_parity(lg, "config4_n1024")
    check_vectors(G, J, lg, V)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n,lo,hi", [(64, 1e-3, 1e3), (200, 1e-6, 1.0), (300, 1e-12, 1.0)])
def test_mixed_precision_reaches_fp64_accuracy(cplx, n, lo, hi):
    # FP32-MFMA Gram in the pre-sweeps, FP64 rotations / W_P / update throughout,
    # FP64 finishing sweeps: the same parity bar as the plain FP64 path
    G, J, lam = jjgen.make(n, cplx, (3 * n) // 7, lo, hi, seed=600 + n)
    lg, V, info = gpu_solve(G, J, precision=1)
    assert info["status"] == 0
    assert info["mixed_sweeps"] >= 1
    check_parity(G, J, lg, "mixed n=%d cplx=%s" % (n, cplx))
    check_vectors(G, J, lg, V)


@pytest.mark.parametrize("cplx", [False, True])
def test_graph_replay_equals_eager(cplx):
    # sweeps replayed from a captured HIP graph and sweeps launched eagerly (the
    # profiled path) run the same kernels in the same order: identical results,
    # also when called on a side stream, and again on a second call
    G, J, _ = jjgen.make(330, cplx, 150, 1e-6, 1.0, seed=4242)
    lg, Vg, ig = gpu_solve(G, J)
    le, Ve, ie = gpu_solve(G, J, profile=1)
    assert ig["status"] == 0 and ie["status"] == 0 and ig["sweeps"] == ie["sweeps"]
    assert np.array_equal(lg, le) and np.array_equal(Vg, Ve)
    jj = _lib()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        Gt = torch.from_numpy(np.ascontiguousarray(G)).to("cuda")
        lam, V, info = jj.solve(Gt, J)
        lam2 = lam.clone()
    side.synchronize()
    assert np.array_equal(lam2.cpu().numpy(), lg)
    lg2, Vg2, _ = gpu_solve(G, J)
    assert np.array_equal(lg2, lg) and np.array_equal(Vg2, Vg)


@pytest.mark.parametrize("groups", [2, 4])
def test_dataflow_sweep_graph_equals_eager(groups):
    # sweeps whose graph keeps only the block-ownership dependencies between
    # groups of pairs: the same data reaches every kernel, so the results are
    # bitwise those of the eager (profiled) sweep
    G, J, _ = jjgen.make(600, False, 250, 1e-8, 1.0, seed=777)
    lg, Vg, ig = gpu_solve(G, J, block_width=16, step_groups=groups)
    le, Ve, ie = gpu_solve(G, J, block_width=16, profile=1)
    assert ig["status"] == 0 and ig["sweeps"] == ie["sweeps"]
    assert np.array_equal(lg, le) and np.array_equal(Vg, Ve)
    check_parity(G, J, lg, "dataflow groups=%d" % groups)


@pytest.mark.parametrize("cplx", [False, True])
def test_mixed_resolves_pivots_fp32_cannot_factor(cplx):
    # one column scaled to entries below 1e-23: its squares underflow in FP32,
    # so every FP32 Gram block holding it has a zero diagonal entry and cannot
    # be factored, while FP64 represents it with full relative accuracy (its
    # eigenvalue is near 1e-46).  Mixed sweeps re-solve those pivots from FP64
    # Gram blocks within the step and stay in FP32; the result meets the FP64
    # parity bar.
    n = 96
    G, J, _ = jjgen.make(n, cplx, 40, 1e-3, 1.0, seed=8080 + cplx)
    c = int(np.flatnonzero(J > 0)[3])
    G[:, c] *= 1e-24 / np.max(np.abs(G[:, c]))
    lg, V, info = gpu_solve(G, J, precision=1)
    assert info["status"] == 0, info
    assert info["mixed_resolved"] >= 1 and info["mixed_sweeps"] >= 2, info
    check_parity(G, J, lg, "mixed re-solve cplx=%s" % cplx)
    check_vectors(G, J, lg, V)


def test_full_size_config4_properties():
    # n = 8192 complex (no oracle run at this size: days of CPU).  Checked
    # against what holds at any size: inertia equal to J's sign counts; the
    # prescribed spectrum within 1e-9 relative (G is the rounded product
    # Q diag(sqrt|lambda|) W, whose eigenvalues move from the prescribed ones by
    # about eps times the column-scaled condition; the measured distance is
    # 5e-11); trace(H) = sum_j j_j ||g_j||^2; residuals and orthonormality of
    # sampled eigenvectors, computed on the CPU one by one from G and J.
    G, J, lam = jjgen.config(4)
    n = G.shape[0]
    jj = _lib()
    Gt = torch.from_numpy(np.ascontiguousarray(G)).to("cuda")
    lg, Vt, info = jj.solve(Gt, J)
    torch.cuda.synchronize()
    lg = lg.cpu().numpy()
    assert info["status"] == 0, info
    assert np.sum(lg > 0) == np.sum(J > 0)
    ref = np.sort(lam)[::-1]
    assert rel_err(lg, ref) <= 1e-9
    tr = np.sum(J.astype(float) * np.sum(np.abs(G) ** 2, axis=0))
    assert abs(np.sum(lg) - tr) <= 1e-12 * np.sum(np.abs(lg))
    idx = np.linspace(0, n - 1, 8).astype(int)
    V = Vt[:, idx].cpu().numpy()
    HV = G @ (J.astype(float)[:, None] * (G.conj().T @ V))
    # residual relative to ||G||_F^2 >= ||G||_2^2, the scale of the rounding of G J G^* v
    res = np.linalg.norm(HV - V * lg[idx][None, :], axis=0) / np.sum(np.abs(G) ** 2)
    assert np.max(res) <= 64 * n * EPS, res
    assert np.max(np.abs(V.conj().T @ V - np.eye(len(idx)))) <= 16 * n * EPS


@pytest.mark.parametrize("cplx", [False, True])
def test_leading_dimensions_and_padding(cplx):
    # G with ldg > n whose padding rows hold NaN, V with ldv > n: the padding is
    # never read or written, and the results are bitwise those of the packed solve
    jj = _lib()
    n, ldg, ldv = 150, 157, 153
    G, J, _ = jjgen.make(n, cplx, 60, 1e-6, 1.0, seed=2718 + cplx)
    dt = torch.complex128 if cplx else torch.float64
    Gp = torch.full((n, ldg), float("nan"), dtype=dt, device="cuda")  # row c = column c of G, padded
    Gp[:, :n] = torch.from_numpy(np.ascontiguousarray(G.T)).cuda()
    Vp = torch.full((n, ldv), 7.0, dtype=dt, device="cuda")
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    o = jj.make_opts(stream=torch.cuda.current_stream().cuda_stream)
    info = jj.jj_info()
    st = jj.jjacobi_solve_ex(1 if cplx else 0, Gp.data_ptr(), J, n, ldg, lam.data_ptr(), Vp.data_ptr(), ldv,
                             0.0, 0, o, info)
    torch.cuda.synchronize()
    assert st == 0
    assert torch.all(Vp[:, n:] == 7.0)
    lref, Vref, _ = gpu_solve(G, J)
    assert np.array_equal(lam.cpu().numpy(), lref)
    assert np.array_equal(Vp[:, :n].cpu().numpy().T, Vref)


@pytest.mark.parametrize("case", range(12))
def test_random_shapes_padded(case):
    # seeded random n (odd and even, several row chunks and a ragged last block),
    # real or complex, block width 16 or 32, and a leading dimension ldg > n whose
    # padding rows hold NaN: element-wise parity with the oracle, status 0
    jj = _lib()
    rng = np.random.default_rng(4242 + case)
    n = int(rng.integers(65, 321))
    cplx = bool(case % 2)
    bw = 16 if case % 4 >= 2 else 32
    ldg = n + int(rng.integers(1, 4))
    G, J, _ = jjgen.make(n, cplx, int(rng.integers(0, n + 1)), float(10.0 ** rng.uniform(-8, -2)), 1.0,
                         seed=6100 + case)
    dt = torch.complex128 if cplx else torch.float64
    Gp = torch.full((n, ldg), float("nan"), dtype=dt, device="cuda")  # row c = column c of G, padded
    Gp[:, :n] = torch.from_numpy(np.ascontiguousarray(G.T)).cuda()
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    V = torch.empty((n, n), dtype=dt, device="cuda")
    o = jj.make_opts(stream=torch.cuda.current_stream().cuda_stream, block_width=bw)
    info = jj.jj_info()
    st = jj.jjacobi_solve_ex(1 if cplx else 0, Gp.data_ptr(), J, n, ldg, lam.data_ptr(), V.data_ptr(), n,
                             0.0, 0, o, info)
    torch.cuda.synchronize()
    assert st == 0, (n, cplx, bw, ldg)
    check_parity(G, J, lam.cpu().numpy(), "random n=%d cplx=%d bw=%d ldg=%d" % (n, cplx, bw, ldg))


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("n", [130, 300, 512])
def test_three_level_pivots(cplx, n):
    # block width 64: pivots of up to 128 columns shortened to their Cholesky
    # factor R and orthogonalised by the blocked block-oriented method on R
    # (Section 5, Algorithm 5.1); ragged blocks (130: 33 + 33 / 32 + 32 columns,
    # 300: six blocks of 50) and equal ones (512: eight of 64)
    G, J, lam = jjgen.make(n, cplx, n // 3, 1e-6, 1.0, seed=5200 + n + 10000 * cplx)
    lg, V, info = gpu_solve(G, J, block_width=64)
    assert info["status"] == 0, info
    assert info["block_width"] > 32
    check_parity(G, J, lg, "three-level n=%d cplx=%s" % (n, cplx))
    check_vectors(G, J, lg, V)


def test_three_level_config4_law_against_stored_oracle():
    # workload 4's law at n = 1024 (complex) with block width 64
    G, J, lam = jjgen.config(4, n=1024)
    lg, V, info = gpu_solve(G, J, block_width=64)
    assert info["status"] == 0 and info["block_width"] == 64, info
    assert np.sum(lg > 0) == np.sum(J > 0)
    check_stored_parity(lg, "config4_n1024")
