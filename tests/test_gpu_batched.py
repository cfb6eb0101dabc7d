"""Batched solves (jjacobi_solve_batched through the C ABI): every problem of a
mixed batch against the CPU oracle, status paths inside a batch, and
determinism of the graph-replayed step loop."""
import numpy as np
import pytest

import jjgen
import oracle
from _pins import EPS, kappa_s, rel_err
from test_gpu_parity import check_parity, check_vectors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def batched(Gs, Js, **kw):
    import paper_1008_4166_amd as jj
    ts = [torch.from_numpy(np.ascontiguousarray(G)).cuda() for G in Gs]
    lams, Vs, infos, worst = jj.solve_batched(ts, Js, **kw)
    torch.cuda.synchronize()
    return [l.cpu().numpy() for l in lams], [V.cpu().numpy() for V in Vs], infos, worst


def _mixed_batch(seed=0):
    sizes = [2, 5, 16, 33, 64, 65, 100, 130, 200, 97, 40, 150]
    Gs, Js = [], []
    for k, n in enumerate(sizes):
        cplx = k % 2 == 1
        G, J, _ = jjgen.make(n, cplx, (k * 7 + n // 3) % (n + 1), 1e-5, 1e2, seed=900 + seed * 100 + k)
        Gs.append(G)
        Js.append(J)
    return Gs, Js


@pytest.mark.parametrize("variant", [dict(), dict(block_width=16), dict(inner_mode=1)])
def test_mixed_batch_matches_oracle(variant):
    Gs, Js = _mixed_batch()
    lams, Vs, infos, worst = batched(Gs, Js, **variant)
    assert worst == 0, [i["status"] for i in infos]
    for G, J, lam, V, info in zip(Gs, Js, lams, Vs, infos):
        assert info["status"] == 0
        check_parity(G, J, lam, "batched n=%d" % G.shape[0])
        check_vectors(G, J, lam, V)


def test_batch_status_paths_and_tiny():
    Gs, Js = _mixed_batch(seed=1)
    Gbad = Gs[3].copy()
    Gbad[1, 2] = np.nan
    Gs.append(Gbad)
    Js.append(Js[3])
    Gs.append(np.array([[-2.0]]))
    Js.append(np.array([-1], dtype=np.int8))
    lams, Vs, infos, worst = batched(Gs, Js)
    assert infos[-2]["status"] == 3
    assert infos[-1]["status"] == 0 and lams[-1][0] == -4.0
    assert worst == 3
    for G, J, lam, info in zip(Gs[:-2], Js[:-2], lams[:-2], infos[:-2]):
        assert info["status"] == 0
        check_parity(G, J, lam)


def test_batch_sweep_cap():
    Gs, Js = _mixed_batch(seed=2)
    lams, Vs, infos, worst = batched(Gs, Js, max_sweeps=1)
    assert worst == 1
    assert any(i["status"] == 1 for i in infos)


def test_batch_deterministic_and_equal_to_replays():
    Gs, Js = _mixed_batch(seed=3)
    a, Va, _, _ = batched(Gs, Js)
    b, Vb, _, _ = batched(Gs, Js)
    for x, y, u, v in zip(a, b, Va, Vb):
        assert np.array_equal(x, y) and np.array_equal(u, v)


def test_batch_of_workload_sizes():
    # a small sample of the mixed-size workload (n in [16, 512], half complex)
    specs = jjgen.batch_recipe(count=16)
    Gs, Js = [], []
    for sp in specs:
        G, J, _ = jjgen.batch_member(sp)
        Gs.append(G)
        Js.append(J)
    lams, Vs, infos, worst = batched(Gs, Js)
    assert worst == 0
    for G, J, lam, info in zip(Gs, Js, lams, infos):
        if G.shape[0] <= 200:
            check_parity(G, J, lam)
        # inertia and trace invariants for all sizes
        assert np.sum(lam > 0) == np.sum(J > 0)
        tr = np.sum(J.astype(float) * np.sum(np.abs(G) ** 2, axis=0))
        assert abs(np.sum(lam) - tr) <= 64 * G.shape[0] * EPS * np.sum(np.abs(lam))


def test_mixed_precision_batch_matches_oracle():
    # FP32-MFMA Gram in each problem's pre-sweeps, FP64 rotations / W_P / update,
    # FP64 finishing sweeps: the FP64 parity bar for every problem
    Gs, Js = _mixed_batch(seed=3)
    lams, Vs, infos, worst = batched(Gs, Js, precision=1)
    assert worst == 0, [i["status"] for i in infos]
    assert max(i["mixed_sweeps"] for i in infos) >= 1
    for G, J, lam, V, info in zip(Gs, Js, lams, Vs, infos):
        check_parity(G, J, lam, "mixed batched n=%d" % G.shape[0])
        check_vectors(G, J, lam, V)


@pytest.fixture(scope="module")
def workload5():
    """The 4096-matrix batch (n ~ U{16..512}, half real, half complex) in its
    configured form (mixed precision on), solved by one jjacobi_solve_batched
    call; returns the members and the eigenvalues."""
    import paper_1008_4166_amd as jj
    specs = jjgen.batch_recipe(count=4096)
    flat, offs, Js, lams_pres = jjgen.make_batch(specs)
    count = len(specs)
    ns = [s["n"] for s in specs]
    dts = [1 if s["cplx"] else 0 for s in specs]
    loff = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    work = torch.from_numpy(flat).cuda()
    vbuf = torch.empty_like(work)
    lam = torch.empty(int(loff[-1]), dtype=torch.float64, device="cuda")
    Gp = [work.data_ptr() + 8 * int(o) for o in offs[:-1]]
    Vp = [vbuf.data_ptr() + 8 * int(o) for o in offs[:-1]]
    Lp = [lam.data_ptr() + 8 * int(o) for o in loff[:-1]]
    opts = jj.make_opts(stream=torch.cuda.current_stream().cuda_stream, precision=1)
    infos = (jj.jj_info * count)()
    worst = jj.jjacobi_solve_batched(count, dts, Gp, Js, ns, ns, Lp, Vp, ns, 0.0, 0, opts, infos)
    torch.cuda.synchronize()
    statuses = [infos[k].status for k in range(count)]
    lam_h = lam.cpu().numpy()
    del work, vbuf

    def member(k):
        g = flat[offs[k]:offs[k + 1]]
        if specs[k]["cplx"]:
            g = g.view(np.complex128)
        return g.reshape(ns[k], ns[k]).T

    return dict(specs=specs, ns=ns, Js=Js, lams_pres=lams_pres, worst=worst, statuses=statuses,
                lam=[lam_h[loff[k]:loff[k + 1]] for k in range(count)], member=member)


def test_full_size_batch_workload5(workload5):
    # every member converged, its inertia equal to J's sign counts, the trace
    # identity sum(lambda) = sum_j j_j ||g_j||^2, its prescribed spectrum within
    # 1e-9 (measured 5e-11; G is the rounded product of the generator)
    w = workload5
    assert w["worst"] == 0, [s for s in w["statuses"] if s]
    for k in range(len(w["ns"])):
        lk = w["lam"][k]
        G = w["member"](k)
        J = w["Js"][k]
        assert np.sum(lk > 0) == np.sum(J > 0), k
        tr = float(np.sum(J.astype(float) * np.sum(np.abs(G) ** 2, axis=0)))
        assert abs(float(np.sum(lk)) - tr) <= 1e-12 * float(np.sum(np.abs(lk))), k
        assert rel_err(lk, np.sort(w["lams_pres"][k])[::-1]) <= 1e-9, k


def _sample(w, pred, count):
    ks = [k for k in range(len(w["ns"])) if pred(k)]
    return [ks[i] for i in np.linspace(0, len(ks) - 1, count).astype(int)]


def test_batch_workload5_small_members_against_oracle(workload5):
    # six members with n <= 256 (one or a few blocked steps) at the parity bar
    w = workload5
    for k in _sample(w, lambda k: w["ns"][k] <= 256, 6):
        check_parity(w["member"](k), w["Js"][k], w["lam"][k], "batch member %d (n=%d)" % (k, w["ns"][k]))


@pytest.mark.parametrize("cplx", [False, True])
def test_batch_workload5_large_members_against_oracle(workload5, cplx):
    # two real and two complex members with n in (400, 512]: several blocks,
    # multi-step sweeps, slot compaction between rounds
    w = workload5
    ks = _sample(w, lambda k: w["ns"][k] > 400 and w["specs"][k]["cplx"] == cplx, 2)
    for k in ks:
        assert w["statuses"][k] == 0
        check_parity(w["member"](k), w["Js"][k], w["lam"][k], "batch member %d (n=%d)" % (k, w["ns"][k]))
