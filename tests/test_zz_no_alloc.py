"""jjacobi_solve_noalloc (fixed device scratch, no allocation) through the C
ABI against jjacobi_solve_ex: two calls in a row, the second with a smaller
input, each bitwise equal to the allocating entry point and at the oracle
parity bar; a problem too large for the scratch is refused before any work."""
import numpy as np
import pytest

import jjgen
from test_gpu_parity import check_parity, check_vectors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _run(entry, G, J, **kw):
    import paper_1008_4166_amd as jj
    n = G.shape[0]
    cplx = np.iscomplexobj(G)
    Gd = torch.from_numpy(np.ascontiguousarray(G.T)).cuda()  # column-major bytes of G
    lam = torch.empty(n, dtype=torch.float64, device="cuda")
    Vt = torch.empty((n, n), dtype=Gd.dtype, device="cuda")
    o = jj.make_opts(stream=torch.cuda.current_stream().cuda_stream, **kw)
    info = jj.jj_info()
    st = getattr(jj, entry)(jj.JJ_C128 if cplx else jj.JJ_F64, Gd.data_ptr(), J, n, n, lam.data_ptr(),
                            Vt.data_ptr(), n, 0.0, 0, o, info)
    torch.cuda.synchronize()
    return st, lam.cpu().numpy(), Vt.cpu().numpy().T, info.as_dict()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_allocating_entry_point(precision):
    cases = [jjgen.make(300, True, 120, 1e-6, 1.0, seed=5150),   # first call: larger, complex
             jjgen.make(150, False, 70, 1e-8, 1.0, seed=5151),   # second call: smaller, real
             jjgen.make(64, False, 32, 1e-3, 1e3, seed=5152)]    # third: n <= 64, the direct path in FP64
    for G, J, _ in cases:
        st0, l0, V0, i0 = _run("jjacobi_solve_ex", G, J, precision=precision)
        st1, l1, V1, i1 = _run("jjacobi_solve_noalloc", G, J, precision=precision)
        assert st0 == 0 and st1 == 0, (i0, i1)
        assert i1["sweeps"] == i0["sweeps"]
        assert np.array_equal(l1, l0) and np.array_equal(V1, V0)
        check_parity(G, J, l1, "noalloc n=%d" % G.shape[0])
        check_vectors(G, J, l1, V1)


def test_noalloc_refuses_what_does_not_fit():
    import paper_1008_4166_amd as jj
    n = 4096  # complex at block width 32: the Gram partials alone exceed the scratch
    J = np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int8)
    G = torch.zeros((n, n), dtype=torch.complex128, device="cuda")
    lam = torch.full((n,), 7.0, dtype=torch.float64, device="cuda")
    V = torch.zeros((n, n), dtype=torch.complex128, device="cuda")  # full-size outputs all the same
    info = jj.jj_info()
    st = jj.jjacobi_solve_noalloc(jj.JJ_C128, G.data_ptr(), J, n, n, lam.data_ptr(), V.data_ptr(), n, 0.0, 0,
                                  jj.make_opts(stream=torch.cuda.current_stream().cuda_stream), info)
    torch.cuda.synchronize()
    assert st == jj.JJ_SCRATCH_TOO_SMALL and info.status == st
    assert "scratch" in jj.jjacobi_status_string(st)
    assert torch.all(lam == 7.0)  # refused before any device work
