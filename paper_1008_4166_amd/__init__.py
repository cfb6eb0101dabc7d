"""MI355X (gfx950) one-sided hyperbolic J-Jacobi eigensolver.

Eigenpairs of H = G J G^* (J = diag(+-1)) by the blocked one-sided J-Jacobi
method of Singer et al. (arXiv:1008.4166).  Every step runs in the HIP kernels
of libjjacobi.so; this module only marshals arguments (PyTorch supplies device
memory and the stream).

Functions with the C names take raw device pointers; ``solve`` and
``solve_batched`` take torch tensors.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import jj_info, jj_opts

JJ_F64, JJ_C128 = 0, 1
JJ_SCRATCH_TOO_SMALL = 5
NOALLOC_SCRATCH_BYTES = 32 << 20


def _J_array(J, n):
    Jh = np.ascontiguousarray(np.asarray(J.cpu() if hasattr(J, "cpu") else J), dtype=np.int8).reshape(-1)
    if Jh.size != n:
        raise ValueError("J must have n entries")
    return Jh


# ---- raw C names (pointers are integers; J may be a host array) ----
def jjacobi_default_opts():
    o = jj_opts()
    _lib.load().jjacobi_default_opts(ctypes.byref(o))
    return o


def jjacobi_solve(G, J, n, ldg, lam, V, tol=0.0, max_sweeps=0):
    Jh = _J_array(J, n)
    return _lib.load().jjacobi_solve(G, Jh.ctypes.data, n, ldg, lam, V, tol, max_sweeps)


def jjacobi_zsolve(G, J, n, ldg, lam, V, tol=0.0, max_sweeps=0):
    Jh = _J_array(J, n)
    return _lib.load().jjacobi_zsolve(G, Jh.ctypes.data, n, ldg, lam, V, tol, max_sweeps)


def jjacobi_solve_ex(dtype, G, J, n, ldg, lam, V, ldv, tol=0.0, max_sweeps=0, opts=None, info=None):
    Jh = _J_array(J, n)
    return _lib.load().jjacobi_solve_ex(dtype, G, Jh.ctypes.data, n, ldg, lam, V, ldv, tol, max_sweeps,
                                        ctypes.byref(opts) if opts is not None else None,
                                        ctypes.byref(info) if info is not None else None)


def jjacobi_solve_noalloc(dtype, G, J, n, ldg, lam, V, ldv, tol=0.0, max_sweeps=0, opts=None, info=None):
    Jh = _J_array(J, n)
    return _lib.load().jjacobi_solve_noalloc(dtype, G, Jh.ctypes.data, n, ldg, lam, V, ldv, tol, max_sweeps,
                                             ctypes.byref(opts) if opts is not None else None,
                                             ctypes.byref(info) if info is not None else None)


def jjacobi_solve_rect(dtype, G, J, m, n, ldg, lam, V, ldv, tol=0.0, max_sweeps=0, opts=None, info=None):
    Jh = _J_array(J, n)
    return _lib.load().jjacobi_solve_rect(dtype, G, Jh.ctypes.data, m, n, ldg, lam, V, ldv, tol, max_sweeps,
                                          ctypes.byref(opts) if opts is not None else None,
                                          ctypes.byref(info) if info is not None else None)


def jjacobi_factor(dtype, H, n, ldh, G, ldg, tol=0.0, opts=None):
    """Returns (status, J (n int8; the first rank entries are the signs), rank)."""
    J = np.zeros(max(n, 1), dtype=np.int8)
    rank = ctypes.c_int(0)
    st = _lib.load().jjacobi_factor(dtype, H, n, ldh, G, ldg, J.ctypes.data, ctypes.byref(rank), tol,
                                    ctypes.byref(opts) if opts is not None else None)
    return st, J[:n], rank.value


def jjacobi_eigh(dtype, H, n, ldh, lam, V, ldv, tol=0.0, max_sweeps=0, opts=None, info=None):
    return _lib.load().jjacobi_eigh(dtype, H, n, ldh, lam, V, ldv, tol, max_sweeps,
                                    ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(info) if info is not None else None)


def jjacobi_solve_batched(count, dtypes, Gs, Js, ns, ldgs, lams, Vs, ldvs, tol=0.0, max_sweeps=0, opts=None,
                          infos=None):
    Jh = [_J_array(J, n) for J, n in zip(Js, ns)]
    arr = lambda t, v: (t * max(len(v), 1))(*v)
    return _lib.load().jjacobi_solve_batched(
        count, arr(ctypes.c_int, dtypes), arr(ctypes.c_void_p, Gs), arr(ctypes.c_void_p, [j.ctypes.data for j in Jh]),
        arr(ctypes.c_int, ns), arr(ctypes.c_int, ldgs), arr(ctypes.c_void_p, lams), arr(ctypes.c_void_p, Vs),
        arr(ctypes.c_int, ldvs), tol, max_sweeps, ctypes.byref(opts) if opts is not None else None, infos)


def jjacobi_last_profile():
    """Profile of the last solve of this thread made with profile=1, as a dict (or None)."""
    pr = _lib.jj_profile()
    if _lib.load().jjacobi_last_profile(ctypes.byref(pr)) != 0:
        return None
    return pr.as_dict()


def jjacobi_status_string(status):
    return _lib.load().jjacobi_status_string(status).decode()


def jjacobi_release_workspace():
    _lib.load().jjacobi_release_workspace()


# ---- torch convenience layer ----
def make_opts(stream=None, **kw):
    o = jjacobi_default_opts()
    if stream is not None:
        o.stream = stream
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def solve(G, J, tol=0.0, max_sweeps=0, overwrite=False, **opts):
    """Eigenpairs of H = G J G^* for a CUDA tensor G (n x n, float64 or
    complex128).  Returns (lam, V, info): lam (n,) float64 descending, V (n, n)
    with unit eigenvector columns, info a dict.  G is copied unless
    ``overwrite`` (then G must be a column-major view, e.g. ``X.t()`` of a
    contiguous X, and is destroyed)."""
    import torch
    if not G.is_cuda:
        raise ValueError("G must be a GPU tensor")
    n = G.shape[0]
    if G.shape != (n, n):
        raise ValueError("G must be square")
    cplx = G.dtype == torch.complex128
    if not cplx and G.dtype != torch.float64:
        raise ValueError("G must be float64 or complex128")
    Gt = G.t()
    if overwrite and Gt.is_contiguous():
        Gc = Gt  # storage of G is column-major already
    else:
        Gc = Gt.contiguous()  # rows of Gc are the columns of G
    lam = torch.empty(n, dtype=torch.float64, device=G.device)
    Vt = torch.empty((n, n), dtype=G.dtype, device=G.device)
    o = make_opts(stream=_current_stream(), **opts)
    info = jj_info()
    st = jjacobi_solve_ex(JJ_C128 if cplx else JJ_F64, Gc.data_ptr(), J, n, max(n, 1), lam.data_ptr(),
                          Vt.data_ptr(), max(n, 1), tol, max_sweeps, o, info)
    d = info.as_dict()
    d["status"] = st
    if st < 0 or st == 4:
        raise RuntimeError("jjacobi_solve_ex: %d (%s)" % (st, jjacobi_status_string(st)))
    return lam, Vt.t(), d


def solve_batched(Gs, Js, tol=0.0, max_sweeps=0, **opts):
    """Many problems in one call; Gs is a list of CUDA tensors (copied)."""
    import torch
    count = len(Gs)
    Gcs = [G.t().contiguous() for G in Gs]
    ns = [G.shape[0] for G in Gs]
    lams = [torch.empty(n, dtype=torch.float64, device=G.device) for n, G in zip(ns, Gs)]
    Vts = [torch.empty((n, n), dtype=G.dtype, device=G.device) for n, G in zip(ns, Gs)]
    dts = [JJ_C128 if G.dtype == torch.complex128 else JJ_F64 for G in Gs]
    infos = (jj_info * max(count, 1))()
    o = make_opts(stream=_current_stream(), **opts)
    st = jjacobi_solve_batched(count, dts, [g.data_ptr() for g in Gcs], Js, ns, [max(n, 1) for n in ns],
                               [l.data_ptr() for l in lams], [v.data_ptr() for v in Vts], [max(n, 1) for n in ns],
                               tol, max_sweeps, o, infos)
    if st < 0 or st == 4:
        raise RuntimeError("jjacobi_solve_batched: %d (%s)" % (st, jjacobi_status_string(st)))
    return lams, [v.t() for v in Vts], [infos[k].as_dict() for k in range(count)], st


def _colmajor(X):
    """Column-major device copy of a 2-D tensor (rows of the result are its columns)."""
    return X.t().contiguous()


def solve_rect(G, J, tol=0.0, max_sweeps=0, **opts):
    """Nonzero eigenpairs of H = G J G^* for a CUDA tensor G of m x n, m >= n,
    full column rank (float64 or complex128).  Returns (lam (n,), V (m, n), info)."""
    import torch
    m, n = G.shape
    cplx = G.dtype == torch.complex128
    if not cplx and G.dtype != torch.float64:
        raise ValueError("G must be float64 or complex128")
    Gc = _colmajor(G)
    lam = torch.empty(n, dtype=torch.float64, device=G.device)
    Vt = torch.empty((n, m), dtype=G.dtype, device=G.device)
    o = make_opts(stream=_current_stream(), **opts)
    info = jj_info()
    st = jjacobi_solve_rect(JJ_C128 if cplx else JJ_F64, Gc.data_ptr(), J, m, n, max(m, 1), lam.data_ptr(),
                            Vt.data_ptr(), max(m, 1), tol, max_sweeps, o, info)
    d = info.as_dict()
    d["status"] = st
    if st < 0 or st == 4:
        raise RuntimeError("jjacobi_solve_rect: %d (%s)" % (st, jjacobi_status_string(st)))
    return lam, Vt.t(), d


def factor(H, tol=0.0, **opts):
    """Front end: (G (n, r) CUDA tensor, J (r,) int8 numpy, status) with H = G J G^*."""
    import torch
    n = H.shape[0]
    cplx = H.dtype == torch.complex128
    Hc = _colmajor(H)
    Gt = torch.empty((n, n), dtype=H.dtype, device=H.device)
    o = make_opts(stream=_current_stream(), **opts)
    st, J, r = jjacobi_factor(JJ_C128 if cplx else JJ_F64, Hc.data_ptr(), n, max(n, 1), Gt.data_ptr(), max(n, 1),
                              tol, o)
    if st < 0 or st == 4:
        raise RuntimeError("jjacobi_factor: %d (%s)" % (st, jjacobi_status_string(st)))
    return Gt.t()[:, :r], J[:r].copy(), st


def eigh(H, tol=0.0, max_sweeps=0, **opts):
    """Eigenpairs of a Hermitian CUDA tensor H (n x n) through the front end and
    the one-sided J-Jacobi solve.  Returns (lam (n,), V (n, n), info); info['rank']
    is the rank found (the last n - rank eigenvalues are zero, their vectors an
    orthonormal basis of H's null space)."""
    import torch
    n = H.shape[0]
    cplx = H.dtype == torch.complex128
    Hc = _colmajor(H)
    lam = torch.empty(n, dtype=torch.float64, device=H.device)
    Vt = torch.empty((n, n), dtype=H.dtype, device=H.device)
    o = make_opts(stream=_current_stream(), **opts)
    info = jj_info()
    st = jjacobi_eigh(JJ_C128 if cplx else JJ_F64, Hc.data_ptr(), n, max(n, 1), lam.data_ptr(), Vt.data_ptr(),
                      max(n, 1), tol, max_sweeps, o, info)
    d = info.as_dict()
    d["status"] = st
    if st < 0 or st == 4:
        raise RuntimeError("jjacobi_eigh: %d (%s)" % (st, jjacobi_status_string(st)))
    return lam, Vt.t(), d
