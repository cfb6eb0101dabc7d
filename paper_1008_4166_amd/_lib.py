"""ctypes binding of libjjacobi.so (argument marshalling only).

The library is loaded from this package directory.  There is no fallback: if
the library is missing or cannot be loaded, every call raises."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libjjacobi.so")


class jj_opts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("block_width", ctypes.c_int), ("inner_max_sweeps", ctypes.c_int),
                ("diag_pass", ctypes.c_int), ("inner_mode", ctypes.c_int), ("precision", ctypes.c_int),
                ("mixed_switch", ctypes.c_double), ("strategy", ctypes.c_int), ("profile", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int),
                ("step_groups", ctypes.c_int),
                ("reserved", ctypes.c_int * 7)]


class jj_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("sweeps", ctypes.c_int), ("block_width", ctypes.c_int),
                ("nblocks", ctypes.c_int), ("pivots_rotated", ctypes.c_longlong), ("final_offdiag", ctypes.c_double),
                ("seconds", ctypes.c_double), ("mixed_sweeps", ctypes.c_int), ("mixed_resolved", ctypes.c_int),
                ("rank", ctypes.c_int), ("inner_mode", ctypes.c_int), ("reserved", ctypes.c_int * 4)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


KINDS = ("gram", "pivot", "update", "final", "other")


class jj_profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_longlong * 8), ("units", ctypes.c_longlong * 8),
                ("rotations", ctypes.c_longlong), ("inner_sweeps", ctypes.c_longlong),
                ("pivot_cols", ctypes.c_longlong), ("pivot_cols3", ctypes.c_longlong), ("n", ctypes.c_int),
                ("nblocks", ctypes.c_int), ("block_width", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("dtype", ctypes.c_int), ("valid", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("ms", "launches", "units")}
        for i, k in enumerate(KINDS):
            d[k] = dict(ms=self.ms[i], launches=self.launches[i], units=self.units[i])
        return d


# exported symbols declared in include/jjacobi.h
ABI_SYMBOLS = ("jjacobi_default_opts", "jjacobi_solve", "jjacobi_zsolve", "jjacobi_solve_ex",
               "jjacobi_solve_noalloc", "jjacobi_solve_rect", "jjacobi_factor", "jjacobi_eigh",
               "jjacobi_solve_batched", "jjacobi_last_profile", "jjacobi_status_string",
               "jjacobi_release_workspace")

_lib = None


def load(path=SO):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libjjacobi.so is not built (run __graft_entry__.build()); there is no fallback path")
    # One HIP runtime per process: PyTorch ships its own libamdhip64, and a
    # second runtime loaded beside it cannot see the GPU that the first one
    # opened.  Loading torch first lets the library's libamdhip64.so.7
    # dependency resolve to the runtime already in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.jjacobi_default_opts.argtypes = [ctypes.POINTER(jj_opts)]
    lib.jjacobi_default_opts.restype = None
    lib.jjacobi_solve.argtypes = [P, P, I, I, P, P, D, I]
    lib.jjacobi_solve.restype = I
    lib.jjacobi_zsolve.argtypes = [P, P, I, I, P, P, D, I]
    lib.jjacobi_zsolve.restype = I
    lib.jjacobi_solve_ex.argtypes = [I, P, P, I, I, P, P, I, D, I, ctypes.POINTER(jj_opts), ctypes.POINTER(jj_info)]
    lib.jjacobi_solve_ex.restype = I
    lib.jjacobi_solve_noalloc.argtypes = lib.jjacobi_solve_ex.argtypes
    lib.jjacobi_solve_noalloc.restype = I
    lib.jjacobi_solve_rect.argtypes = [I, P, P, I, I, I, P, P, I, D, I, ctypes.POINTER(jj_opts),
                                       ctypes.POINTER(jj_info)]
    lib.jjacobi_solve_rect.restype = I
    lib.jjacobi_factor.argtypes = [I, P, I, I, P, I, P, ctypes.POINTER(I), D, ctypes.POINTER(jj_opts)]
    lib.jjacobi_factor.restype = I
    lib.jjacobi_eigh.argtypes = [I, P, I, I, P, P, I, D, I, ctypes.POINTER(jj_opts), ctypes.POINTER(jj_info)]
    lib.jjacobi_eigh.restype = I
    lib.jjacobi_solve_batched.argtypes = [I, P, P, P, P, P, P, P, P, D, I, ctypes.POINTER(jj_opts),
                                          ctypes.POINTER(jj_info)]
    lib.jjacobi_solve_batched.restype = I
    lib.jjacobi_last_profile.argtypes = [ctypes.POINTER(jj_profile)]
    lib.jjacobi_last_profile.restype = I
    lib.jjacobi_status_string.argtypes = [I]
    lib.jjacobi_status_string.restype = ctypes.c_char_p
    lib.jjacobi_release_workspace.argtypes = []
    lib.jjacobi_release_workspace.restype = None
    # host planning helpers (no GPU work), used by the CPU tests
    lib.jjx_plan_nblocks.argtypes = [I, I]
    lib.jjx_plan_nblocks.restype = I
    lib.jjx_plan_offsets.argtypes = [I, I, P]
    lib.jjx_plan_offsets.restype = None
    lib.jjx_plan_round_robin.argtypes = [I, P]
    lib.jjx_plan_round_robin.restype = None
    lib.jjx_plan_modulus.argtypes = [I, P, P]
    lib.jjx_plan_modulus.restype = I
    lib.jjx_plan_sign_order.argtypes = [I, P, P]
    lib.jjx_plan_sign_order.restype = None
    lib.jjx_check_args.argtypes = [I, P, P, I, I, P, P, I]
    lib.jjx_check_args.restype = I
    _lib = lib
    return lib
