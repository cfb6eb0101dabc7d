"""Seeded synthetic inputs with a known spectrum (see jjgen.c for the recipe).

Shared by the tests (which hand the same input to the CPU oracle and to the GPU
library), the smoke check and the benchmark.  Holds none of the eigensolver's
arithmetic.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libjjgen.so")
BASE_SEED = 10084166


def build(out=_SO):
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
                           "-fPIC", "-o", out, os.path.join(_HERE, "jjgen.c"), "-lm"])
    return out


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.jjgen_make.restype = ctypes.c_int
        lib.jjgen_make.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_ulonglong, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.jjgen_uniform.restype = None
        lib.jjgen_uniform.argtypes = [ctypes.c_ulonglong, ctypes.c_ulonglong, ctypes.c_longlong, ctypes.c_void_p]
        _lib = lib
    return _lib


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def make(n, cplx=False, p=None, lo=1e-3, hi=1e3, nrot=None, seed=BASE_SEED, haar=True, threads=None):
    """Return (G, J, lam): G (n, n) Fortran-ordered float64/complex128, J int8
    signs, lam the prescribed eigenvalues of H = G J G^* (lam[i] pairs with
    column i of Q; unsorted)."""
    lib = _load()
    p = n // 2 if p is None else p
    nrot = n if nrot is None else nrot
    J = np.zeros(max(n, 1), dtype=np.int8)
    lam = np.zeros(max(n, 1), dtype=np.float64)
    G = np.zeros((n, n), dtype=np.complex128 if cplx else np.float64, order="F")
    rc = lib.jjgen_make(n, 1 if cplx else 0, p, lo, hi, nrot, seed, 1 if haar else 0,
                        J.ctypes.data, lam.ctypes.data, G.ctypes.data if n else None,
                        threads or _threads())
    if rc != 0:
        raise ValueError("jjgen_make: invalid arguments")
    return G, J[:n], lam[:n]


def uniform(seed, stream, count):
    out = np.zeros(max(count, 1), dtype=np.float64)
    _load().jjgen_uniform(seed, stream, count, out.ctypes.data)
    return out[:count]


# The five workloads.  Readings where the wording is open: k = n random
# J-rotations; J-sign positions shuffled; Haar Q.
CONFIGS = {
    1: dict(n=64, cplx=False, p=32, lo=1e-3, hi=1e3),
    2: dict(n=1024, cplx=True, p=512, lo=1e-6, hi=1.0),
    3: dict(n=4096, cplx=False, p=3000, lo=1e-12, hi=1.0),
    4: dict(n=8192, cplx=True, p=4096, lo=1e-8, hi=1e2),
}


def config(k, n=None):
    """Input of workload k (1..4).  ``n`` downsizes it (same spectrum law and
    inertia fraction) for cases the oracle must finish in seconds."""
    c = dict(CONFIGS[k])
    if n is not None and n != c["n"]:
        c["p"] = int(round(c["p"] * n / c["n"]))
        c["n"] = n
    return make(c["n"], c["cplx"], c["p"], c["lo"], c["hi"], nrot=c["n"], seed=BASE_SEED + k - 1)


def batch_recipe(count=4096, nmin=16, nmax=512, seed=BASE_SEED + 4):
    """Sizes, kinds and inertia of the batched workload: n ~ U{nmin..nmax},
    first half real, second half complex, p ~ U{0..n}, |lambda| in [1e-6, 1e3]."""
    u = uniform(seed, 1, count)
    v = uniform(seed, 2, count)
    ns = np.minimum(nmin + np.floor(u * (nmax - nmin + 1)).astype(np.int64), nmax)
    ps = np.minimum(np.floor(v * (ns + 1)).astype(np.int64), ns)
    cplx = np.arange(count) >= count // 2
    return [dict(n=int(ns[i]), cplx=bool(cplx[i]), p=int(ps[i]), lo=1e-6, hi=1e3, seed=seed * 7919 + i)
            for i in range(count)]


def batch_member(spec):
    return make(spec["n"], spec["cplx"], spec["p"], spec["lo"], spec["hi"], nrot=spec["n"], seed=spec["seed"])
