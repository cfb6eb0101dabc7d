"""Host-side logic of the library (no GPU): block partition (eq. 3.2-3.3),
pair schedules (Sections 4.1-4.2), sign ordering, argument validation, and
the exported C ABI."""
import ctypes
import itertools
import os
import re

import numpy as np
import pytest

import paper_1008_4166_amd as jj

lib = jj._lib.load()
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "jjacobi.h")).read()
    names = set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(jjacobi_\w+)\s*\(", hdr, flags=re.M))
    assert names == set(jj._lib.ABI_SYMBOLS)
    for name in names:
        assert hasattr(lib, name)


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors of jj_opts, jj_info and jj_profile against the C
    # compiler's layout of the header (field offsets and sizes)
    import subprocess
    structs = {"jj_opts": jj._lib.jj_opts, "jj_info": jj._lib.jj_info, "jj_profile": jj._lib.jj_profile}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "jjacobi.h"', "int main(void) {"]
    for sname, cls in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (sname, sname))
        for fname, _ in cls._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (sname, fname, sname, fname))
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for sname, cls in structs.items():
        assert int(out["%s size" % sname]) == ctypes.sizeof(cls), sname
        for fname, _ in cls._fields_:
            assert int(out["%s.%s" % (sname, fname)]) == getattr(cls, fname).offset, (sname, fname)


@pytest.mark.parametrize("n,nt", [(1, 32), (2, 32), (3, 32), (64, 32), (65, 32), (100, 16), (4096, 32),
                                  (4097, 32), (1024, 32), (8192, 32), (5, 2), (33, 4), (7, 7)])
def test_partition(n, nt):
    nbl = lib.jjx_plan_nblocks(n, nt)
    if n < 2:
        assert nbl == 1
        return
    assert nbl >= 2 and nbl % 2 == 0 and nbl <= n
    off = np.zeros(nbl + 1, dtype=np.int32)
    lib.jjx_plan_offsets(n, nbl, off.ctypes.data)
    sizes = np.diff(off)
    assert off[0] == 0 and off[-1] == n
    assert sizes.max() - sizes.min() <= 1 and np.all(np.diff(sizes) <= 0)  # eq. 3.3
    assert sizes.max() <= max(nt, 1) or nbl == 2 and sizes.max() <= (n + 1) // 2
    assert sizes.min() >= 1


@pytest.mark.parametrize("nbl", [2, 4, 6, 8, 32, 128, 256])
def test_round_robin(nbl):
    h = nbl // 2
    pairs = np.zeros((nbl - 1, h, 2), dtype=np.int32)
    lib.jjx_plan_round_robin(nbl, pairs.ctypes.data)
    seen = set()
    for t in range(nbl - 1):
        blocks = pairs[t].reshape(-1)
        assert sorted(blocks.tolist()) == list(range(nbl))  # disjoint and complete
        for i, j in pairs[t]:
            assert i < j
            seen.add((i, j))
    assert seen == set(itertools.combinations(range(nbl), 2))  # every pair once per sweep


@pytest.mark.parametrize("nbl", [2, 4, 6, 10, 64])
def test_modulus(nbl):
    h = nbl // 2
    pairs = np.zeros((nbl, h, 2), dtype=np.int32)
    counts = np.zeros(nbl, dtype=np.int32)
    assert lib.jjx_plan_modulus(nbl, pairs.ctypes.data, counts.ctypes.data) == nbl
    seen = []
    for t in range(nbl):
        ps = pairs[t, :counts[t]]
        blocks = ps.reshape(-1)
        assert len(set(blocks.tolist())) == blocks.size  # disjoint
        assert counts[t] in (h, h - 1)
        seen += [tuple(p) for p in ps]
    assert sorted(seen) == sorted(itertools.combinations(range(nbl), 2))


def test_sign_order_stable():
    J = np.array([-1, 1, 1, -1, 1, -1, -1, 1], dtype=np.int8)
    cm = np.zeros(8, dtype=np.int32)
    lib.jjx_plan_sign_order(8, J.ctypes.data, cm.ctypes.data)
    assert cm.tolist() == [1, 2, 4, 7, 0, 3, 5, 6]


def test_argument_validation_without_gpu():
    J = np.ones(4, dtype=np.int8)
    ok = ctypes.c_void_p(16)  # never dereferenced: validation returns first
    f = lib.jjx_check_args
    assert f(0, ok, J.ctypes.data, 4, 4, ok, ok, 4) == 0
    assert f(2, ok, J.ctypes.data, 4, 4, ok, ok, 4) == -1
    assert f(0, None, J.ctypes.data, 4, 4, ok, ok, 4) == -2
    assert f(0, ok, None, 4, 4, ok, ok, 4) == -3
    assert f(0, ok, J.ctypes.data, -1, 4, ok, ok, 4) == -4
    assert f(0, ok, J.ctypes.data, 4, 3, ok, ok, 4) == -5
    assert f(0, ok, J.ctypes.data, 4, 4, None, ok, 4) == -6
    assert f(0, ok, J.ctypes.data, 4, 4, ok, None, 4) == -7
    assert f(0, ok, J.ctypes.data, 4, 4, ok, ok, 2) == -8
    Jb = np.array([1, 0, 1, -1], dtype=np.int8)
    assert f(0, ok, Jb.ctypes.data, 4, 4, ok, ok, 4) == -3
    assert f(0, None, None, 0, 0, None, None, 0) == 0  # n = 0: nothing to do
    # the public entry points reject the same arguments before any HIP call
    assert jj.jjacobi_solve_ex(0, 0, J, 4, 4, 16, 16, 4) == -2
    assert jj.jjacobi_solve_ex(7, 16, J, 4, 4, 16, 16, 4) == -1
    assert jj.jjacobi_solve(16, Jb, 4, 4, 16, 16) == -3
    assert jj.jjacobi_solve_batched(-1, [], [], [], [], [], [], [], []) == -1
    assert jj.jjacobi_status_string(2).startswith("numerical breakdown")
