"""One solve of a workload, for profilers (rocprofv3 kernel traces and
hardware counters): generates the seeded input, runs one warm-up solve and
then one timed solve (or the front end: factor H = G J G^* of the Hermitian H
built from the same input), and prints what ran.

    python -m paper_1008_4166_amd.profile_run --workload 3 [--n N] [--block-width B]
                                              [--precision P] [--front-end] [--warmup W]
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--n", type=int, default=0, help="downsize the workload (0: its own size)")
    ap.add_argument("--block-width", type=int, default=0)
    ap.add_argument("--precision", type=int, default=0)
    ap.add_argument("--front-end", action="store_true", help="factor H = G J G^* instead of solving")
    ap.add_argument("--warmup", type=int, default=1)
    args = ap.parse_args()

    import numpy as np
    import torch

    import jjgen
    import paper_1008_4166_amd as jj

    G, J, _ = jjgen.config(args.workload, n=args.n or None)
    n = G.shape[0]
    cplx = np.iscomplexobj(G)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    if args.front_end:
        H = G @ (J.astype(float)[:, None] * G.conj().T)
        Hd = torch.from_numpy(np.ascontiguousarray(H.T)).to(dev)  # column-major bytes of H
        Gd = torch.empty_like(Hd)
        o = jj.make_opts(stream=stream)
        for _ in range(args.warmup):
            jj.jjacobi_factor(jj.JJ_C128 if cplx else jj.JJ_F64, Hd.data_ptr(), n, n, Gd.data_ptr(), n, 0.0, o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, Jf, r = jj.jjacobi_factor(jj.JJ_C128 if cplx else jj.JJ_F64, Hd.data_ptr(), n, n, Gd.data_ptr(), n, 0.0,
                                      o)
        torch.cuda.synchronize()
        print("front end: workload %d n=%d status %d rank %d %.2f ms" % (args.workload, n, st, r,
                                                                         1e3 * (time.perf_counter() - t0)))
        return
    pristine = torch.from_numpy(np.ascontiguousarray(G.T)).to(dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty_like(pristine)
    o = jj.make_opts(stream=stream, block_width=args.block_width, precision=args.precision)
    for k in range(args.warmup + 1):
        Gw = pristine.clone()
        info = jj.jj_info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = jj.jjacobi_solve_ex(jj.JJ_C128 if cplx else jj.JJ_F64, Gw.data_ptr(), J, n, n, lam.data_ptr(),
                                 Vt.data_ptr(), n, 0.0, 0, o, info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print("%s: workload %d n=%d status %d sweeps %d block width %d %.1f ms" % (
            "warm-up" if k < args.warmup else "solve", args.workload, n, st, info.sweeps, info.block_width,
            1e3 * dt), flush=True)


if __name__ == "__main__":
    main()
