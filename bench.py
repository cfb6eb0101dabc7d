"""Benchmark: one step = one complete solve (all steps of the hot path: sign
reordering and partition, block sweeps of Gram / pivot solve / update, and
the eigenpair finalisation) of the n = 4096 real FP64 workload (J with 3000
positive entries, |lambda| log-uniform in [1e-12, 1], G = Q diag(sqrt|lambda|) W).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-mixed]
                    [--no-batched] [--no-c4] [--copy-probe-mb MB]

Prints one JSON line.  value = eigenpairs/s = n * K / (time of K solves), with
every solve's input G already resident in HBM (one pristine device copy per
solve, made before the timed region, because a solve overwrites G).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6  # MFMA and vector
WORKLOAD = 3


def note(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_work(prof, n, cplx):
    """Algorithmic flops and HBM bytes per launch of each kernel kind.

    Gram, per pair of m columns: the Hermitian m x m block costs n*m*(m+1)
    real flops (half of the 2*n*m^2 of a full product) and reads n*m*s bytes.
    Update, per pair whose W_P is not the identity: 2*n*m^2 flops, n*m*s read
    plus n*m*s written.  (complex: flops x4, s = 16.)  Pivot solve: each inner
    sweep forms three length-m dot products for all m(m-1)/2 pairs (6m flops
    each, real) and each rotation updates two columns of R and of W_P (12m
    flops); plus the Cholesky factorisation, m^3/3 flops."""
    s = 16 if cplx else 8
    cf = 4 if cplx else 1
    m = 2 * prof["block_width"] if prof["nblocks"] >= 2 else n
    out = {}
    g = prof["gram"]
    if g["launches"]:
        units = g["units"] / g["launches"]
        out["gram"] = dict(flops=cf * units * n * m * (m + 1), bytes=units * n * m * s, ms=g["ms"] / g["launches"])
    u = prof["update"]
    if u["launches"]:
        units = u["units"] / u["launches"]
        out["update"] = dict(flops=cf * units * 2 * n * m * m, bytes=units * 2 * n * m * s,
                             ms=u["ms"] / u["launches"])
    p = prof["pivot"]
    if p["launches"]:
        mm = prof["pivot_cols"] / max(1, p["units"])  # mean solved pivot size
        dots = prof["inner_sweeps"] * mm * (mm - 1) / 2 * 6 * mm
        rots = prof["rotations"] * 12 * mm
        chol = prof["pivot_cols3"] / 3.0
        out["pivot"] = dict(flops=cf * (dots + rots + chol) / p["launches"], bytes=0.0, ms=p["ms"] / p["launches"])
    f = prof["final"]
    if f["launches"]:
        out["final"] = dict(flops=3.0 * n * n * cf, bytes=2.0 * n * n * s, ms=f["ms"] / f["launches"])
    return out


def _code_tokens(text):
    """Source text without C/C++ comments, whitespace runs collapsed: what the
    compiler sees, so that a comment-only edit keeps the recorded counters."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def sources_sha256():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1008_4166_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8", errors="replace") as fh:
            h.update(_code_tokens(fh.read()).encode())
    return h.hexdigest()


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_n4096_f64_solve.md")
    if not os.path.exists(path):
        return None
    vals, sha, ff, wf = {}, None, None, None
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) == 2 and t[0] == "sources_sha256":
                sha = t[1]
            elif len(t) == 2 and t[0] == "fetch_factor":
                ff = float(t[1])
            elif len(t) == 2 and t[0] == "write_factor":
                wf = float(t[1])
            elif len(t) == 6 and t[0] == "kernel":
                vals[t[1]] = (float(t[3]), float(t[5]))
    if sha != sources_sha256() or kernel not in vals or ff is None or wf is None:
        return None
    fk, wk = vals[kernel]
    return (fk * ff + wk * wf) * 1024.0


def roofline(prof, n, cplx):
    work = algorithmic_work(prof, n, cplx)
    kinds = {k: prof[k]["ms"] for k in ("gram", "pivot", "update", "final")}
    dom = max(kinds, key=kinds.get)
    w = work[dom]
    if dom == "pivot":
        # plain FP64 ALU work (no MFMA): 256 CUs x 64 FP64 FMA lanes x 2 flops x 2.4 GHz
        ach = w["flops"] / (w["ms"] * 1e-3) / 1e12
        r = dict(bound="alu", achieved=ach, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s")
    else:
        ai = w["flops"] / max(w["bytes"], 1.0)
        if ai < PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9):
            ach = w["bytes"] / (w["ms"] * 1e-3) / 1e9
            r = dict(bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s")
        else:
            ach = w["flops"] / (w["ms"] * 1e-3) / 1e12
            r = dict(bound="mfma", achieved=ach, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s")
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = pmc_traffic(dom)
    r["kernel"] = dom
    r["avg_launch_ms"] = w["ms"]
    return r, work


def host_cpu():
    """CPU model and thread counts of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model, logical_cpus=os.cpu_count(), usable_cpus=len(os.sched_getaffinity(0)))


def cpu_baseline(n_full, sweeps_full, batch_every=16, batch_procs=16):
    """The oracle as it stands on the host cores, on bounded samples.

    Single solves: one full oracle solve (every sweep, single-threaded) of the
    n = 1024 instance of the same workload law, measured; `value` scales it to
    n = 4096 by n^3 and by the ratio of the oracle's sweep counts (41 on the
    n = 4096 input, stored with its eigenvalues), labelled extrapolated.
    Batched: the oracle over a process pool (the members are independent) on
    every `batch_every`-th member of the 4096-matrix batch, scaled to mats/s."""
    import jjgen
    import oracle
    ns = 1024
    G, J, _ = jjgen.config(WORKLOAD, n=ns)
    t = time.perf_counter()
    r = oracle.solve(G, J, vectors=False)
    dt = time.perf_counter() - t
    t_full = dt * (n_full / ns) ** 3 * sweeps_full / max(1, r["sweeps"])
    G1, J1, _ = jjgen.config(1)
    t1 = time.perf_counter()
    oracle.solve(G1, J1, vectors=False)
    dt1 = time.perf_counter() - t1
    out = dict(value=n_full / t_full, unit="eigenpairs/s", cores=1, kind="oracle", host=host_cpu(),
               extrapolated=True,
               sample="one full single-threaded oracle solve (all %d sweeps) of the n=%d instance of the workload "
                      "law, %.1f s measured; value scaled to n=%d by (%d/%d)^3 and by the oracle's %d sweeps on "
                      "the n=%d input" % (r["sweeps"], ns, dt, n_full, n_full, ns, sweeps_full, n_full),
               measured=dict(n=ns, seconds=dt, sweeps=r["sweeps"], status=r["status"], eigenpairs_per_s=ns / dt),
               workload1_seconds=dt1)
    out["batched"] = cpu_baseline_batched(batch_every, batch_procs)
    return out


_BATCH_SAMPLE = []


def _oracle_member(k):
    import oracle
    G, J = _BATCH_SAMPLE[k]
    t = time.perf_counter()
    r = oracle.solve(G, J, vectors=False)
    return time.perf_counter() - t, r["status"]


def cpu_baseline_batched(every, procs):
    """The oracle over `procs` worker processes on every `every`-th member of
    the batched workload; mats/s = members / wall time of the pool."""
    import multiprocessing as mp

    import jjgen
    specs = jjgen.batch_recipe(count=4096)[::every]
    procs = max(1, min(procs, len(os.sched_getaffinity(0))))
    _BATCH_SAMPLE.clear()
    for sp in specs:
        G, J, _ = jjgen.batch_member(sp)
        _BATCH_SAMPLE.append((G, J))
    with mp.get_context("fork").Pool(procs) as pool:
        t = time.perf_counter()
        res = pool.map(_oracle_member, range(len(specs)), chunksize=1)
        wall = time.perf_counter() - t
    _BATCH_SAMPLE.clear()
    return dict(value=len(specs) / wall, unit="mats/s", cores=procs, kind="oracle",
                sample="%d members (every %d-th of the 4096-matrix batch, %d real / %d complex), one oracle solve "
                       "each over a pool of %d processes, %.1f s wall" % (
                           len(specs), every, sum(not s["cplx"] for s in specs), sum(s["cplx"] for s in specs),
                           procs, wall),
                seconds=wall, cpu_seconds=float(sum(x[0] for x in res)),
                statuses={str(v): [x[1] for x in res].count(v) for v in set(x[1] for x in res)})


def bench_batched(jj, torch, count, loop_sample):
    """Mixed-size batch: `count` matrices, n ~ U{16..512}, half real float64 and
    half complex128, inertia ~ U{0..n}, |lambda| log-uniform in [1e-6, 1e3].
    One jjacobi_solve_batched call (graph-replayed device step loop) with mixed
    precision on (FP32-MFMA Gram in each problem's pre-sweeps) and one in plain
    FP64, each against a loop of single jjacobi_solve_ex calls of the same form
    on an evenly spaced sample."""
    import jjgen
    specs = jjgen.batch_recipe(count=count)
    t = time.perf_counter()
    flat, offs, Js, lams_pres = jjgen.make_batch(specs)
    gen_s = time.perf_counter() - t
    note("batch of %d generated in %.1f s" % (count, gen_s))
    dev = torch.device("cuda:0")
    pristine = torch.from_numpy(flat).to(dev)
    work = torch.empty_like(pristine)
    vbuf = torch.empty_like(pristine)
    ns = [s["n"] for s in specs]
    loff = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    lam = torch.empty(int(loff[-1]), dtype=torch.float64, device=dev)
    dts = [1 if s["cplx"] else 0 for s in specs]
    base, vbase, lbase = work.data_ptr(), vbuf.data_ptr(), lam.data_ptr()
    Gp = [base + 8 * int(o) for o in offs[:-1]]
    Vp = [vbase + 8 * int(o) for o in offs[:-1]]
    Lp = [lbase + 8 * int(o) for o in loff[:-1]]
    stream = torch.cuda.current_stream().cuda_stream
    col2 = []  # squared column norms of every input (trace invariant)
    for k in range(count):
        g = flat[offs[k]:offs[k + 1]]
        c2 = (np.abs(g.view(np.complex128)) ** 2 if specs[k]["cplx"] else g * g).reshape(ns[k], ns[k]).sum(axis=1)
        col2.append(c2)
    idx = list(range(0, count, max(1, count // max(1, loop_sample))))[:loop_sample]
    out, lam_by_form = {}, {}
    for form, extra in (("mixed", dict(precision=1)), ("fp64", {})):
        opts = jj.make_opts(stream=stream, **extra)
        infos = (jj.jj_info * count)()

        def run():
            work.copy_(pristine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = jj.jjacobi_solve_batched(count, dts, Gp, Js, ns, ns, Lp, Vp, ns, 0.0, 0, opts, infos)
            torch.cuda.synchronize()
            return st, time.perf_counter() - t0

        st_warm, dt_warm = run()  # includes the block-width autotuning of each size bucket (first form)
        st, dt = run()
        note("batched %s: %.2f s" % (form, dt))
        statuses = [infos[k].status for k in range(count)]
        sweeps = [infos[k].sweeps for k in range(count)]
        msw = [infos[k].mixed_sweeps for k in range(count)]
        lam_h = lam.cpu().numpy()
        lam_by_form[form] = lam_h
        # invariants of every result: Sylvester inertia and trace(H) = sum_i j_i ||g_i||^2;
        # accuracy against the prescribed spectrum
        inertia_bad, tr_err, pres_err = 0, 0.0, []
        for k in range(count):
            lk = lam_h[loff[k]:loff[k + 1]]
            inertia_bad += int(np.sum(lk > 0) != np.sum(Js[k] > 0))
            tr = float(np.sum(Js[k].astype(float) * col2[k]))
            tr_err = max(tr_err, abs(float(np.sum(lk)) - tr) / float(np.sum(np.abs(lk))))
            pres = np.sort(lams_pres[k])[::-1]
            pres_err.append(float(np.max(np.abs(lk - pres) / np.abs(pres))))
        # loop of single solves of the same form on the sample, scaled to the whole batch
        work.copy_(pristine)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in idx:
            info = jj.jj_info()
            jj.jjacobi_solve_ex(dts[k], Gp[k], Js[k], ns[k], ns[k], Lp[k], Vp[k], ns[k], 0.0, 0, opts, info)
        torch.cuda.synchronize()
        dt_loop = (time.perf_counter() - t0) * count / len(idx)
        out[form] = dict(value=count / dt, seconds=dt, worst_status=st,
                         status_counts={str(v): statuses.count(v) for v in set(statuses)},
                         sweeps_max=max(sweeps), sweeps_mean=float(np.mean(sweeps)),
                         mixed_sweeps_mean=float(np.mean(msw)),
                         loop_of_single_solves=dict(value=count / dt_loop, unit="mats/s", sample=len(idx),
                                                    seconds_scaled=dt_loop),
                         speedup_vs_loop=dt_loop / dt, first_call_seconds=dt_warm,
                         invariants=dict(inertia_mismatches=inertia_bad, max_trace_rel_err=tr_err),
                         vs_prescribed_rel=dict(max=max(pres_err), median=float(np.median(pres_err))))
    a, b = lam_by_form["mixed"], lam_by_form["fp64"]
    out["mixed"]["vs_fp64_max_rel"] = float(np.max(np.abs(a - b) / np.abs(b)))
    out["mixed"]["speedup_vs_fp64_batch"] = out["fp64"]["seconds"] / out["mixed"]["seconds"]
    return dict(metric="batched mats/s (mixed precision on)", value=out["mixed"]["value"], unit="mats/s",
                count=count, speedup_vs_loop=out["mixed"]["speedup_vs_loop"], gen_seconds=gen_s,
                gbytes=flat.nbytes / 1e9, mixed=out["mixed"], fp64=out["fp64"],
                workload="4096 matrices, n ~ U{16..512}, half float64 half complex128, p ~ U{0..n}, "
                         "|lambda| log-uniform [1e-6, 1e3]" if count == 4096 else "batch of %d" % count)


def bench_small(jj, torch, k, reps):
    """Workloads 1 (n = 64 real) and 2 (n = 1024 complex, b = 32): median solve
    time over `reps` solves, sweeps, accuracy against the prescribed spectrum
    and against the stored oracle eigenvalues where they exist."""
    import jjgen
    G, J, lam_pres = jjgen.config(k)
    n = G.shape[0]
    cplx = np.iscomplexobj(G)
    dev = torch.device("cuda:0")
    pristine = torch.from_numpy(np.ascontiguousarray(G.T)).to(dev)
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty((n, n), dtype=pristine.dtype, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    o = jj.make_opts(stream=stream, block_width=32)
    times = []
    for r in range(reps + 1):
        Gw = pristine.clone()
        info = jj.jj_info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = jj.jjacobi_solve_ex(jj.JJ_C128 if cplx else jj.JJ_F64, Gw.data_ptr(), J, n, n, lam.data_ptr(),
                                 Vt.data_ptr(), n, 0.0, 0, o, info)
        torch.cuda.synchronize()
        if st != 0:
            raise RuntimeError("workload %d solve status %d" % (k, st))
        if r > 0:  # the first solve is a warm-up
            times.append(time.perf_counter() - t0)
    lh = lam.cpu().numpy()
    ref = np.sort(lam_pres)[::-1]
    out = dict(n=n, dtype="complex128" if cplx else "float64", seconds_median=float(np.median(times)),
               eigenpairs_per_s=n / float(np.median(times)), sweeps=info.sweeps,
               ms_per_sweep=1e3 * float(np.median(times)) / max(1, info.sweeps),
               vs_prescribed_max_rel=float(np.max(np.abs(lh - ref) / np.abs(ref))))
    ora, osw = stored_oracle(k)
    if ora is not None:
        out["vs_oracle_max_rel"] = float(np.max(np.abs(lh - ora) / np.abs(ora)))
        out["oracle_sweeps"] = osw
    return out


def bench_config4(jj, torch, steps):
    """n = 8192 complex Hermitian workload (p = 4096, |lambda| log-uniform in
    [1e-8, 1e2]): plain complex128 solves against the mixed form (FP32-MFMA
    Gram in the pre-sweeps, complex128 rotations, W_P and update throughout),
    timed back to back on the same input; accuracy against the prescribed
    spectrum and between the two forms."""
    import jjgen
    t = time.perf_counter()
    G, J, lam_pres = jjgen.config(4)
    gen_s = time.perf_counter() - t
    n = G.shape[0]
    dev = torch.device("cuda:0")
    pristine = torch.from_numpy(np.ascontiguousarray(G.T)).to(dev)
    del G
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty((n, n), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    ref = np.sort(lam_pres)[::-1]
    res = {}
    note("n=8192 complex input generated in %.1f s" % gen_s)
    # untimed one-sweep solve first: the library's block-width choice for this
    # size class (two timed sweeps per candidate) happens there
    Gw = pristine.clone()
    jj.jjacobi_solve_ex(jj.JJ_C128, Gw.data_ptr(), J, n, n, lam.data_ptr(), Vt.data_ptr(), n, 0.0, 1,
                        jj.make_opts(stream=stream), jj.jj_info())
    torch.cuda.synchronize()
    del Gw
    for name, extra in (("complex128", {}), ("mixed", dict(precision=1))):
        o = jj.make_opts(stream=stream, **extra)
        times, infos = [], []
        for _ in range(steps):
            Gw = pristine.clone()
            info = jj.jj_info()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = jj.jjacobi_solve_ex(jj.JJ_C128, Gw.data_ptr(), J, n, n, lam.data_ptr(), Vt.data_ptr(), n, 0.0, 0,
                                     o, info)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if st != 0:
                raise RuntimeError("n=8192 complex solve status %d" % st)
            infos.append(info.as_dict())
            note("n=8192 %s solve: %.2f s, %d sweeps" % (name, times[-1], info.sweeps))
            del Gw
        lh = lam.cpu().numpy()
        res[name] = dict(seconds=min(times), eigenpairs_per_s=n / min(times), sweeps=infos[-1]["sweeps"],
                         block_width=infos[-1]["block_width"],
                         mixed_sweeps=infos[-1]["mixed_sweeps"],
                         ms_per_sweep=1e3 * min(times) / infos[-1]["sweeps"],
                         vs_prescribed_max_rel=float(np.max(np.abs(lh - ref) / np.abs(ref))),
                         inertia_ok=bool(np.sum(lh > 0) == np.sum(J > 0)), lam=lh)
    a, b = res["complex128"].pop("lam"), res["mixed"].pop("lam")
    res["mixed"]["vs_complex128_max_rel"] = float(np.max(np.abs(a - b) / np.abs(a)))
    res["mixed"]["speedup_vs_complex128"] = res["complex128"]["seconds"] / res["mixed"]["seconds"]
    # complex128 per block width: whole solves at 32 and 64 (three-level pivots),
    # three sweeps at 16
    per = {}
    for bw, cap in ((32, 0), (64, 0), (16, 3)):
        o = jj.make_opts(stream=stream, block_width=bw)
        Gw = pristine.clone()
        info = jj.jj_info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = jj.jjacobi_solve_ex(jj.JJ_C128, Gw.data_ptr(), J, n, n, lam.data_ptr(), Vt.data_ptr(), n, 0.0, cap, o,
                                 info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del Gw
        row = dict(seconds=dt, sweeps=info.sweeps, ms_per_sweep=1e3 * dt / max(1, info.sweeps), status=st,
                   whole_solve=cap == 0)
        if cap == 0:
            lh = lam.cpu().numpy()
            row["vs_prescribed_max_rel"] = float(np.max(np.abs(lh - ref) / np.abs(ref)))
            row["vs_complex128_default_max_rel"] = float(np.max(np.abs(lh - a) / np.abs(a)))
        per[str(bw)] = row
        note("n=8192 complex128 block width %d: %.2f s, %d sweeps" % (bw, dt, info.sweeps))
    res["per_block_width"] = per
    return dict(workload="n=8192 complex Hermitian, J with 4096 positive, |lambda| log-uniform [1e-8, 1e2]",
                steps=steps, gen_seconds=gen_s, **res)


def bench_inner_modes(jj, torch, ks=(3, 2)):
    """The two pivot variants side by side on workloads 3 and 2: block-oriented
    (one inner pass over each pivot's off-diagonal block per step, Section 3.4;
    the default) and full pivot diagonalisation (inner sweeps until no rotation,
    Section 3.3).  Per variant: one graph-replayed solve (time, sweeps) after a
    warm-up, and one profiled solve for the per-kernel times and the roofline
    of its dominant kernel."""
    import jjgen
    out = {}
    for k in ks:
        G, J, lam_pres = jjgen.config(k)
        n = G.shape[0]
        cplx = np.iscomplexobj(G)
        dev = torch.device("cuda:0")
        pristine = torch.from_numpy(np.ascontiguousarray(G.T)).to(dev)
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        Vt = torch.empty((n, n), dtype=pristine.dtype, device=dev)
        stream = torch.cuda.current_stream().cuda_stream
        ref = np.sort(lam_pres)[::-1]
        res = {}
        for name, mode in (("block_oriented", 0), ("full", 1)):
            row = {}
            for profiled in (False, False, True):
                o = jj.make_opts(stream=stream, block_width=32, inner_mode=mode, profile=1 if profiled else 0)
                Gw = pristine.clone()
                info = jj.jj_info()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = jj.jjacobi_solve_ex(jj.JJ_C128 if cplx else jj.JJ_F64, Gw.data_ptr(), J, n, n, lam.data_ptr(),
                                         Vt.data_ptr(), n, 0.0, 0, o, info)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if st != 0:
                    raise RuntimeError("workload %d inner_mode %d: status %d" % (k, mode, st))
                if profiled:
                    pr = jj.jjacobi_last_profile()
                    rf, wk = roofline(pr, n, cplx)
                    row["roofline"] = rf
                    row["kernel_ms_per_solve"] = {kk: pr[kk]["ms"] for kk in ("gram", "pivot", "update", "final")}
                    row["inner_sweeps"] = pr["inner_sweeps"]
                    row["rotations"] = pr["rotations"]
                else:
                    row["seconds"] = dt  # the second unprofiled solve is kept (the first is a warm-up)
                    row["sweeps"] = info.sweeps
            lh = lam.cpu().numpy()
            row["vs_prescribed_max_rel"] = float(np.max(np.abs(lh - ref) / np.abs(ref)))
            row["ms_per_sweep"] = 1e3 * row["seconds"] / max(1, row["sweeps"])
            res[name] = row
            note("workload %d %s: %.1f ms, %d sweeps" % (k, name, 1e3 * row["seconds"], row["sweeps"]))
        res["full_over_block_oriented_time"] = res["full"]["seconds"] / res["block_oriented"]["seconds"]
        out["config%d" % k] = res
    return out


def bench_pairing(jj, torch, ks=(3, 2)):
    """Round-robin (Section 4.2, the default) against modulus pairing (Section
    4.1, one more step per sweep) on workloads 3 and 2: time and sweeps of one
    graph-replayed solve each after a warm-up, block width 32."""
    import jjgen
    out = {}
    for k in ks:
        G, J, _ = jjgen.config(k)
        n = G.shape[0]
        cplx = np.iscomplexobj(G)
        dev = torch.device("cuda:0")
        pristine = torch.from_numpy(np.ascontiguousarray(G.T)).to(dev)
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        Vt = torch.empty((n, n), dtype=pristine.dtype, device=dev)
        stream = torch.cuda.current_stream().cuda_stream
        res = {}
        for name, strat in (("round_robin", 0), ("modulus", 1)):
            o = jj.make_opts(stream=stream, block_width=32, strategy=strat)
            for rep in range(2):
                Gw = pristine.clone()
                info = jj.jj_info()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = jj.jjacobi_solve_ex(jj.JJ_C128 if cplx else jj.JJ_F64, Gw.data_ptr(), J, n, n, lam.data_ptr(),
                                         Vt.data_ptr(), n, 0.0, 0, o, info)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if st != 0:
                    raise RuntimeError("workload %d strategy %d: status %d" % (k, strat, st))
            res[name] = dict(seconds=dt, sweeps=info.sweeps, ms_per_sweep=1e3 * dt / max(1, info.sweeps))
            note("workload %d %s pairing: %.1f ms, %d sweeps" % (k, name, 1e3 * dt, info.sweeps))
        res["modulus_over_round_robin_time"] = res["modulus"]["seconds"] / res["round_robin"]["seconds"]
        out["config%d" % k] = res
    return out


def stored_long_oracle(k):
    """Long-double oracle eigenvalues of workload k (the adjudicator), or None."""
    path = os.path.join(ROOT, "tests", "golden", "config%d_lambda_long.txt" % k)
    if not os.path.exists(path):
        return None
    return np.loadtxt(path, dtype=np.longdouble).astype(np.float64)


def stored_oracle(k):
    path = os.path.join(ROOT, "tests", "golden", "config%d_lambda_double.txt" % k)
    if not os.path.exists(path):
        return None, None
    sweeps = None
    with open(path) as f:
        for line in f:
            if line.startswith("# status"):
                sweeps = int(line.split()[4])
    return np.loadtxt(path), sweeps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--block-width", type=int, default=0, help="0: library choice (tuned)")
    ap.add_argument("--inner-mode", type=int, default=-1, help="-1: library choice")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--loop-sample", type=int, default=64)
    ap.add_argument("--no-c4", action="store_true", help="skip the n=8192 complex leg")
    ap.add_argument("--no-small", action="store_true", help="skip the n=64 and n=1024 legs")
    ap.add_argument("--c4-steps", type=int, default=1)
    ap.add_argument("--no-inner-modes", action="store_true", help="skip the pivot-variant comparison")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the timed region, one device copy of this many MiB (a reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X and has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    import jjgen
    import paper_1008_4166_amd as jj

    t = time.perf_counter()
    G, J, lam_pres = jjgen.config(WORKLOAD)
    gen_s = time.perf_counter() - t
    n = G.shape[0]
    dev = torch.device("cuda:0")
    # G is Fortran-ordered: G.T is C-contiguous with the column-major bytes of G
    pristine = torch.from_numpy(np.ascontiguousarray(G.T)).to(dev)
    K, W = args.steps, args.warmup
    if args.copy_probe_mb > 0:
        a = torch.empty(args.copy_probe_mb * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    work = [pristine.clone() for _ in range(K + W)]
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty((n, n), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    # Solves replay one captured HIP graph per sweep.  The last timed solve is
    # the profiled one: it launches the same kernels eagerly, each recording a
    # pair of HIP events at its own dispatch start and end, which give the
    # per-kernel durations of the roofline below (it is a little slower than a
    # replayed solve, and it is counted in the timed region).
    opts = jj.make_opts(stream=stream, block_width=args.block_width, inner_mode=args.inner_mode, profile=0)
    popts = jj.make_opts(stream=stream, block_width=args.block_width, inner_mode=args.inner_mode, profile=1)
    infos = []

    def step(Gbuf, profiled):
        info = jj.jj_info()
        st = jj.jjacobi_solve_ex(jj.JJ_F64, Gbuf.data_ptr(), J, n, n, lam.data_ptr(), Vt.data_ptr(), n, 0.0, 0,
                                 popts if profiled else opts, info)
        if st not in (0,):
            raise RuntimeError("solve status %d (%s)" % (st, jj.jjacobi_status_string(st)))
        infos.append(info.as_dict())
        return jj.jjacobi_last_profile() if profiled else None

    note("workload 3 (n=%d) generated in %.1f s; %d warm-up + %d timed solves" % (n, gen_s, W, K))
    for i in range(W):
        step(work[i], False)
    torch.cuda.synchronize()
    profs = []
    t0 = time.perf_counter()
    for i in range(K):
        profs.append(step(work[W + i], not args.no_profile and i == K - 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    ms_step = dt / K * 1e3
    timed_infos = infos[W:]
    sweeps = [i["sweeps"] for i in timed_infos]

    # accuracy of the last timed solve
    lam_h = lam.cpu().numpy()
    ref, oracle_sweeps = stored_oracle(WORKLOAD)
    acc = {"vs_prescribed_max_rel": float(np.max(np.abs(lam_h - np.sort(lam_pres)[::-1]) / np.abs(np.sort(lam_pres)[::-1])))}
    if ref is not None:
        acc["vs_oracle_max_rel"] = float(np.max(np.abs(lam_h - ref) / np.abs(ref)))
        acc["vs_oracle_p99_rel"] = float(np.percentile(np.abs(lam_h - ref) / np.abs(ref), 99))
    ref_long = stored_long_oracle(WORKLOAD)
    if ref_long is not None:
        # the long-double oracle separates the input's conditioning from error
        acc["vs_long_oracle_max_rel"] = float(np.max(np.abs(lam_h - ref_long) / np.abs(ref_long)))
        if ref is not None:
            acc["oracle_vs_long_oracle_max_rel"] = float(np.max(np.abs(ref - ref_long) / np.abs(ref_long)))

    out = {
        "metric": "eigenpairs/s (n=4096 FP64 solve); sweep time, FP64-MFMA fraction reported alongside",
        "value": n * K / dt,
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "blocked real symmetric indefinite n=4096 float64, J with 3000 positive, "
                               "|lambda| log-uniform [1e-12, 1], plain FP64",
                   "n": n, "block_width": timed_infos[-1]["block_width"], "nblocks": timed_infos[-1]["nblocks"],
                   "pairing": "round-robin", "inner_mode": timed_infos[-1]["inner_mode"]},
        "sweeps": sweeps,
        "ms_per_sweep": ms_step / (sum(sweeps) / len(sweeps)),
        "c_time_model": (dt / K) / n ** 3,
        "accuracy": acc,
        "gen_seconds": gen_s,
    }
    if not args.no_profile and profs[-1] is not None:
        pr = profs[-1]
        rf, wk = roofline(pr, n, False)
        out["roofline"] = rf
        out["kernels"] = {k: dict(ms_total=pr[k]["ms"], launches=pr[k]["launches"],
                                  avg_ms=wk[k]["ms"] if k in wk else None,
                                  gflops_per_launch=wk[k]["flops"] / 1e9 if k in wk else None,
                                  gbytes_per_launch=wk[k]["bytes"] / 1e9 if k in wk else None)
                          for k in ("gram", "pivot", "update", "final", "other")}
        out["inner"] = dict(rotations=pr["rotations"], inner_sweeps=pr["inner_sweeps"])
    # mixed-precision form (FP32-MFMA Gram in pre-sweeps, FP64 rotations, W_P and update)
    note("timed solves: %.1f ms each" % ms_step)
    if not args.no_mixed:
        mopts = jj.make_opts(stream=stream, block_width=args.block_width, inner_mode=args.inner_mode, precision=1)
        mwork = [pristine.clone() for _ in range(K)]
        minfos = []
        torch.cuda.synchronize()
        t0m = time.perf_counter()
        for i in range(K):
            info = jj.jj_info()
            st = jj.jjacobi_solve_ex(jj.JJ_F64, mwork[i].data_ptr(), J, n, n, lam.data_ptr(), Vt.data_ptr(), n, 0.0,
                                     0, mopts, info)
            if st != 0:
                raise RuntimeError("mixed solve status %d" % st)
            minfos.append(info.as_dict())
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0m
        lam_m = lam.cpu().numpy()
        macc = {"vs_fp64_gpu_max_rel": float(np.max(np.abs(lam_m - lam_h) / np.abs(lam_h)))}
        if ref is not None:
            macc["vs_oracle_max_rel"] = float(np.max(np.abs(lam_m - ref) / np.abs(ref)))
        if ref_long is not None:
            macc["vs_long_oracle_max_rel"] = float(np.max(np.abs(lam_m - ref_long) / np.abs(ref_long)))
        out["mixed"] = dict(value=n * K / dtm, ms_per_step=dtm / K * 1e3, sweeps=[i["sweeps"] for i in minfos],
                            mixed_sweeps=[i["mixed_sweeps"] for i in minfos], accuracy=macc,
                            speedup_vs_fp64=ms_step / (dtm / K * 1e3))
    if not args.no_small:
        note("workloads 1 and 2")
        out["config1"] = bench_small(jj, torch, 1, 20)
        out["config2"] = bench_small(jj, torch, 2, 5)
    if not args.no_inner_modes:
        note("pivot variants (block-oriented / full) on workloads 3 and 2")
        out["inner_modes"] = bench_inner_modes(jj, torch)
        note("pairing strategies (round-robin / modulus) on workloads 3 and 2")
        out["pairing"] = bench_pairing(jj, torch)
    if not args.no_batched:
        note("batched leg")
        out["batched"] = bench_batched(jj, torch, args.batch_count, args.loop_sample)
    if not args.no_c4:
        note("n=8192 complex leg")
        del work
        out["config4"] = bench_config4(jj, torch, args.c4_steps)
    if not args.no_cpu:
        note("cpu baseline (oracle samples)")
        out["cpu_baseline"] = cpu_baseline(n, oracle_sweeps if oracle_sweeps else 14)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
