"""Benchmark of the displaced-probing hot path on one MI355X.

One JSON line per run.  --workload picks the lattice problem:

  gauge16-nested (default; the headline line)
      Gauge-covariant 3-colour Laplacian on a 16^4 torus, links
      U = exp(i 0.4 H) (seed 1), m2 = 0.05, displacement p = 4 along
      dimension 0, nested displaced colourings at distances 1, 2, 4, 8
      (3 / 5 / 16 / 960 colours).  One step is the probed trace estimate of
      the finest level for one noise sample: 960 x 3 = 2880 diluted
      Z2-complex probes, generated on the device, solved by batched CG (FP32
      vectors and links, FP32 accumulation, FP64 reliable updates, tol 1e-8)
      and contracted with the displacement.
  uneven-batch
      64 independent gauge 3-colour instances (extents from {4..12}^4, m2,
      eps and p drawn per instance), each with its own distance-4 colouring;
      one step is one noise sample of every instance in one multi-instance
      call (BF16 vectors and links, FP64 reliable updates, tol 1e-8).  The
      same instances solved one call at a time are timed beside it.
  gauge32-grad
      32^4 x 3, eps = 0.5, m2 = 0.01, p = 8, distance-8 colouring (32
      colours); one step is one sample of the trace and its adjoint gradient
      (dT/dm2 and dT/dU for every link): 96 forward and 96 adjoint solves in
      FP64, tol 1e-10, and the force pass.
  gauge8-plain
      8^4 x 3, eps = 0.3, m2 = 0.1, p = 2, distance-4 colouring (best
      order, 64 colours); one step is one sample solved by plain
      single-right-hand-side FP64 CG (W = 1), tol 1e-10.

value = RHS * site * CG-iteration / s over the K timed steps (iterations
counted per right-hand side up to its own convergence).  The roofline object
is for the stencil kernel (the dominant kernel): its launches are timed with
HIP events on the stream they run on, inside the timed region, and the
library reports their algorithmic bytes.  cpu_baseline is the FP64 oracle
on a bounded sample of the same right-hand sides.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "RHS*site*CG-iter/s (probed Tr(P A^-1), batched mixed-precision CG)"
UNIT = "RHS*site*CG-iter/s"
WORKLOADS = ("gauge16-nested", "uneven-batch", "gauge32-grad", "gauge8-plain")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default per workload)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gauge16-nested", choices=WORKLOADS)
    ap.add_argument("--rhs-block", type=int, default=None, help="W (0: autotune; default per workload)")
    ap.add_argument("--inner", default=None, help="inner storage precision (default per workload)")
    ap.add_argument("--delta", type=float, default=0.0,
                    help="reliable-update residual drop (0: the library default for the precision)")
    ap.add_argument("--graph", type=int, default=0, help="replay CG iteration groups from hipGraphs")
    ap.add_argument("--profile", type=int, default=1, help="time the stencil launches with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the comparison runs")
    ap.add_argument("--cpu-rhs", type=int, default=0, help="right-hand sides per oracle call in the CPU sample (0: cores)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (reference for byte counters)")
    return ap.parse_args()


def kernel_sha():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2106_01275_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def host_threads():
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))


def roofline(stats, tag):
    """Stencil roofline from the library's event timings and algorithmic bytes."""
    launches = sum(s["stencil_launches"] for s in stats)
    ms = sum(s["stencil_ms"] for s in stats)
    nbytes = sum(s["stencil_bytes"] for s in stats)
    if not launches or ms <= 0:
        return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": "k_stencil", "launches": 0}
    achieved = nbytes / (ms / 1e3) / 1e9
    per_launch = nbytes / launches
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"stencil_{tag}_traffic.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        alg = t.get("alg_bytes_per_launch", 0)
        if t.get("kernels_hip_sha") == kernel_sha() and abs(alg - per_launch) <= 0.05 * per_launch:
            traffic = t.get("hbm_bytes_per_launch")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "k_stencil (q = A p, p^H q)",
            "launches": launches, "avg_launch_us": ms / launches * 1e3, "alg_bytes_per_launch": per_launch}


def timed(torch, fn, steps, warmup):
    for s in range(warmup):
        fn(1000 + s, False)
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for s in range(steps):
        res.append(fn(s, True))
    torch.cuda.synchronize()
    return res, time.perf_counter() - t0


def cpu_oracle(dims, nc, m2, U, B, tol, maxit=100000):
    """Times the FP64 oracle's CG (one right-hand side per host thread)."""
    import oracle
    t = time.perf_counter()
    _, its, _ = oracle.cg_many(dims, nc, m2, U, B, tol=tol, maxit=maxit)
    t = time.perf_counter() - t
    its = np.where(its < 0, maxit, its)
    return float(its.sum()) * int(np.prod(dims)), t


def cpu_budget(dims, nc, m2, U, col, m, seed, tol, chunk, budget=10.0, maxit=100000, max_samples=64):
    """Times the oracle on right-hand sides of samples 0, 1, ... in order (diluted Z2-complex
    probes of the colouring), chunk at a time, until `budget` seconds of CPU work; returns
    (work, seconds, right-hand sides used)."""
    import oracle
    work = t = 0.0
    used = 0
    for smp in range(max_samples):
        for j0 in range(0, m * nc, chunk):
            js = range(j0, min(j0 + chunk, m * nc))
            B = np.stack([oracle.probe(dims, nc, col, seed, smp, j // nc, j % nc, True, oracle.Z2_COMPLEX)
                          for j in js])
            wk, tc = cpu_oracle(dims, nc, m2, U, B, tol, maxit)
            work, t, used = work + wk, t + tc, used + len(js)
            if t >= budget:
                return work, t, used
    return work, t, used


# --------------------------------------------------------------------- workloads


def run_gauge16(a, torch, dp, workloads):
    w = workloads.GAUGE_16
    inner = a.inner or "f32"
    W_req = 32 if a.rhs_block is None else a.rhs_block
    steps = a.steps or 3
    dims, nc, p, N = w.dims, w.nc, w.p, w.volume
    t0 = time.time()
    cols, ncols, _ = dp.build_coloring(dims, p, list(w.ks), "natural")
    t_color = time.time() - t0
    level = len(w.ks) - 1
    col = np.ascontiguousarray(cols[level])
    m = int(ncols[level])
    U = w.links()
    c = dp.context(0)
    Ug = torch.from_numpy(U).cuda()
    colg = torch.from_numpy(col).cuda()
    op = c.operator(dims, nc, w.m2, Ug)
    opts = c.opts(tol=w.tol, inner=inner, rhs_block=W_req, reliable_delta=a.delta, use_graph=a.graph)

    def step(sample, in_timed):
        ps = c.probe_spec(dims, nc, colg, m, w.noise_seed, sample, 1, "z2_complex", True)
        opts.profile = a.profile if in_timed else 0
        return c.trace_estimate([op], [ps], [p], opts)[0]

    res, elapsed = timed(torch, step, steps, a.warmup)
    stats = [r["solve"] for r in res]
    rhs_iters = sum(s["rhs_iters"] for s in stats)
    W = stats[0]["rhs_block"]
    Ts = np.array([r["T"] for r in res])
    sec_per_sample = elapsed / steps
    tt = None
    if steps >= 2:
        var = float(np.var(Ts, ddof=1))
        s_star = max(1, int(np.ceil(var / (1e-3 * abs(Ts.mean())) ** 2)))
        tt = {"samples": s_star, "seconds": s_star * sec_per_sample, "per_sample_var": var,
              "T_mean": [Ts.mean().real, Ts.mean().imag]}
    extra = {"time_to_trace_1e-3": tt}
    if not a.no_plain and tt is not None:
        # time to 1e-3 relative error per nested level (k = 1, 2, 4, 8) and for plain Hutchinson (one
        # colour): per-sample variance from 8 samples (the finest level: the timed samples), samples
        # needed = var / (1e-3 |T|)^2, seconds = that many samples at the measured seconds per sample
        opts.profile = 0
        levels = []
        lv_cols = [(f"k={k}", cols[i], int(ncols[i])) for i, k in enumerate(w.ks)]
        lv_cols.insert(0, ("hutchinson", np.zeros(N, dtype=np.int32), 1))
        for name, cl, ml in lv_cols:
            if name == f"k={w.ks[level]}":
                sec, var, Tm = sec_per_sample, tt["per_sample_var"], complex(*tt["T_mean"])
            else:
                ps = c.probe_spec(dims, nc, torch.from_numpy(np.ascontiguousarray(cl)).cuda(), ml, w.noise_seed,
                                  0, 8, "z2_complex", True)
                torch.cuda.synchronize()
                tl = time.perf_counter()
                r = c.trace_estimate([op], [ps], [p], opts)[0]
                torch.cuda.synchronize()
                sec = (time.perf_counter() - tl) / 8
                var, Tm = float(np.var(r["per_sample"], ddof=1)), r["T"]
            need = max(1, int(np.ceil(var / (1e-3 * abs(Tm)) ** 2)))
            levels.append({"level": name, "colours": ml, "rhs_per_sample": ml * nc, "seconds_per_sample": sec,
                           "per_sample_var": var, "samples_for_1e-3": need, "seconds_to_1e-3": need * sec})
        extra["levels_time_to_1e-3"] = levels
    if not a.no_plain:
        # one probe set for the displacements n = 0..8 (Sec. 4.3): the same solves, nine contractions
        ps = c.probe_spec(dims, nc, colg, m, w.noise_seed, 0, 1, "z2_complex", True)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        rm = c.trace_multi(op, ps, list(range(9)), c.opts(tol=w.tol, inner=inner, rhs_block=W))
        torch.cuda.synchronize()
        tm = time.perf_counter() - tm
        extra["multi_displacement"] = {"displacements": list(range(9)), "seconds": tm,
                                       "seconds_one_displacement": sec_per_sample,
                                       "T": [[r_["T"].real, r_["T"].imag] for r_ in rm]}
        if level == len(w.ks) - 1 and level > 0:
            # every coarser nested level from the finest level's solves (one sample)
            coarse = [(torch.from_numpy(np.ascontiguousarray(cols[i])).cuda(), int(ncols[i])) for i in range(level)]
            torch.cuda.synchronize()
            tn = time.perf_counter()
            rn = c.trace_levels(op, ps, p, coarse, c.opts(tol=w.tol, inner=inner, rhs_block=W))
            torch.cuda.synchronize()
            tn = time.perf_counter() - tn
            extra["levels_from_finest"] = {"levels": [f"k={k}" for k in w.ks[:level]] + [f"k={w.ks[level]}"],
                                           "seconds": tn, "seconds_finest_alone": sec_per_sample,
                                           "T": [[r_["T"].real, r_["T"].imag] for r_ in rn[1:] + rn[:1]]}
        # plain single-RHS FP64 GPU solver on a few of the same right-hand sides
        nplain = 8
        ps = c.probe_spec(dims, nc, colg, m, w.noise_seed, 0, 1, "z2_complex", True)
        Bp = c.make_probes(ps, 0, nplain)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        (_,), (stp,) = c.solve_batch([op], [Bp], c.opts(tol=w.tol, inner="f64", rhs_block=1))
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        sec = tp / nplain * (m * nc)
        extra["plain_fp64_single_rhs"] = {"rhs": nplain, "seconds_per_sample_extrapolated": sec,
                                          "rhs_site_iter_per_s": stp["rhs_iters"] * N / tp,
                                          "speedup_batched_mixed": sec / sec_per_sample}
    cpu = None
    if not a.no_cpu_baseline:
        threads = host_threads()
        work, tc, used = cpu_budget(dims, nc, w.m2, U, col, m, w.noise_seed, w.tol, a.cpu_rhs or threads)
        cpu = {"value": work / tc, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"the first {used} of the {m * nc} right-hand sides of sample 0 (FP64 CG, tol {w.tol}), "
                         f"{tc:.1f} s"}
    config = {"workload": "gauge-16^4x3-nested: 16^4 torus, 3 colours, m2=0.05, eps=0.4, p=4, "
                          "nested distances 1,2,4,8 (finest level, 960 colours, 2880 diluted RHS "
                          "per step), Z2 complex noise, tol 1e-8",
              "rhs_per_step": sum(s["nrhs"] for s in stats) // steps, "rhs_block": W, "inner": inner,
              "colours": [int(v) for v in ncols], "coloring_seconds": t_color}
    return (steps, elapsed, rhs_iters * N, inner, config, roofline(stats, f"gauge16_{inner}_w{W}"), cpu,
            stats, extra)


def run_uneven(a, torch, dp, workloads):
    inst = workloads.uneven_batch()
    inner = a.inner or "bf16"
    # the width from the autotuner (rhs_block 0): 32 for this batch, the measured best
    # (W = 16/32/64/128: 133/123/141/159 ms per step)
    W_req = 0 if a.rhs_block is None else a.rhs_block
    steps = a.steps or 3
    c = dp.context(0)
    t0 = time.time()
    ops, cols, links = [], [], []
    for w in inst:
        col, m, _ = dp.build_coloring(w.dims, w.p, w.ks[0], w.order)
        U = w.links()
        links.append(U)
        cols.append((torch.from_numpy(np.ascontiguousarray(col)).cuda(), m, col))
        ops.append(c.operator(w.dims, w.nc, w.m2, torch.from_numpy(U).cuda()))
    t_color = time.time() - t0
    opts = c.opts(tol=inst[0].tol, inner=inner, rhs_block=W_req, reliable_delta=a.delta, use_graph=a.graph)

    def specs(sample):
        return [c.probe_spec(w.dims, w.nc, cg, m, w.noise_seed, sample, 1, "z2_complex", True)
                for w, (cg, m, _) in zip(inst, cols)]

    def step(sample, in_timed):
        opts.profile = a.profile if in_timed else 0
        return c.trace_estimate(ops, specs(sample), [w.p for w in inst], opts)

    res, elapsed = timed(torch, step, steps, a.warmup)
    stats = [r["solve"] for rr in res for r in rr]
    work = sum(s["rhs_iters"] * w.volume for rr in res for s, w in zip((r["solve"] for r in rr), inst))
    W = stats[0]["rhs_block"]
    extra = {}
    if not a.no_plain:
        # the same instances, one call each (same options, same samples)
        seq_opts = c.opts(tol=inst[0].tol, inner=inner, rhs_block=W, reliable_delta=a.delta,
                          use_graph=a.graph)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for s in range(steps):
            for i, ps in enumerate(specs(s)):
                c.trace_estimate([ops[i]], [ps], [inst[i].p], seq_opts)
        torch.cuda.synchronize()
        ts = time.perf_counter() - ts
        extra["one_call_per_instance"] = {"seconds": ts, "speedup_multi_instance": ts / elapsed}
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        threads = host_threads()
        work_c, tc, used = 0.0, 0.0, 0
        for w, (_, m, col), U in zip(inst, cols, links):
            B = oracle.probes(w.dims, w.nc, col, m, w.noise_seed, 0, 1, oracle.Z2_COMPLEX, True)
            wk, t = cpu_oracle(w.dims, w.nc, w.m2, U, B, w.tol)
            work_c += wk
            tc += t
            used += 1
            if tc > 10.0:
                break
        cpu = {"value": work_c / tc, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"all right-hand sides of sample 0 of the first {used} instances "
                         f"(FP64 CG, tol {inst[0].tol}), {tc:.1f} s"}
    config = {"workload": "uneven-batch-64: 64 gauge 3-colour instances, extents from {4,6,8,10,12}^4, "
                          "m2 ~ U[0.05,0.5], eps ~ U[0.2,0.5], p in {1,2,3}, distance-4 colourings, one "
                          "Z2 complex sample per instance per step, tol 1e-8",
              "rhs_per_step": sum(s["nrhs"] for s in stats) // steps, "rhs_block": W, "inner": inner,
              "sites": sum(w.volume for w in inst), "coloring_seconds": t_color}
    return steps, elapsed, work, inner, config, roofline(stats, f"batch64_{inner}_w{W}"), cpu, stats, extra


def run_gauge32(a, torch, dp, workloads):
    w = workloads.GAUGE_32
    # FP32 storage with FP64 reliable updates: the same iterations and true residuals <= 1e-10 as FP64
    # storage (T and dT/dm2 agree to 3e-8) in 0.6 of the time
    inner = a.inner or "f32"
    W_req = 0 if a.rhs_block is None else a.rhs_block
    steps = a.steps or 1
    dims, nc, p, N = w.dims, w.nc, w.p, w.volume
    t0 = time.time()
    col, m, order = dp.build_coloring(dims, p, w.ks[0], w.order)
    t_color = time.time() - t0
    U = w.links()
    c = dp.context(0)
    Ug = torch.from_numpy(U).cuda()
    colg = torch.from_numpy(np.ascontiguousarray(col)).cuda()
    op = c.operator(dims, nc, w.m2, Ug)
    opts = c.opts(tol=w.tol, inner=inner, rhs_block=W_req, reliable_delta=a.delta, use_graph=a.graph)

    def step(sample, in_timed):
        ps = c.probe_spec(dims, nc, colg, m, w.noise_seed, sample, 1, "z2_complex", True)
        opts.profile = a.profile if in_timed else 0
        T, dm2, dU, dUb, st = c.trace_grad(op, ps, p, opts)
        return {"T": T, "dm2": dm2, "solve": st}

    res, elapsed = timed(torch, step, steps, a.warmup)
    stats = [r["solve"] for r in res]
    rhs_iters = sum(s["rhs_iters"] for s in stats)
    W = stats[0]["rhs_block"]
    cpu = None
    if not a.no_cpu_baseline:
        threads = host_threads()
        maxit = 20
        work, tc, used = cpu_budget(dims, nc, w.m2, U, col, m, w.noise_seed, w.tol, a.cpu_rhs or threads,
                                    maxit=maxit, max_samples=1)
        cpu = {"value": work / tc, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"first {maxit} CG iterations of the first {used} of the {m * nc} forward right-hand "
                         f"sides of sample 0 (FP64), {tc:.1f} s"}
    config = {"workload": f"gauge-32^4x3-grad: 32^4 torus, 3 colours, m2=0.01, eps=0.5, p=8, distance-8 "
                          f"colouring ({m} colours, {order} order), trace + adjoint gradient per step "
                          f"({m * nc} forward + {m * nc} adjoint RHS), Z2 complex noise, tol 1e-10",
              "rhs_per_step": sum(s["nrhs"] for s in stats) // steps, "rhs_block": W, "inner": inner,
              "coloring_seconds": t_color}
    extra = {"T": [res[0]["T"].real, res[0]["T"].imag], "dT_dm2": [res[0]["dm2"].real, res[0]["dm2"].imag]}
    return (steps, elapsed, rhs_iters * N, inner, config, roofline(stats, f"gauge32_{inner}_w{W}"), cpu,
            stats, extra)


def run_gauge8(a, torch, dp, workloads):
    w = workloads.GAUGE_8
    inner = a.inner or "f64"
    W_req = 1 if a.rhs_block is None else a.rhs_block
    steps = a.steps or 3
    dims, nc, p, N = w.dims, w.nc, w.p, w.volume
    col, m, order = dp.build_coloring(dims, p, w.ks[0], w.order)
    U = w.links()
    c = dp.context(0)
    colg = torch.from_numpy(np.ascontiguousarray(col)).cuda()
    op = c.operator(dims, nc, w.m2, torch.from_numpy(U).cuda())
    opts = c.opts(tol=w.tol, inner=inner, rhs_block=W_req, reliable_delta=a.delta, use_graph=a.graph)

    def step(sample, in_timed):
        ps = c.probe_spec(dims, nc, colg, m, w.noise_seed, sample, 1, "z2_complex", True)
        opts.profile = a.profile if in_timed else 0
        return c.trace_estimate([op], [ps], [p], opts)[0]

    res, elapsed = timed(torch, step, steps, a.warmup)
    stats = [r["solve"] for r in res]
    rhs_iters = sum(s["rhs_iters"] for s in stats)
    W = stats[0]["rhs_block"]
    cpu = None
    if not a.no_cpu_baseline:
        threads = host_threads()
        work, tc, used = cpu_budget(dims, nc, w.m2, U, col, m, w.noise_seed, w.tol, a.cpu_rhs or 4 * threads)
        cpu = {"value": work / tc, "unit": UNIT, "cores": threads, "kind": "oracle",
               "sample": f"{used} right-hand sides of samples 0, 1, ... ({m * nc} per sample; FP64 CG, "
                         f"tol {w.tol}), {tc:.1f} s"}
    config = {"workload": f"gauge-8^4x3-plain: 8^4 torus, 3 colours, m2=0.1, eps=0.3, p=2, distance-4 "
                          f"colouring ({m} colours, {order} order), one Z2 complex sample per step, "
                          f"single-RHS CG, tol 1e-10",
              "rhs_per_step": sum(s["nrhs"] for s in stats) // steps, "rhs_block": W, "inner": inner}
    return (steps, elapsed, rhs_iters * N, inner, config, roofline(stats, f"gauge8_{inner}_w{W}"), cpu,
            stats, {})


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1", "n_gpus": a.gpus}),
              flush=True)
        sys.exit(2)
    import torch

    import paper_2106_01275_amd as dp
    import workloads

    run = {"gauge16-nested": run_gauge16, "uneven-batch": run_uneven, "gauge32-grad": run_gauge32,
           "gauge8-plain": run_gauge8}[a.workload]
    steps, elapsed, work, inner, config, roof, cpu, stats, extra = run(a, torch, dp, workloads)
    out = {
        "metric": METRIC,
        "value": work / elapsed,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": inner,
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "cpu_baseline": cpu,
        "solve": {"rhs_iters": sum(s["rhs_iters"] for s in stats),
                  "max_iters": max(s["max_iters"] for s in stats),
                  "reliable_updates": sum(s["reliable_updates"] for s in stats),
                  "max_true_resid": max(s["max_true_resid"] for s in stats),
                  "nconverged": sum(s["nconverged"] for s in stats), "nrhs": sum(s["nrhs"] for s in stats)},
    }
    # whole-job bandwidth of the CG iterations: per stencil launch (one per CG iteration and slot)
    # an iteration moves 10 vector passes plus the links, (10 V W + 4 L) / (2 V W + 4 L) times the
    # stencil's own algorithmic bytes (every workload here is 3-colour with links); over the timed
    # wall time, with reliable updates, checks and contractions inside it but not counted
    cb = {"f64": 16, "f32": 8, "bf16": 4}[inner]
    vw, lk = cb * 3 * config["rhs_block"], cb * 9
    st_bytes = sum(s_["stencil_bytes_all"] for s_ in stats)
    if st_bytes > 0:
        cg_bytes = st_bytes * (10 * vw + 4 * lk) / (2 * vw + 4 * lk)
        out["cg_bandwidth"] = {"alg_bytes": cg_bytes, "achieved": cg_bytes / elapsed / 1e9, "unit": "GB/s",
                               "frac": cg_bytes / elapsed / 1e9 / HBM_PEAK_GBS}
    out.update(extra)
    if a.copy_ref_mib:
        # a plain copy kernel of known size: reads and writes copy_ref_mib MiB
        src = torch.ones(a.copy_ref_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_ref_mib"] = a.copy_ref_mib
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
