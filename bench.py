"""Benchmark of the displaced-probing hot path on one MI355X.

Workload (the 16^4 x 3 nested-level lattice): gauge-covariant 3-colour
Laplacian on a 16^4 torus, links U = exp(i 0.4 H) (seed 1), m2 = 0.05,
displacement p = 4 along dimension 0, nested displaced colourings at
distances 1, 2, 4, 8 (3 / 5 / 16 / 960 colours); one step is the probed
trace estimate of the finest level for one noise sample: 960 x 3 = 2880
diluted Z2-complex probes, generated on the device, solved by batched CG
(FP32 vectors and links, FP32 accumulation, FP64 reliable updates,
tol 1e-8) and contracted with the displacement.  Samples 0..K-1 are the K
timed steps.

Printed: one JSON line.  value = RHS * site * CG-iteration / s over the timed
steps (iterations counted per right-hand side up to its own convergence).
The roofline object is for the stencil kernel (the dominant kernel),
timed live with HIP events on the stream it runs on.  cpu_baseline is the
FP64 oracle (one right-hand side per host thread) on a bounded sample of
the same right-hand sides.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rhs-block", type=int, default=32)
    ap.add_argument("--inner", default="f32")
    ap.add_argument("--delta", type=float, default=1e-3, help="reliable-update residual drop")
    ap.add_argument("--graph", type=int, default=0, help="replay CG iteration groups from hipGraphs")
    ap.add_argument("--profile", type=int, default=1, help="time the stencil launches with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-rhs", type=int, default=0, help="right-hand sides in the CPU sample (0: cores)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (reference for byte counters)")
    return ap.parse_args()


def kernel_sha():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2106_01275_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    import torch

    import paper_2106_01275_amd as dp
    import workloads

    w = workloads.GAUGE_16
    dims, nc, p = w.dims, w.nc, w.p
    N = w.volume
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
    opts = c.opts(tol=w.tol, inner=a.inner, rhs_block=a.rhs_block, reliable_delta=a.delta, profile=1,
                  use_graph=a.graph)

    def step(sample, prof=a.profile):
        ps = c.probe_spec(dims, nc, colg, m, w.noise_seed, sample, 1, "z2_complex", True)
        opts.profile = prof
        return c.trace_estimate([op], [ps], [p], opts)[0]

    for s in range(a.warmup):
        step(1000 + s)
    torch.cuda.synchronize()
    res = []
    t_start = time.perf_counter()
    for s in range(a.steps):
        res.append(step(s))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start

    rhs_iters = sum(r["solve"]["rhs_iters"] for r in res)
    nrhs = sum(r["solve"]["nrhs"] for r in res)
    value = rhs_iters * N / elapsed
    Ts = np.array([r["T"] for r in res])
    launches = sum(r["solve"]["stencil_launches"] for r in res)
    st_ms = sum(r["solve"]["stencil_ms"] for r in res)
    W = res[0]["solve"]["rhs_block"]
    vbytes = {"f64": 16, "f32": 8, "bf16": 4}[a.inner] * nc     # per site per RHS
    lbytes = {"f64": 16, "f32": 8, "bf16": 4}[a.inner] * nc * nc  # per link
    alg_bytes = N * (2 * vbytes * W + 4 * lbytes)                 # read p, write q, links once
    avg_s = st_ms / 1e3 / max(launches, 1)
    achieved = alg_bytes / avg_s / 1e9 if launches else None

    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"stencil_gauge16_{a.inner}_w{W}_traffic.json")
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("kernels_hip_sha") == kernel_sha() and t.get("rhs_block") == W and t.get("inner") == a.inner:
            traffic = t.get("hbm_bytes_per_launch")

    # time-to-trace at 1e-3 relative error from the per-sample spread
    sec_per_sample = elapsed / a.steps
    tt = None
    if a.steps >= 2:
        var = float(np.var(Ts, ddof=1))
        s_star = max(1, int(np.ceil(var / (1e-3 * abs(Ts.mean())) ** 2)))
        tt = {"samples": s_star, "seconds": s_star * sec_per_sample, "per_sample_var": var,
              "T_mean": [Ts.mean().real, Ts.mean().imag]}

    # plain single-RHS FP64 GPU solver on a few of the same right-hand sides
    plain = None
    if not a.no_plain:
        nplain = 8
        ps = c.probe_spec(dims, nc, colg, m, w.noise_seed, 0, 1, "z2_complex", True)
        Bp = c.make_probes(ps, 0, nplain)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        (Xp,), (stp,) = c.solve_batch([op], [Bp], c.opts(tol=w.tol, inner="f64", rhs_block=1))
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        sec = tp / nplain * (m * nc)
        plain = {"rhs": nplain, "seconds_per_sample_extrapolated": sec,
                 "rhs_site_iter_per_s": stp["rhs_iters"] * N / tp,
                 "speedup_batched_mixed": sec / sec_per_sample}

    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        cores = os.cpu_count() or 1
        try:
            cores = len(os.sched_getaffinity(0))
        except Exception:
            pass
        omp = int(os.environ.get("OMP_NUM_THREADS", cores))
        threads = min(cores, omp)
        ncpu = a.cpu_rhs or threads
        B = oracle.probes(dims, nc, col, m, w.noise_seed, 0, 1, oracle.Z2_COMPLEX, True)[:ncpu]
        tc = time.perf_counter()
        X, its, rel = oracle.cg_many(dims, nc, w.m2, U, B, tol=w.tol)
        tc = time.perf_counter() - tc
        cpu = {"value": float(its.sum()) * N / tc, "unit": "RHS*site*CG-iter/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{ncpu} of the {m * nc} right-hand sides of one sample (FP64 CG, tol {w.tol}), "
                         f"{tc:.1f} s"}

    out = {
        "metric": "RHS*site*CG-iter/s (probed Tr(P A^-1), batched mixed-precision CG)",
        "value": value,
        "unit": "RHS*site*CG-iter/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.inner,
        "data": "synthetic",
        "config": {"workload": "gauge-16^4x3-nested: 16^4 torus, 3 colours, m2=0.05, eps=0.4, p=4, "
                               "nested distances 1,2,4,8 (finest level, 960 colours, 2880 diluted RHS "
                               "per step), Z2 complex noise, tol 1e-8",
                   "rhs_per_step": nrhs // a.steps, "rhs_block": W, "inner": a.inner,
                   "colours": [int(v) for v in ncols], "coloring_seconds": t_color},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                     "kernel": "k_stencil (q = A p, p^H q)", "launches": launches,
                     "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "time_to_trace_1e-3": tt,
        "plain_fp64_single_rhs": plain,
        "solve": {"rhs_iters": rhs_iters, "max_iters": max(r["solve"]["max_iters"] for r in res),
                  "reliable_updates": sum(r["solve"]["reliable_updates"] for r in res),
                  "max_true_resid": max(r["solve"]["max_true_resid"] for r in res)},
    }
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
