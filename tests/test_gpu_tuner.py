"""The launch autotuner against explicit sweeps.

The stencil tuner (rhs_block given, DP_STENCIL unset) picks a stencil mode
and workgroup count per shape by timing CG iterations; here every candidate
it considers is forced in turn (DP_STENCIL=m,n) and timed
by the same solve, and the tuned choice must be within 6% of the fastest
(least of repeated timings of the finalists).  For a multi-instance batch the width
comes from a traffic model; it must be within 6% of the fastest of the
widths 16..128 timed one by one.
"""
import sys
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2106_01275_amd as dp  # noqa: E402

SLACK = 1.06


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _candidates(dims, W, inner):
    """The tuner's candidate launches (mode, workgroups) for a shape."""
    N = int(np.prod(dims))
    units = -(-N // (256 // W)) if W > 1 else max(-(-N // 256), -(-N // 8))
    base = units if units <= 8 else min(units, 1024) - min(units, 1024) % 8
    grids = [base] + [n for n in (256, 512, 1024, 2048) if n < units and n != base]
    out = []
    for n in grids:
        slabs = n >= 8 and n % 8 == 0 and dims[0] % 8 == 0
        n0 = dims[0] // 8
        valid = {0: True, 1: W >= 16, 2: W >= 64, 3: slabs and n0 % 2 == 0 and W >= 16,
                 4: slabs and n0 == 2 and dims[3] % 2 == 0 and W >= 32, 5: W == 1 and inner != "bf16",
                 6: slabs and n0 % 4 == 0 and W >= 32}
        out += [(mode, n) for mode in range(7) if valid[mode]]
    return out


def _rule_mode(dims, n, W, inner):
    """The library's built-in mode for a grid of n workgroups (kernels.hip's
    rule over the same validity as _candidates)."""
    slabs = n >= 8 and n % 8 == 0 and dims[0] % 8 == 0
    n0 = dims[0] // 8
    bf = inner == "bf16"
    if W == 1 and not bf:
        return 5
    if W >= 64:
        return 2
    if not bf and slabs and n0 == 2 and dims[3] % 2 == 0 and W >= 32:
        return 4
    if not bf and slabs and n0 % 4 == 0 and W >= 32:
        return 6
    if not bf and slabs and n0 % 2 == 0 and W >= 16:
        return 3
    return 1 if W >= 16 else 0


def _launch(cfg, dims, W, inner):
    """The launch a choice stands for: (-1, n) is the rule's mode on n
    workgroups, the same launch as (that mode, n)."""
    mode, n = cfg
    return (_rule_mode(dims, n, W, inner), n) if mode < 0 else (mode, n)


def _solve_time(c, op, B, inner, W, iters, reps):
    # exactly `iters` CG iterations: tol unreachable, no reliable update due
    o = c.opts(tol=1e-30, max_iter=iters, inner=inner, rhs_block=W, reliable_delta=1e-300)
    best = 1e30
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        c.solve_batch([op], [B], o, check=False)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def _iter_time(c, dims, nc, U, B, inner, W, reps=3):
    """Wall time of one CG iteration (stencil, finish, update): the least
    times of solves of 24 and of 8 iterations, differenced (operator
    set-up, initialisation, final residual and read-out cancel), after one
    untimed solve (which tunes, when the context tunes)."""
    op = c.operator(dims, nc, 0.05, U)
    _solve_time(c, op, B, inner, W, 8, 1)
    return (_solve_time(c, op, B, inner, W, 24, reps) - _solve_time(c, op, B, inner, W, 8, reps)) / 16


@pytest.mark.parametrize("dims", [(16, 16, 16, 16), (32, 32, 32, 32)])
def test_stencil_tuner_matches_sweep(monkeypatch, tmp_path, dims):
    """Every candidate launch timed once; then the tuned choice and the three
    fastest candidates timed again, round-robin in rotating order, six times
    each (the least time per CG iteration of each is compared)."""
    inner, W, nc = "f32", 32, 3
    N = int(np.prod(dims))
    rng = np.random.default_rng(3)
    # timing only: links need not be unitary
    U = torch.from_numpy(rng.standard_normal((4, N, nc, nc)) * 0.3 + 0j).cuda()
    B = torch.from_numpy(rng.standard_normal((W, N, nc)) + 1j * rng.standard_normal((W, N, nc))).cuda()
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("DP_TUNE_CACHE", str(cache))
    monkeypatch.delenv("DP_STENCIL", raising=False)
    ct = dp.Context(0)
    _iter_time(ct, dims, nc, U, B, inner, W, reps=1)
    ct.close()
    key = f"stencil gfx950 dims={'x'.join(map(str, dims))} nc={nc} prec=1 links=1 W={W}"
    text = cache.read_text()
    assert key in text
    tuned = tuple(int(v) for v in text.split(key)[1].split('"')[2].split(","))
    # the built-in choice is one of the explicit launches: time it as that
    # launch, in one context (two contexts running the same launch have
    # differed by up to 10%, which must not count against the tuner)
    tuned = _launch(tuned, dims, W, inner)
    monkeypatch.delenv("DP_TUNE_CACHE")

    def forced(cfg):
        monkeypatch.setenv("DP_STENCIL", ",".join(map(str, cfg)))
        c = dp.Context(0)
        monkeypatch.delenv("DP_STENCIL")
        return c

    times = {}
    for cfg in dict.fromkeys(_launch(c, dims, W, inner) for c in _candidates(dims, W, inner)):
        c = forced(cfg)
        times[cfg] = _iter_time(c, dims, nc, U, B, inner, W, reps=2)
        c.close()
    top = sorted(times, key=times.get)[:3]
    finalists = [tuned] + [t for t in top if t != tuned]
    runs = {cfg: [] for cfg in finalists}
    for rnd in range(6):
        # each finalist takes every position in the round in turn (the first
        # context of a round has run measurably slower), each timing in a
        # context of its own (a context kept over the rounds ran one launch
        # 10% slower than another context did, in all six rounds)
        k = rnd % len(finalists)
        for cfg in finalists[k:] + finalists[:k]:
            c = forced(cfg)
            runs[cfg].append(_iter_time(c, dims, nc, U, B, inner, W, reps=1))
            c.close()
    # the least time of each (the launch's own cost; slower rounds are
    # interference, which reached 9% between two contexts running the same
    # launch)
    low = {cfg: float(np.min(v)) for cfg, v in runs.items()}
    best = min(low, key=low.get)
    _say(dims, "tuned", tuned, "least ms per iteration", {k: round(v * 1e3, 3) for k, v in low.items()},
         "medians", {k: round(float(np.median(v)) * 1e3, 3) for k, v in runs.items()})
    assert low[tuned] <= SLACK * low[best], (tuned, low)


def test_width_tuner_pays_for_the_last_block():
    """96 right-hand sides on 16^4 (the count of one gradient solve): the
    tuned width against the widths 8..128 timed one by one on whole solves
    (a width of 64 solves 128 lanes, one of 32 solves 96)."""
    dims, nc, nrhs, inner = (16, 16, 16, 16), 3, 96, "f32"
    N = int(np.prod(dims))
    rng = np.random.default_rng(5)
    U = torch.from_numpy(workloads.random_links(dims, 0.5, 2)).cuda()
    B = torch.from_numpy(rng.standard_normal((nrhs, N, nc)) + 1j * rng.standard_normal((nrhs, N, nc))).cuda()
    c = dp.Context(0)
    op = c.operator(dims, nc, 0.05, U)

    def solve_time(W):
        o = c.opts(tol=1e-8, inner=inner, rhs_block=W)
        _, st = c.solve_batch([op], [B], o)
        best = 1e30
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            c.solve_batch([op], [B], o)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return best, st[0]["rhs_block"]

    t_tuned, W_tuned = solve_time(0)
    times = {W: solve_time(W)[0] for W in (8, 16, 32, 64, 128)}
    best = min(times, key=times.get)
    _say("96 RHS on 16^4: tuned", W_tuned, f"{t_tuned * 1e3:.2f} ms", "sweep",
         {k: round(v * 1e3, 2) for k, v in times.items()})
    assert t_tuned <= SLACK * times[best], (W_tuned, t_tuned, best, times[best])
    c.close()


def test_batch_width_model_matches_sweep():
    """The 64-instance uneven BF16 batch: the width of the traffic model
    (rhs_block = 0) against the widths 16, 32, 64, 128 timed one by one."""
    inst = workloads.uneven_batch()
    c = dp.Context(0)
    ops, specs = [], []
    for w in inst:
        col, m, _ = dp.build_coloring(w.dims, w.p, w.ks[0], w.order)
        ops.append(c.operator(w.dims, w.nc, w.m2, torch.from_numpy(w.links()).cuda()))
        specs.append(c.probe_spec(w.dims, w.nc, torch.from_numpy(np.ascontiguousarray(col)).cuda(), m,
                                  w.noise_seed, 0, 1, "z2_complex", True))
    ps = [w.p for w in inst]

    def step_time(W):
        o = c.opts(tol=1e-8, inner="bf16", rhs_block=W)
        r = c.trace_estimate(ops, specs, ps, o)
        best = 1e30
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            c.trace_estimate(ops, specs, ps, o)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return best, r[0]["solve"]["rhs_block"]

    t_model, W_model = step_time(0)
    times = {W: step_time(W)[0] for W in (16, 32, 64, 128)}
    best = min(times, key=times.get)
    _say("batch width: model", W_model, f"{t_model * 1e3:.1f} ms", "sweep",
         {k: round(v * 1e3, 1) for k, v in times.items()})
    assert t_model <= SLACK * times[best], (W_model, t_model, best, times[best])
    c.close()
