"""Every nested level from the finest level's solves (dp_trace_levels,
Sec. 2.3), through the C ABI: each coarse level's estimate against the
oracle's direct estimate of that level (its own probes solved), the
per-solution terms against the oracle's reuse formula, the finest level equal
to dp_trace_estimate, an identity map equal to the finest level, and the
nesting check."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2106_01275_amd as dp  # noqa: E402

DIMS, NC, M2, P = (8, 4, 4, 4), 3, 0.2, 1


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return dp.context(0)


@pytest.fixture(scope="module")
def setup(ctx):
    U = workloads.random_links(DIMS, 0.4, 7, NC)
    cols, ncols = oracle.coloring_nested(DIMS, P, (1, 2, 4), oracle.NATURAL)
    colg = [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in cols]
    op = ctx.operator(DIMS, NC, M2, torch.from_numpy(U).cuda())
    ps = ctx.probe_spec(DIMS, NC, colg[-1], int(ncols[-1]), 9, 0, 2, "z2_complex", True)
    return U, cols, ncols, colg, op, ps


def test_levels_match_oracle(ctx, setup):
    _say("trace_levels vs oracle")
    U, cols, ncols, colg, op, ps = setup
    coarse = [(colg[0], int(ncols[0])), (colg[1], int(ncols[1]))]
    res = ctx.trace_levels(op, ps, P, coarse, ctx.opts(tol=1e-12, inner="f64", rhs_block=32))
    lev = oracle.trace_levels(DIMS, NC, M2, U, P, cols, ncols, 9, 0, 2, oracle.Z2_COMPLEX, True, tol=1e-13)
    for r, l in ((res[1], 0), (res[2], 1), (res[0], 2)):
        d = oracle.trace(DIMS, NC, M2, U, P, cols[l], int(ncols[l]), 9, 0, 2, oracle.Z2_COMPLEX, True, tol=1e-13)
        assert abs(r["T"] - d["T"]) < 1e-9 * abs(d["T"]), (l, r["T"], d["T"])
        assert np.abs(r["per_sample"] - d["per_sample"]).max() < 1e-9 * abs(d["T"])
        assert np.abs(r["tj"] - lev[l]["tj"]).max() < 1e-9 * np.abs(lev[l]["tj"]).max()
    nr = 2 * int(ncols[-1]) * NC
    assert res[0]["solve"]["nrhs"] == res[0]["solve"]["nconverged"] == nr


def test_finest_level_and_identity_map(ctx, setup):
    """out[0] is dp_trace_estimate's result (same solves and kernels,
    bit-identical); a coarse level equal to the finest colouring (identity
    map) gives the finest level's numbers exactly."""
    _say("trace_levels finest level and identity map")
    U, cols, ncols, colg, op, ps = setup
    o = ctx.opts(tol=1e-10, inner="f32", rhs_block=32)
    res = ctx.trace_levels(op, ps, P, [(colg[-1], int(ncols[-1]))], o)
    single = ctx.trace_estimate([op], [ps], [P], o)[0]
    assert res[0]["T"] == single["T"] and np.array_equal(res[0]["tj"], single["tj"])
    assert res[1]["T"] == res[0]["T"] and np.array_equal(res[1]["tj"], res[0]["tj"])
    assert len(ctx.trace_levels(op, ps, P, [], o)) == 1


def test_mixed_precision_levels(ctx, setup):
    """FP32 storage with FP64 reliable updates (tol 1e-10) against FP64: every
    level's estimate to 1e-6."""
    _say("trace_levels FP32 vs FP64")
    U, cols, ncols, colg, op, ps = setup
    coarse = [(colg[0], int(ncols[0])), (colg[1], int(ncols[1]))]
    r64 = ctx.trace_levels(op, ps, P, coarse, ctx.opts(tol=1e-12, inner="f64", rhs_block=32))
    r32 = ctx.trace_levels(op, ps, P, coarse, ctx.opts(tol=1e-10, inner="f32", rhs_block=32))
    for a, b in zip(r32, r64):
        assert abs(a["T"] - b["T"]) < 1e-6 * abs(b["T"])


def test_rejects_colourings_not_nested(ctx, setup):
    """A coarse colouring that splits a fine class, or a colour outside
    [0, ncolors), is refused before any solve."""
    _say("trace_levels nesting check")
    U, cols, ncols, colg, op, ps = setup
    o = ctx.opts(tol=1e-10, inner="f64", rhs_block=32)
    fine = cols[-1]
    c = int(np.argmax(np.bincount(fine)))  # a fine class of at least two sites
    x1, x2 = np.flatnonzero(fine == c)[:2]
    split = np.zeros_like(fine)
    split[x2] = 1  # puts x1 and x2 of one fine class in different coarse classes
    assert fine[x1] == fine[x2]
    split = torch.from_numpy(split).cuda()
    with pytest.raises(dp.DPError) as e:
        ctx.trace_levels(op, ps, P, [(split, 2)], o)
    assert e.value.status == dp.EINVAL
    big = colg[0].clone()
    big[5] = int(ncols[0])  # out of range
    with pytest.raises(dp.DPError) as e:
        ctx.trace_levels(op, ps, P, [(big, int(ncols[0]))], o)
    assert e.value.status == dp.EINVAL
