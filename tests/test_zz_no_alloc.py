"""dp_solve_noalloc (no device allocation: workspace in a static device
array) against dp_solve_batch, the entry point it is a variant of: the same
kernels at the same width give bit-identical solutions, and both meet the
oracle's FP64 solve (1e-10 FP64 at tol 1e-12, 1e-8 mixed precision at tol 1e-10).  Two
calls in a row, the second on a smaller input, so that the scratch array
holds the first call's contents when the second starts."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2106_01275_amd as dp  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return dp.context(0)


def _case(ctx, dims, nc, seed, nrhs, m2):
    U = workloads.random_links(dims, 0.3, seed, nc) if nc == 3 else None
    col, n, _ = oracle.coloring(dims, 1, 2, oracle.NATURAL)
    ps = ctx.probe_spec(dims, nc, torch.from_numpy(col).cuda(), n, seed, 0, 4, "z2_complex", True)
    B = ctx.make_probes(ps, 0, nrhs)
    op = ctx.operator(dims, nc, m2, None if U is None else torch.from_numpy(U).cuda())
    return U, B, op


@pytest.mark.parametrize("inner,rhs_block", [("f64", 16), ("f32", 32), ("bf16", 16), ("f32", 0)])
def test_noalloc_matches_solve_batch(ctx, inner, rhs_block):
    # FP64 to 1e-12 (solution within 1e-10 of the oracle's), mixed to 1e-10
    # (within 1e-8): the solution error is up to the condition number times
    # the relative residual
    tol = 1e-12 if inner == "f64" else 1e-10
    cases = [((6, 4, 6, 4), 3, 31, 45, 0.1), ((4, 4, 4, 2), 3, 32, 13, 0.2)]  # second call smaller
    for dims, nc, seed, nrhs, m2 in cases:
        _say("noalloc", inner, rhs_block, dims, nrhs)
        U, B, op = _case(ctx, dims, nc, seed, nrhs, m2)
        o = ctx.opts(tol=tol, inner=inner, rhs_block=rhs_block)
        Xn, sn = ctx.solve_noalloc(op, B, o)
        W = sn["rhs_block"]
        # solve_batch times the stencil launches of a new shape and keeps the
        # fastest; the no-alloc entry point never times (before that it takes
        # the built-in launch), but takes a choice the context already holds.
        # Called again after solve_batch, it runs the same launches, so the
        # two solutions must be bit-identical.
        (Xb,), (sb,) = ctx.solve_batch([op], [B], ctx.opts(tol=tol, inner=inner, rhs_block=W))
        err0 = (Xn - Xb).abs().max().item() / Xb.abs().max().item()
        assert err0 < (2e-10 if inner == "f64" else 2e-8), (inner, dims, err0)  # each within the oracle bar
        Xn, sn = ctx.solve_noalloc(op, B, o)
        torch.cuda.synchronize()
        assert torch.equal(Xn, Xb), (inner, dims)
        assert sn["rhs_iters"] == sb["rhs_iters"] and sn["nconverged"] == nrhs
        assert sn["max_true_resid"] <= tol
        # against the oracle's FP64 CG on a few right-hand sides
        Bh = B.cpu().numpy()
        for j in (0, nrhs // 2, nrhs - 1):
            xo, _, _ = oracle.cg(dims, nc, m2, U, Bh[j], tol=1e-13)
            err = np.abs(Xn[j].cpu().numpy().ravel() - xo.ravel()).max() / np.abs(xo).max()
            assert err < (1e-10 if inner == "f64" else 1e-8), (inner, j, err)


def test_noalloc_rejects_what_does_not_fit(ctx):
    """A lattice whose workspace exceeds the static array, and options that
    would allocate, are refused with DP_EINVAL before any device work."""
    dims = (16, 16, 16, 16)
    U = torch.zeros((4, 16 ** 4, 3, 3), dtype=torch.complex128, device="cuda")
    op = ctx.operator(dims, 3, 0.1, U)
    B = torch.zeros((1, 16 ** 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(dp.DPError) as e:
        ctx.solve_noalloc(op, B, ctx.opts(tol=1e-8, inner="f32", rhs_block=32))
    assert e.value.status == dp.EINVAL and "scratch" in str(e.value)
    dims = (4, 4, 4, 4)
    op = ctx.operator(dims, 1, 0.5)
    B = torch.ones((2, 256, 1), dtype=torch.complex128, device="cuda")
    for kw in ({"use_graph": 1}, {"profile": 1}):
        with pytest.raises(dp.DPError) as e:
            ctx.solve_noalloc(op, B, ctx.opts(tol=1e-8, rhs_block=2, **kw))
        assert e.value.status == dp.EINVAL
