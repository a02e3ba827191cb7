"""Deflation (Sec. Deflation) through the C ABI: the device eigensolver
against the oracle's dense eigenpairs, the exact part Tr(P A^{-1} Q) against
the free-field closed form, the deflated estimate against the oracle's
(each side with its own vectors: the split is unique once the vectors span
an invariant subspace with a gap after it), the all-distinct-colour
identity, mixed precision against FP64, and at the 16^4 x 3 size the
eigen-residuals, orthonormality and the saving in CG iterations."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2106_01275_amd as dp  # noqa: E402

D4 = (4, 4, 4, 4)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return dp.context(0)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def gauge4():
    U = workloads.random_links(D4, 0.3, 1)
    w, V = oracle.lowest_eigenpairs(D4, 3, 0.1, U, 13)
    return U, w, V


def test_eigenpairs_match_dense(ctx, gauge4):
    """4^4 x 3 gauge Laplacian (eps 0.3, m2 0.1): the 12 lowest Ritz values
    and their span against numpy eigh of the dense operator."""
    _say("deflation eigenpairs 4^4x3 nvec 12")
    U, w, V = gauge4
    assert w[12] - w[11] > 1e-3  # a gap after the kept vectors
    op = ctx.operator(D4, 3, 0.1, cuda(U))
    d = ctx.deflation(op, 12, tol=1e-12, seed=3)
    assert d.subspace == 16 and d.outer > 0
    assert np.all(d.resid <= 1e-12)
    assert np.max(np.abs(d.evals - w[:12]) / w[:12]) < 1e-11
    Vg = d.vectors(D4, 3).cpu().numpy().reshape(12, -1)
    assert np.max(np.abs(Vg.conj() @ Vg.T - np.eye(12))) < 1e-10
    # same span: the singular values of V_dense^H V_gpu are all 1
    sv = np.linalg.svd(V.reshape(13, -1)[:12].conj() @ Vg.T, compute_uv=False)
    assert np.max(np.abs(sv - 1)) < 1e-9
    d.close()


def test_deflated_part_free_field_closed_form(ctx):
    """4^4 free field, m2 0.5, the lowest shell (9 modes): Tr(P A^{-1} Q) =
    1/m2 + 6/(m2 + 2) for p = 1, and 1/m2 + 8/(m2 + 2) for p = 0."""
    _say("deflation free field closed form")
    m2 = 0.5
    op = ctx.operator(D4, 1, m2, None)
    d = ctx.deflation(op, 9, tol=1e-12, seed=1)
    assert np.max(np.abs(d.evals - np.array([m2] + [m2 + 2] * 8))) < 1e-11
    col = torch.zeros(256, dtype=torch.int32, device="cuda")
    ps = ctx.probe_spec(D4, 1, col, 1, 3, 0, 2, "z2_complex", False)
    for p, ref in ((1, 1 / m2 + 6 / (m2 + 2)), (0, 1 / m2 + 8 / (m2 + 2))):
        r = ctx.trace_deflated(op, d, p, ps, ctx.opts(tol=1e-12, inner="f64", rhs_block=8))
        assert abs(r["T_defl"] - ref) < 1e-10 * ref
    d.close()


def test_all_distinct_colours_exact(ctx):
    """Every site its own colour: the deflated estimate is Tr(P A^{-1})
    exactly for any noise (4^4 free field, m2 0.5, p 1: the Fourier closed
    form 6.73722476756959)."""
    _say("deflation all-distinct identity")
    exact, _ = workloads.free_field_trace(D4, 0.5, 1)
    op = ctx.operator(D4, 1, 0.5, None)
    d = ctx.deflation(op, 9, tol=1e-12)
    col = torch.arange(256, dtype=torch.int32, device="cuda")
    ps = ctx.probe_spec(D4, 1, col, 256, 7, 0, 1, "z2_complex", False)
    r = ctx.trace_deflated(op, d, 1, ps, ctx.opts(tol=1e-12, inner="f64", rhs_block=64))
    assert abs(r["T"] - exact) < 1e-10 * exact
    d.close()


@pytest.mark.parametrize("p", [1, 2])
def test_deflated_trace_matches_oracle(ctx, gauge4, p):
    """Distance-2 colouring, diluted Z2-complex probes of two samples: the
    per-sample deflated estimates, T and Tr(P A^{-1} Q) against the oracle
    (FP64 CG to 1e-12 on both sides)."""
    _say("deflated trace vs oracle p", p)
    U, w, V = gauge4
    col, m, _ = oracle.coloring(D4, p, 2, oracle.NATURAL)
    op = ctx.operator(D4, 3, 0.1, cuda(U))
    d = ctx.deflation(op, 12, tol=1e-12, seed=2)
    ps = ctx.probe_spec(D4, 3, cuda(col), m, 9, 0, 2, "z2_complex", True)
    r = ctx.trace_deflated(op, d, p, ps, ctx.opts(tol=1e-12, inner="f64", rhs_block=16))
    o = oracle.trace_deflated(D4, 3, 0.1, U, p, col, m, 9, 0, 2, oracle.Z2_COMPLEX, True, V[:12])
    scale = abs(o["T"])
    assert abs(r["T_defl"] - o["T_defl"]) < 1e-9 * abs(o["T_defl"])
    assert abs(r["T"] - o["T"]) < 1e-8 * scale
    assert np.abs(r["per_sample"] - o["per_sample"]).max() < 1e-8 * scale
    assert np.abs(r["tj"] - o["tj"]).max() < 1e-8 * np.abs(o["tj"]).max()
    assert r["solve"]["nconverged"] == r["solve"]["nrhs"] == 2 * m * 3
    d.close()


@pytest.mark.parametrize("inner", ["f32", "bf16"])
def test_deflated_mixed_precision(ctx, gauge4, inner):
    """FP32 / BF16 storage with FP64 reliable updates against the FP64 solve
    of the same deflated right-hand sides (tol 1e-10): the estimate to 1e-7."""
    _say("deflated mixed precision", inner)
    U, _, _ = gauge4
    col, m, _ = oracle.coloring(D4, 1, 2, oracle.NATURAL)
    op = ctx.operator(D4, 3, 0.1, cuda(U))
    d = ctx.deflation(op, 12, tol=1e-12)
    ps = ctx.probe_spec(D4, 3, cuda(col), m, 4, 0, 1, "z2_complex", True)
    r64 = ctx.trace_deflated(op, d, 1, ps, ctx.opts(tol=1e-12, inner="f64", rhs_block=32))
    rlo = ctx.trace_deflated(op, d, 1, ps, ctx.opts(tol=1e-10, inner=inner, rhs_block=32))
    assert abs(rlo["T"] - r64["T"]) < 1e-7 * abs(r64["T"])
    assert rlo["solve"]["max_true_resid"] <= 1e-10
    d.close()


def test_wide_subspace_and_blocks(ctx, gauge4):
    """60 vectors (a 128-vector subspace: two 64-wide tiles in the Gram
    kernel) and 64-wide right-hand-side blocks: Ritz values against dense
    eigh, the deflated estimate against the oracle, and graph replay equal to
    the eager launches."""
    _say("deflation 60 vectors, W 64 blocks, graph replay")
    U, _, _ = gauge4
    w, V = oracle.lowest_eigenpairs(D4, 3, 0.1, U, 61)
    op = ctx.operator(D4, 3, 0.1, cuda(U))
    d = ctx.deflation(op, 60, tol=1e-11, seed=5)
    assert d.subspace == 128
    assert np.max(np.abs(d.evals - w[:60]) / w[:60]) < 1e-10
    col, m, _ = oracle.coloring(D4, 1, 2, oracle.NATURAL)
    ps = ctx.probe_spec(D4, 3, cuda(col), m, 6, 0, 2, "z2_complex", True)
    r = ctx.trace_deflated(op, d, 1, ps, ctx.opts(tol=1e-12, inner="f64", rhs_block=64))
    rg = ctx.trace_deflated(op, d, 1, ps, ctx.opts(tol=1e-12, inner="f64", rhs_block=64, use_graph=1))
    assert np.array_equal(r["tj"], rg["tj"])
    o = oracle.trace_deflated(D4, 3, 0.1, U, 1, col, m, 6, 0, 2, oracle.Z2_COMPLEX, True, V[:60])
    gap = (w[60] - w[59]) / w[59]
    tol = max(1e-8, 1e-11 / gap)
    assert abs(r["T_defl"] - o["T_defl"]) < tol * abs(o["T_defl"])
    assert np.abs(r["per_sample"] - o["per_sample"]).max() < tol * abs(o["T"])
    d.close()


def test_bad_arguments(ctx):
    op = ctx.operator(D4, 1, 0.5, None)
    for nvec in (0, 104):
        with pytest.raises(dp.DPError):
            ctx.deflation(op, nvec)
    d = ctx.deflation(op, 4, tol=1e-10)
    other = ctx.operator(D4, 1, 0.25, None)
    col = torch.zeros(256, dtype=torch.int32, device="cuda")
    ps = ctx.probe_spec(D4, 1, col, 1, 3, 0, 1, "z2_complex", False)
    with pytest.raises(dp.DPError):
        ctx.trace_deflated(other, d, 1, ps, ctx.opts(tol=1e-10))
    d.close()


def test_fullsize_16(ctx):
    """16^4 x 3 gauge Laplacian (m2 0.05, eps 0.4, links seed 1), 32 vectors:
    Ritz residuals <= 1e-8, orthonormal vectors, Ritz values inside
    [m2, m2 + 16] and ascending; the deflated right-hand sides of the
    distance-1 level (p 4, four samples, 36 right-hand sides) need fewer CG
    iterations than the plain probes, and the two estimates agree within their
    spread."""
    _say("deflation 16^4x3 nvec 32")
    dims, nc, m2 = (16, 16, 16, 16), 3, 0.05
    U = workloads.random_links(dims, 0.4, 1, nc)
    op = ctx.operator(dims, nc, m2, cuda(U))
    d = ctx.deflation(op, 32, tol=1e-8)
    assert np.all(d.resid <= 1e-8)
    assert np.all(np.diff(d.evals) >= -1e-12) and d.evals[0] >= m2 - 1e-9 and d.evals[-1] <= m2 + 16
    Vg = d.vectors(dims, nc).reshape(32, -1)
    G = (Vg.conj() @ Vg.T).cpu().numpy()
    assert np.max(np.abs(G - np.eye(32))) < 1e-9
    col, m, _ = dp.build_coloring(dims, 4, 1, "natural")
    ps = ctx.probe_spec(dims, nc, cuda(col), m, 0, 0, 4, "z2_complex", True)
    o = ctx.opts(tol=1e-8, inner="f32", rhs_block=32)
    rp = ctx.trace_estimate([op], [ps], [4], o)[0]
    rd = ctx.trace_deflated(op, d, 4, ps, o)
    _say("iterations plain", rp["solve"]["rhs_iters"], "deflated", rd["solve"]["rhs_iters"],
         "T", rp["T"], rd["T"], "stderr", rp["stderr"], rd["stderr"])
    _say("Ritz values", d.evals[:3], d.evals[-1], "outer", d.outer)
    assert rd["solve"]["rhs_iters"] < rp["solve"]["rhs_iters"]
    assert abs(rd["T"] - rp["T"]) < 6 * np.hypot(rp["stderr"], rd["stderr"])
    d.close()
