"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: probes bit-exact; FP64 operator 1e-14, FP32 1e-6, BF16 1e-2
(relative, from the unit roundoff of the storage format times the few
operations per entry); FP64 solves and traces 1e-10 relative at CG tol
<= 1e-12; mixed precision 1e-6 relative after FP64 refinement.
"""
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


def cuda(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _probe_setup(ctx, dims, nc, p, k, order, seed, s0, ns, noise, dilute):
    col, n, _ = oracle.coloring(dims, p, k, {"natural": 0, "redblack": 1, "best": 2}[order])
    colg = cuda(col)
    ps = ctx.probe_spec(dims, nc, colg, n, seed, s0, ns, noise, dilute)
    return col, n, colg, ps


# ------------------------------------------------------------------ probes


@pytest.mark.parametrize("dims,nc,noise,dilute,p,k", [((4, 4, 4, 4), 1, "real_z2", False, 1, 2),
                                                      ((8, 8, 8, 8), 3, "z2_complex", True, 2, 4),
                                                      ((6, 4, 5, 3), 3, "z4", False, 1, 2),
                                                      ((5, 3, 4, 2), 3, "z4", True, 3, 1)])
def test_make_probes_bit_exact(ctx, dims, nc, noise, dilute, p, k):
    _say("probes", dims, nc, noise, dilute)
    col, n, colg, ps = _probe_setup(ctx, dims, nc, p, k, "natural", 12345, 2, 2, noise, dilute)
    kind = {"real_z2": 0, "z2_complex": 1, "z4": 2}[noise]
    want = oracle.probes(dims, nc, col, n, 12345, 2, 2, kind, dilute)
    got = ctx.make_probes(ps, 0, want.shape[0]).cpu().numpy()
    assert np.array_equal(got, want)
    # an offset window of the enumeration
    got2 = ctx.make_probes(ps, 3, 5).cpu().numpy()
    assert np.array_equal(got2, want[3:8])


# ------------------------------------------------------------------ operator


@pytest.mark.parametrize("prec,rtol", [("f64", 1e-14), ("f32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("dims,nc,links,nrhs", [((4, 4, 4, 4), 1, False, 3), ((4, 4, 4, 4), 3, True, 1),
                                                ((6, 4, 5, 3), 3, True, 17), ((4, 6, 2, 5), 3, True, 64),
                                                ((3, 4, 4, 5), 3, True, 100), ((5, 4, 3, 4), 1, True, 20),
                                                ((2, 2, 2, 2), 3, False, 5),
                                                # grouped-site stencils: x0 x x3 quads (two-slice
                                                # slabs, even D3, W = 32), x0 lines of four (slabs of
                                                # 4k slices: 32 x ...), x0 pairs (other even slabs)
                                                ((16, 4, 4, 4), 3, True, 32), ((16, 4, 4, 4), 1, False, 32),
                                                ((32, 4, 2, 2), 3, True, 32), ((32, 4, 2, 2), 1, False, 32),
                                                ((16, 2, 4, 3), 3, True, 16),
                                                ((16, 4, 2, 3), 3, True, 32),
                                                # one right-hand side: a site split over 32 threads
                                                ((4, 4, 4, 4), 1, False, 1), ((6, 4, 5, 3), 3, False, 1),
                                                ((5, 3, 4, 3), 1, True, 1), ((2, 2, 2, 2), 3, True, 1)])
def test_apply_matches_oracle(ctx, prec, rtol, dims, nc, links, nrhs):
    _say("apply", prec, dims, nc, links, nrhs)
    N = int(np.prod(dims))
    rng = np.random.default_rng(7)
    U = workloads.random_links(dims, 0.7, 3, nc) if links else None
    V = rng.standard_normal((nrhs, N, nc)) + 1j * rng.standard_normal((nrhs, N, nc))
    op = ctx.operator(dims, nc, 0.3, None if U is None else cuda(U))
    got = ctx.apply(op, cuda(V), prec).cpu().numpy()
    want = np.stack([oracle.apply(dims, nc, 0.3, U, v) for v in V])
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err < rtol, err


# ------------------------------------------------------------------ solves


@pytest.mark.parametrize("dims,nc,nrhs,block", [((4, 4, 4, 4), 3, 5, 0), ((6, 4, 5, 3), 3, 33, 16),
                                                ((4, 4, 4, 4), 1, 1, 1), ((3, 5, 4, 4), 3, 70, 64),
                                                ((8, 8, 8, 8), 3, 300, 256)])
def test_solve_batch_fp64_matches_oracle(ctx, dims, nc, nrhs, block):
    _say("solve f64", dims, nc, nrhs, block)
    N = int(np.prod(dims))
    rng = np.random.default_rng(11)
    U = workloads.random_links(dims, 0.5, 5, nc)
    B = rng.standard_normal((nrhs, N, nc)) + 1j * rng.standard_normal((nrhs, N, nc))
    op = ctx.operator(dims, nc, 0.2, cuda(U))
    (X,), (st,) = ctx.solve_batch([op], [cuda(B)], ctx.opts(tol=1e-12, rhs_block=block))
    Xo, it, rel = oracle.cg_many(dims, nc, 0.2, U, B, tol=1e-12)
    X = X.cpu().numpy()
    assert st["nconverged"] == nrhs and st["max_true_resid"] < 1e-11
    assert np.abs(X - Xo).max() < 1e-10 * np.abs(Xo).max()
    assert abs(st["max_iters"] - it.max()) <= 2


@pytest.mark.parametrize("inner,block", [("f32", 32), ("f32", 64), ("bf16", 64), ("f32", 128), ("f32", 256),
                                         ("bf16", 256)])
def test_solve_batch_mixed_matches_oracle(ctx, inner, block):
    _say("solve mixed", inner, block)
    dims, nc, nrhs = (6, 4, 5, 4), 3, 70
    N = int(np.prod(dims))
    rng = np.random.default_rng(12)
    U = workloads.random_links(dims, 0.4, 6, nc)
    B = rng.standard_normal((nrhs, N, nc)) + 1j * rng.standard_normal((nrhs, N, nc))
    op = ctx.operator(dims, nc, 0.1, cuda(U))
    (X,), (st,) = ctx.solve_batch([op], [cuda(B)], ctx.opts(tol=1e-10, inner=inner, rhs_block=block))
    Xo, it, rel = oracle.cg_many(dims, nc, 0.1, U, B, tol=1e-13)
    X = X.cpu().numpy()
    assert st["nconverged"] == nrhs and st["max_true_resid"] <= 1e-10
    assert st["reliable_updates"] >= 1
    err = np.abs(X - Xo).max() / np.abs(Xo).max()
    assert err < 1e-8, err


@pytest.mark.parametrize("inner,graph", [("f32", 0), ("f32", 1), ("bf16", 0), ("bf16", 1)])
def test_deferred_x_update_matches_oracle(ctx, monkeypatch, inner, graph):
    """Mixed precision takes the x updates of an iteration group in pairs (the
    first of a pair leaves x alone, the second recovers the skipped direction
    from p and r); DP_XDEFER=0 writes x at every update.  Both must reach the
    oracle's solution, take about as many iterations, and a lane whose beta
    is tiny (an eigenvector of the free field converges in one step) must
    update its x at once.  Eager launches and graph replay."""
    _say("deferred x update", inner, "graph", graph)
    dims, nc, nrhs = (8, 6, 4, 4), 3, 40
    N = int(np.prod(dims))
    rng = np.random.default_rng(31)
    B = rng.standard_normal((nrhs, N, nc)) + 1j * rng.standard_normal((nrhs, N, nc))
    B[3] = 1.0 + 0.5j  # constant: an eigenvector of the free-field operator
    Xo, it, rel = oracle.cg_many(dims, nc, 0.1, None, B, tol=1e-13)
    op = ctx.operator(dims, nc, 0.1, None)
    iters = {}
    for xd in ("1", "0"):
        monkeypatch.setenv("DP_XDEFER", xd)
        (X,), (st,) = ctx.solve_batch([op], [cuda(B)],
                                      ctx.opts(tol=1e-10, inner=inner, rhs_block=32, use_graph=graph))
        X = X.cpu().numpy()
        assert st["nconverged"] == nrhs and st["max_true_resid"] <= 1e-10, (xd, st)
        err = np.abs(X - Xo).max() / np.abs(Xo).max()
        assert err < 1e-8, (xd, err)
        assert np.abs(X[3] - Xo[3]).max() < 1e-9 * np.abs(Xo[3]).max(), xd
        iters[xd] = st["rhs_iters"]
    assert abs(iters["1"] - iters["0"]) <= 0.05 * iters["0"] + 2, iters


@pytest.mark.parametrize("inner", ["f32", "bf16"])
def test_deferred_x_update_every_stop(ctx, monkeypatch, inner):
    """Stopped after exactly k iterations (max_iter = k, k = 1..7: groups
    that end after an odd or an even number of updates), the iterate is the
    same with the x updates paired as with one x update per iteration, to
    the storage precision: no deferred step is lost or counted twice at a
    group's end."""
    _say("deferred x update at every stop", inner)
    dims, nc, nrhs = (6, 4, 5, 4), 3, 32
    N = int(np.prod(dims))
    rng = np.random.default_rng(41)
    U = workloads.random_links(dims, 0.4, 6, nc)
    B = rng.standard_normal((nrhs, N, nc)) + 1j * rng.standard_normal((nrhs, N, nc))
    op = ctx.operator(dims, nc, 0.1, cuda(U))
    rtol = 1e-5 if inner == "f32" else 5e-2
    for k in range(1, 8):
        xs = {}
        for xd in ("1", "0"):
            monkeypatch.setenv("DP_XDEFER", xd)
            (X,), (st,) = ctx.solve_batch([op], [cuda(B)],
                                          ctx.opts(tol=1e-14, max_iter=k, inner=inner, rhs_block=32), check=False)
            # (a BF16 lane that holds for its reliable update counts no iteration)
            assert st["max_iters"] == k if inner == "f32" else 0 < st["max_iters"] <= k, (k, xd, st)
            xs[xd] = X.cpu().numpy()
        err = np.abs(xs["1"] - xs["0"]).max() / np.abs(xs["0"]).max()
        assert err < rtol, (k, err)


def test_solve_empty_and_zero_rhs(ctx):
    dims, nc = (4, 4, 4, 4), 3
    op = ctx.operator(dims, nc, 0.5, None)
    B = torch.zeros((0, 256, 3), dtype=torch.complex128, device="cuda")
    (X,), (st,) = ctx.solve_batch([op], [B], ctx.opts(tol=1e-10))
    assert st["nrhs"] == 0
    B = torch.zeros((3, 256, 3), dtype=torch.complex128, device="cuda")
    (X,), (st,) = ctx.solve_batch([op], [B], ctx.opts(tol=1e-10))
    assert st["nconverged"] == 3 and torch.all(X == 0)


def test_solve_failure_statuses(ctx):
    dims = (4, 4, 4, 4)
    # not an eigenvector: a constant vector would converge in one step
    B = cuda(np.random.default_rng(2).standard_normal((2, 256, 1)).astype(np.complex128))
    op = ctx.operator(dims, 1, 0.5, None)
    (X,), (st,) = ctx.solve_batch([op], [B], ctx.opts(tol=1e-12, max_iter=1), check=False)
    assert st["nconverged"] == 0 and st["max_iters"] == 1
    with pytest.raises(dp.DPError) as e:
        ctx.solve_batch([op], [B], ctx.opts(tol=1e-12, max_iter=1))
    assert e.value.status == dp.ENOCONV
    bad = ctx.operator(dims, 1, -9.0, None)  # negative definite
    with pytest.raises(dp.DPError) as e:
        ctx.solve_batch([bad], [B], ctx.opts(tol=1e-12))
    assert e.value.status == dp.EBREAKDOWN
    for w in (3, 512, -4):  # not a power of two, above the largest width 256, negative
        with pytest.raises(dp.DPError) as e:
            ctx.solve_batch([op], [B], ctx.opts(tol=1e-12, rhs_block=w))
        assert e.value.status == dp.EINVAL
    with pytest.raises(dp.DPError) as e:
        ctx.solve_batch([ctx.operator((4, 4, 0, 4), 1, 0.5, None)], [B], ctx.opts(tol=1e-12))
    assert e.value.status == dp.EINVAL


def test_block_vectors_over_4gib_refused(ctx):
    """The stencil addresses a block vector through 32-bit byte offsets: a
    width whose vectors (N * nc * W elements of the inner precision) reach
    4 GiB is refused before anything is allocated (32^4 x 3 at W = 256:
    12.9 GB in FP64, 6.4 GB in FP32)."""
    dims = (32, 32, 32, 32)
    op = ctx.operator(dims, 3, 0.5, None)
    B = torch.zeros((1, 32 ** 4, 3), dtype=torch.complex128, device="cuda")
    B[0, 0, 0] = 1.0
    for inner in ("f64", "f32"):
        with pytest.raises(dp.DPError) as e:
            ctx.solve_batch([op], [B], ctx.opts(tol=1e-8, inner=inner, rhs_block=256))
        assert e.value.status == dp.EINVAL and "4 GiB" in str(e.value)


def test_binding_rejects_bad_sizes(ctx):
    """The kernels trust the sizes they are given: the binding checks every
    tensor's element count (and device) on the host before any call."""
    dims, c128 = (4, 4, 4, 4), torch.complex128
    with pytest.raises(ValueError):
        ctx.operator(dims, 3, 0.5, torch.zeros((4, 255, 3, 3), dtype=c128, device="cuda"))
    op = ctx.operator(dims, 1, 0.5, None)
    with pytest.raises(ValueError):
        ctx.solve_batch([op], [torch.zeros((2, 255, 1), dtype=c128, device="cuda")], ctx.opts(tol=1e-10))
    with pytest.raises(ValueError):
        ctx.probe_spec(dims, 1, torch.zeros(255, dtype=torch.int32, device="cuda"), 1, 0, 0, 1, "z2_complex", False)
    with pytest.raises(ValueError):
        ctx.apply(op, torch.zeros((1, 256, 3), dtype=c128, device="cuda"))


# ------------------------------------------------------------------ traces


def test_trace_free_field_4(ctx):
    """4^4 free field, m2 = 0.5, p = 1, distance-2 colouring (8 colours), real
    Rademacher probes from seed 0, CG tol 1e-12: the GPU estimate equals the
    oracle's; with one colour per site it equals the Fourier closed form."""
    _say("trace free 4^4")
    dims = (4, 4, 4, 4)
    col, n, colg, ps = _probe_setup(ctx, dims, 1, 1, 2, "best", 0, 0, 4, "real_z2", False)
    assert n == 8
    op = ctx.operator(dims, 1, 0.5, None)
    r = ctx.trace_estimate([op], [ps], [1], ctx.opts(tol=1e-12))[0]
    o = oracle.trace(dims, 1, 0.5, None, 1, col, n, 0, 0, 4, oracle.REAL_Z2, False, tol=1e-12)
    assert abs(r["T"] - o["T"]) < 1e-10 * abs(o["T"])
    assert np.abs(r["per_sample"] - o["per_sample"]).max() < 1e-10 * abs(o["T"])
    assert abs(r["stderr"] - o["stderr"]) < 1e-8 * o["stderr"]
    assert r["solve"]["max_iters"] <= 10
    exact, _ = workloads.free_field_trace(dims, 0.5, 1)
    alld = cuda(np.arange(256, dtype=np.int32))
    ps2 = ctx.probe_spec(dims, 1, alld, 256, 3, 0, 1, "real_z2", False)
    r2 = ctx.trace_estimate([op], [ps2], [1], ctx.opts(tol=1e-13))[0]
    assert abs(r2["T"] - exact) < 1e-11 * exact


@pytest.mark.parametrize("inner,block", [("f64", 1), ("f64", 64), ("f32", 64), ("bf16", 64)])
def test_trace_gauge_8(ctx, inner, block):
    """8^4 x 3 gauge Laplacian, eps = 0.3 (links seed 1), m2 = 0.1, p = 2,
    distance-4 colouring (best order: 64 colours), diluted Z2 complex noise,
    192 right-hand sides.  Plain FP64 single-RHS (W = 1), batched FP64 and
    mixed precision all agree with the oracle."""
    _say("trace gauge 8^4", inner, block)
    w = workloads.GAUGE_8
    U = w.links()
    col, n, colg, ps = _probe_setup(ctx, w.dims, 3, 2, 4, "best", 0, 0, 1, "z2_complex", True)
    assert n == 64
    op = ctx.operator(w.dims, 3, w.m2, cuda(U))
    r = ctx.trace_estimate([op], [ps], [2], ctx.opts(tol=1e-11, inner=inner, rhs_block=block))[0]
    o = _oracle_gauge8(col, n, U)
    tol = 1e-10 if inner == "f64" else 1e-6
    assert abs(r["T"] - o["T"]) < tol * abs(o["T"]), (r["T"], o["T"])
    scale = np.abs(o["tj"]).max()
    assert np.abs(r["tj"] - o["tj"]).max() < tol * scale
    assert r["solve"]["max_true_resid"] < 1e-10


def test_bf16_iterations_near_fp64(ctx):
    """BF16 storage with the default reliable-update drop (0.002) and held lanes
    converges in about as many iterations as FP64 CG on the same probes (a
    lane never iterates past what BF16 resolves)."""
    _say("bf16 iteration count vs fp64")
    w = workloads.GAUGE_8
    U = w.links()
    col, n, colg, ps = _probe_setup(ctx, w.dims, 3, 2, 4, "best", 0, 0, 1, "z2_complex", True)
    op = ctx.operator(w.dims, 3, w.m2, cuda(U))
    r = ctx.trace_estimate([op], [ps], [2], ctx.opts(tol=1e-8, inner="bf16", rhs_block=64))[0]
    B = oracle.probes(w.dims, 3, col, n, 0, 0, 1, oracle.Z2_COMPLEX, True)
    _, its, _ = oracle.cg_many(w.dims, 3, w.m2, U, B, tol=1e-8)
    st = r["solve"]
    assert st["nconverged"] == len(B) and st["max_true_resid"] <= 1e-8
    assert st["rhs_iters"] <= 1.25 * its.sum() + 2 * len(B), (st["rhs_iters"], its.sum())
    assert st["max_iters"] <= 1.5 * its.max() + 5, (st["max_iters"], its.max())


_GAUGE8 = {}


def _oracle_gauge8(col, n, U):
    if "r" not in _GAUGE8:
        w = workloads.GAUGE_8
        _GAUGE8["r"] = oracle.trace(w.dims, 3, w.m2, U, 2, col, n, 0, 0, 1, oracle.Z2_COMPLEX, True,
                                    tol=1e-12)
    return _GAUGE8["r"]


@pytest.mark.parametrize("dims,nc,p,k,noise,dilute,ns", [((4, 4, 4, 4), 3, 1, 2, "z4", False, 2),
                                                         ((6, 4, 5, 3), 3, 2, 1, "z2_complex", True, 1),
                                                         ((5, 4, 4, 4), 1, 0, 1, "real_z2", False, 3)])
def test_trace_small_cases(ctx, dims, nc, p, k, noise, dilute, ns):
    _say("trace small", dims, nc, p, k, noise)
    U = workloads.random_links(dims, 0.5, 9, nc)
    col, n, colg, ps = _probe_setup(ctx, dims, nc, p, k, "natural", 77, 1, ns, noise, dilute)
    op = ctx.operator(dims, nc, 0.25, cuda(U))
    r = ctx.trace_estimate([op], [ps], [p], ctx.opts(tol=1e-12))[0]
    kind = {"real_z2": 0, "z2_complex": 1, "z4": 2}[noise]
    o = oracle.trace(dims, nc, 0.25, U, p, col, n, 77, 1, ns, kind, dilute, tol=1e-12)
    assert abs(r["T"] - o["T"]) < 1e-10 * abs(o["T"])


def test_trace_single_colour_is_hutchinson(ctx):
    dims = (4, 4, 4, 4)
    col = np.zeros(256, dtype=np.int32)
    colg = cuda(col)
    ps = ctx.probe_spec(dims, 1, colg, 1, 5, 0, 6, "real_z2", False)
    op = ctx.operator(dims, 1, 0.5, None)
    r = ctx.trace_estimate([op], [ps], [1], ctx.opts(tol=1e-12))[0]
    o = oracle.trace(dims, 1, 0.5, None, 1, col, 1, 5, 0, 6, oracle.REAL_Z2, False, tol=1e-12)
    assert abs(r["T"] - o["T"]) < 1e-10 * abs(o["T"])


# ------------------------------------------------------------------ gradient


@pytest.mark.parametrize("dims,inner", [((4, 4, 4, 4), "f64"), ((2, 4, 2, 4), "f64"), ((4, 4, 4, 4), "f32")])
def test_trace_grad_matches_oracle(ctx, dims, inner):
    _say("grad", dims, inner)
    U = workloads.random_links(dims, 0.5, 3)
    col, n, colg, ps = _probe_setup(ctx, dims, 3, 1, 2, "natural", 17, 0, 2, "z2_complex", True)
    op = ctx.operator(dims, 3, 0.2, cuda(U))
    T, g, dU, dUb, st = ctx.trace_grad(op, ps, 1, ctx.opts(tol=1e-12 if inner == "f64" else 1e-11,
                                                           inner=inner))
    To, go, dUo, dUbo = oracle.trace_grad(dims, 3, 0.2, U, 1, col, n, 17, 0, 2, oracle.Z2_COMPLEX, True,
                                          tol=1e-13)
    tol = 1e-9 if inner == "f64" else 1e-6
    assert abs(T - To) < tol * abs(To)
    assert abs(g - go) < tol * abs(go)
    s = np.abs(dUo).max()
    assert np.abs(dU.cpu().numpy() - dUo).max() < tol * s
    assert np.abs(dUb.cpu().numpy() - dUbo).max() < tol * s


@pytest.mark.parametrize("nc", [3, 1])
def test_trace_grad_every_width(ctx, nc):
    """The force kernels at every kind of width: one thread per entry (W = 1,
    4), lanes summed inside a wavefront (W = 8, 32, 64) and across wavefronts
    (W = 128, 256), each against the oracle's gradient (FP64, 1e-9); the
    6x4x4x4 distance-2 colouring (6 colours, two samples) gives 36 (nc = 3)
    or 12 right-hand sides, so most widths end in a ragged or mostly empty
    block."""
    dims = (6, 4, 4, 4)
    _say("grad widths", nc)
    U = workloads.random_links(dims, 0.5, 4, nc)
    col, n, colg, ps = _probe_setup(ctx, dims, nc, 1, 2, "natural", 19, 0, 2, "z2_complex", True)
    op = ctx.operator(dims, nc, 0.25, cuda(U))
    To, go, dUo, dUbo = oracle.trace_grad(dims, nc, 0.25, U, 1, col, n, 19, 0, 2, oracle.Z2_COMPLEX, True,
                                          tol=1e-13)
    s = np.abs(dUo).max()
    for W in (1, 4, 8, 32, 64, 128, 256):
        T, g, dU, dUb, st = ctx.trace_grad(op, ps, 1, ctx.opts(tol=1e-12, inner="f64", rhs_block=W))
        assert st["rhs_block"] == W
        assert abs(g - go) < 1e-9 * abs(go), W
        assert np.abs(dU.cpu().numpy() - dUo).max() < 1e-9 * s, W
        assert np.abs(dUb.cpu().numpy() - dUbo).max() < 1e-9 * s, W


def test_grad_free_field_closed_form(ctx):
    """All-distinct colouring on the 4^4 free field: dT/dm2 equals the
    closed-form derivative -sum_k cos(k0 p)/lambda(k)^2."""
    dims = (4, 4, 4, 4)
    _, dexact = workloads.free_field_trace(dims, 0.5, 1)
    colg = cuda(np.arange(256, dtype=np.int32))
    ps = ctx.probe_spec(dims, 1, colg, 256, 1, 0, 1, "real_z2", False)
    op = ctx.operator(dims, 1, 0.5, None)
    T, g, _, _, _ = ctx.trace_grad(op, ps, 1, ctx.opts(tol=1e-13), want_links=False)
    assert abs(g.real - dexact) < 1e-10 * abs(dexact) and abs(g.imag) < 1e-12


def test_autograd_function_matches_finite_differences(ctx):
    """The torch.autograd.Function maps the Wirtinger pair to PyTorch's
    convention: check a real loss against central differences in m2 and
    along a random su(3) direction of the links."""
    dims = (2, 4, 2, 4)
    N = 64
    U0 = workloads.random_links(dims, 0.5, 8)
    col, n, _ = oracle.coloring(dims, 1, 2, 0)
    colg = cuda(col)
    opts = dp.Context.opts(tol=1e-13)
    m2 = torch.tensor(0.3, dtype=torch.float64, device="cuda", requires_grad=True)
    U = cuda(U0).requires_grad_(True)

    def loss(m2_, U_):
        T = dp.probed_trace(m2_, U_, dims, 3, 1, colg, n, seed=4, nsamples=1, noise="z2_complex",
                            dilute=True, opts=opts)
        return (T * (0.7 - 0.4j)).real + T.abs() ** 2 * 0.1

    L = loss(m2, U)
    L.backward()
    h = 1e-5
    with torch.no_grad():
        fd = (loss(m2 + h, U) - loss(m2 - h, U)) / (2 * h)
    assert abs(fd.item() - m2.grad.item()) < 1e-6 * max(1.0, abs(fd.item()))
    rng = np.random.default_rng(3)
    G = rng.standard_normal((4, N, 3, 3)) + 1j * rng.standard_normal((4, N, 3, 3))
    X = 0.5 * (G + np.conj(np.swapaxes(G, -1, -2)))
    w_, Q = np.linalg.eigh(X)

    def rot(t):
        E = (Q * np.exp(1j * t * w_)[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))
        return cuda(E @ U0)

    with torch.no_grad():
        fdU = (loss(m2, rot(h)) - loss(m2, rot(-h))).item() / (2 * h)
    dUdt = cuda(1j * X @ U0)
    an = torch.sum((U.grad.conj() * dUdt).real).item()  # PyTorch: dL = Re<grad, dU>
    assert abs(fdU - an) < 1e-6 * max(1.0, abs(fdU)), (fdU, an)


# ------------------------------------------------------------------ graphs


def test_graph_replay_matches_eager(ctx):
    """Iteration groups replayed from captured hipGraphs give bit-identical
    results to eager launches, on every replay, with eager work between."""
    dims, nc = (6, 4, 5, 4), 3
    U = workloads.random_links(dims, 0.4, 21, nc)
    col, n, colg, ps = _probe_setup(ctx, dims, nc, 1, 2, "natural", 5, 0, 2, "z2_complex", True)
    op = ctx.operator(dims, nc, 0.1, cuda(U))
    for inner in ("f64", "f32"):
        o_e = ctx.opts(tol=1e-10, inner=inner, rhs_block=32)
        o_g = ctx.opts(tol=1e-10, inner=inner, rhs_block=32, use_graph=1)
        ref = ctx.trace_estimate([op], [ps], [1], o_e)[0]
        for rep in range(3):
            g = ctx.trace_estimate([op], [ps], [1], o_g)[0]
            assert np.array_equal(g["tj"], ref["tj"]), (inner, rep)
            assert g["solve"]["rhs_iters"] == ref["solve"]["rhs_iters"]
            e = ctx.trace_estimate([op], [ps], [1], o_e)[0]  # eager work between replays
            assert np.array_equal(e["tj"], ref["tj"])
        B = ctx.make_probes(ps, 0, 40)
        (Xe,), _ = ctx.solve_batch([op], [B], o_e)
        (Xg,), _ = ctx.solve_batch([op], [B], o_g)
        assert torch.equal(Xe, Xg)


def test_graph_replay_two_solves_per_call(ctx):
    """A captured iteration group is replayed only with the kernel arguments
    it was captured with: the FP64 gradient (whose forward and adjoint solves
    write different solution buffers) and one call over two instances of
    different shapes and colour counts (solved one after the other) give
    bit-identical results with and without graph replay."""
    dims, nc = (6, 4, 5, 4), 3
    U = workloads.random_links(dims, 0.4, 22, nc)
    col, n, colg, ps = _probe_setup(ctx, dims, nc, 1, 2, "natural", 7, 0, 1, "z2_complex", True)
    op = ctx.operator(dims, nc, 0.1, cuda(U))
    o_e = ctx.opts(tol=1e-11, inner="f64", rhs_block=16)
    o_g = ctx.opts(tol=1e-11, inner="f64", rhs_block=16, use_graph=1)
    Te, ge, dUe, dUbe, _ = ctx.trace_grad(op, ps, 1, o_e)
    for rep in range(2):
        Tg, gg, dUg, dUbg, _ = ctx.trace_grad(op, ps, 1, o_g)
        assert Tg == Te and gg == ge, rep
        assert torch.equal(dUg, dUe) and torch.equal(dUbg, dUbe), rep
    # the FP64 gradient against the oracle as well (the graphs must not mix
    # the two solves' buffers)
    To, go, dUo, dUbo = oracle.trace_grad(dims, nc, 0.1, U, 1, col, n, 7, 0, 1, oracle.Z2_COMPLEX, True, tol=1e-12)
    assert abs(gg - go) < 1e-9 * abs(go)
    assert np.abs(dUg.cpu().numpy() - dUo).max() < 1e-9 * np.abs(dUo).max()
    # two instances that the multi-instance engine does not take together
    # (nc = 1 free field and nc = 3 with links): solved in turn in one call
    dims1 = (4, 4, 4, 4)
    col1, n1, colg1, ps1 = _probe_setup(ctx, dims1, 1, 1, 2, "natural", 3, 0, 2, "real_z2", False)
    op1 = ctx.operator(dims1, 1, 0.5)
    for inner in ("f64", "f32"):
        oe = ctx.opts(tol=1e-10, inner=inner, rhs_block=16)
        og = ctx.opts(tol=1e-10, inner=inner, rhs_block=16, use_graph=1)
        ref = ctx.trace_estimate([op, op1], [ps, ps1], [1, 1], oe)
        for rep in range(2):
            got = ctx.trace_estimate([op, op1], [ps, ps1], [1, 1], og)
            for i in range(2):
                assert np.array_equal(got[i]["tj"], ref[i]["tj"]), (inner, rep, i)
        o1 = oracle.trace(dims1, 1, 0.5, None, 1, col1, n1, 3, 0, 2, oracle.REAL_Z2, False, tol=1e-12)
        assert abs(got[1]["T"] - o1["T"]) < (1e-9 if inner == "f64" else 1e-6) * abs(o1["T"])


# ------------------------------------------------------------------ autotuner


def test_autotuned_width(ctx, tmp_path, monkeypatch):
    """rhs_block = 0 times candidate widths on the real kernels, caches the
    times (also in the DP_TUNE_CACHE file) and gives the same estimate as an
    explicit run at the chosen width."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("DP_TUNE_CACHE", str(cache))
    dims, nc = (8, 8, 8, 8), 3
    U = workloads.random_links(dims, 0.3, 1)
    col, n, colg, ps = _probe_setup(ctx, dims, nc, 2, 4, "best", 0, 0, 1, "z2_complex", True)
    op = ctx.operator(dims, nc, 0.1, cuda(U))
    c2 = dp.Context(0)  # fresh context: empty tuning cache
    r = c2.trace_estimate([op], [ps], [2], c2.opts(tol=1e-10, inner="f32", rhs_block=0))[0]
    W = r["solve"]["rhs_block"]
    assert W in (8, 16, 32, 64, 128, 256)
    assert f"width gfx950 dims=8x8x8x8 nc=3 prec=1 links=1 W={W}" in cache.read_text()
    r2 = c2.trace_estimate([op], [ps], [2], c2.opts(tol=1e-10, inner="f32", rhs_block=W))[0]
    assert np.array_equal(r["tj"], r2["tj"])
    c3 = dp.Context(0)  # a new context reads the cache file
    r3 = c3.trace_estimate([op], [ps], [2], c3.opts(tol=1e-10, inner="f32", rhs_block=0))[0]
    assert r3["solve"]["rhs_block"] == W
    c2.close()
    c3.close()


# ------------------------------------------------------------------ stencil launches


def _forced_context(monkeypatch, cfg):
    """A context whose stencil launches are forced to cfg = (mode,
    workgroups) (the DP_STENCIL variable is read at context creation)."""
    monkeypatch.setenv("DP_STENCIL", ",".join(str(v) for v in cfg))
    c = dp.Context(0)
    monkeypatch.delenv("DP_STENCIL")
    return c


@pytest.mark.parametrize("prec,rtol", [("f64", 1e-14), ("f32", 2e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("dims,nc,links,nrhs,modes", [
    # two-slice slabs (D0 = 16): pairs, quads; four-slice slabs (D0 = 32): lines
    ((16, 4, 4, 4), 3, True, 32, (0, 1, 3, 4)), ((32, 4, 4, 2), 3, True, 32, (0, 1, 3, 6)),
    ((16, 2, 4, 4), 1, False, 64, (0, 1, 2, 3, 4)), ((32, 2, 4, 2), 3, True, 16, (0, 1, 3)),
    # 360 sites: each XCD's 45 end in a part tile (the LDS copies of the
    # tiles ahead take site 0 for the missing ones)
    ((6, 4, 5, 3), 3, True, 32, (0, 1)), ((6, 4, 5, 3), 3, True, 16, (1,))])
def test_apply_every_stencil_mode(monkeypatch, prec, rtol, dims, nc, links, nrhs, modes):
    """Every stencil launch the tuner may pick gives the operator: each
    admissible mode (the BF16 grouped ones included), on a grid of 8 and of
    16 workgroups, against the oracle's operator."""
    _say("apply modes", prec, dims, nc, links, nrhs, modes)
    N = int(np.prod(dims))
    rng = np.random.default_rng(17)
    U = workloads.random_links(dims, 0.7, 4, nc) if links else None
    V = rng.standard_normal((nrhs, N, nc)) + 1j * rng.standard_normal((nrhs, N, nc))
    want = np.stack([oracle.apply(dims, nc, 0.3, U, v) for v in V])
    for mode in modes:
        for nblk in (8, 16):
            c = _forced_context(monkeypatch, (mode, nblk))
            op = c.operator(dims, nc, 0.3, None if U is None else cuda(U))
            got = c.apply(op, cuda(V), prec).cpu().numpy()
            c.close()
            err = np.abs(got - want).max() / np.abs(want).max()
            assert err < rtol, (mode, nblk, err)


def test_stencil_choice_solves(monkeypatch):
    """Solves through forced launches (FP32 lines on 16 workgroups; BF16
    pairs, whose grouped stencil sums r^H q and r^H p itself, and the BF16
    LDS tiles on 8) meet the oracle like the default launch."""
    dims, nc = (32, 4, 4, 2), 3
    U = workloads.random_links(dims, 0.4, 8, nc)
    col, n, _ = oracle.coloring(dims, 1, 2, oracle.NATURAL)
    o = oracle.trace(dims, nc, 0.1, U, 1, col, n, 2, 0, 1, oracle.Z2_COMPLEX, True, tol=1e-12)
    for cfg, inner in (((6, 16), "f32"), ((3, 16), "bf16"), ((1, 8), "bf16")):
        c = _forced_context(monkeypatch, cfg)
        colg = cuda(col)
        ps = c.probe_spec(dims, nc, colg, n, 2, 0, 1, "z2_complex", True)
        op = c.operator(dims, nc, 0.1, cuda(U))
        r = c.trace_estimate([op], [ps], [1], c.opts(tol=1e-10, inner=inner, rhs_block=32))[0]
        c.close()
        assert abs(r["T"] - o["T"]) < 1e-6 * abs(o["T"]), (cfg, inner, r["T"], o["T"])
        assert np.abs(r["tj"] - o["tj"]).max() < 1e-6 * np.abs(o["tj"]).max()
