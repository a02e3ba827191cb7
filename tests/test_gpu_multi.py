"""One probe set, many displacements (Sec. 4.3) through the C ABI: the
probes of one (p0, k0) colouring are solved once and contracted with every
displacement n.  Parity with the oracle's trace for each n (same colouring,
same noise), the free-field closed form per n with an all-distinct colouring,
and identity with the single-displacement call."""
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


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("inner,tol", [("f64", 1e-10), ("f32", 1e-6)])
def test_trace_multi_matches_oracle(ctx, inner, tol):
    """8x4x4x4 x 3 gauge Laplacian (eps 0.4, links seed 3, m2 0.2), the
    (p0, k0) = (2, 2) colouring, diluted Z2-complex probes of two samples,
    contracted with n = -3, -1, 0, 1, 2, 3, 5."""
    _say("trace_multi vs oracle", inner)
    dims, nc, m2 = (8, 4, 4, 4), 3, 0.2
    U = workloads.random_links(dims, 0.4, 3, nc)
    col, m, _ = oracle.coloring(dims, 2, 2, oracle.NATURAL)
    ps = ctx.probe_spec(dims, nc, cuda(col), m, 5, 0, 2, "z2_complex", True)
    op = ctx.operator(dims, nc, m2, cuda(U))
    disps = [-3, -1, 0, 1, 2, 3, 5]
    res = ctx.trace_multi(op, ps, disps, ctx.opts(tol=1e-12 if inner == "f64" else 1e-10, inner=inner,
                                                  rhs_block=32))
    ors = [oracle.trace(dims, nc, m2, U, n, col, m, 5, 0, 2, oracle.Z2_COMPLEX, True, tol=1e-13) for n in disps]
    for r, o, n in zip(res, ors, disps):
        assert r["p"] == n
        # per displacement: relative to the size of the terms summed into
        # T_n (the far displacements have small traces made of large terms)
        scale = max(abs(o["T"]), 0.5 * np.abs(o["tj"]).sum() / 2)
        assert abs(r["T"] - o["T"]) < tol * scale, (n, r["T"], o["T"])
        assert np.abs(r["per_sample"] - o["per_sample"]).max() < tol * scale
        tscale = np.abs(o["tj"]).max()
        assert np.abs(r["tj"] - o["tj"]).max() < tol * tscale
    assert res[0]["solve"]["nconverged"] == res[0]["solve"]["nrhs"] == 2 * m * nc


def test_trace_multi_equals_single_displacement(ctx):
    """The contraction for n = p of the multi-displacement call is the one
    dp_trace_estimate computes (same solves, same kernels: bit-identical)."""
    _say("trace_multi == trace_estimate")
    w = workloads.GAUGE_8
    U = w.links()
    col, m, _ = oracle.coloring(w.dims, w.p, 4, oracle.BEST)
    ps = ctx.probe_spec(w.dims, 3, cuda(col), m, 0, 0, 1, "z2_complex", True)
    op = ctx.operator(w.dims, 3, w.m2, cuda(U))
    o = ctx.opts(tol=1e-10, inner="f32", rhs_block=64)
    single = ctx.trace_estimate([op], [ps], [w.p], o)[0]
    multi = ctx.trace_multi(op, ps, [0, w.p, 2 * w.p], o)
    assert multi[1]["T"] == single["T"]
    assert np.array_equal(multi[1]["tj"], single["tj"])


def test_trace_multi_free_field_closed_form(ctx):
    """4^4 free field, m2 = 0.5: with an all-distinct colouring (distance 8
    covers the 4^4 torus) every probe is one site, so the estimate of
    Tr(P_n A^{-1}) is exact for every n; it must equal the Fourier closed form
    sum_k cos(k0 n) / (m2 + sum_mu 4 sin^2(k_mu/2)) and be symmetric in n."""
    _say("trace_multi free field")
    dims, m2 = (4, 4, 4, 4), 0.5
    col, m, _ = oracle.coloring(dims, 0, 8, oracle.NATURAL)
    assert m == 256
    ps = ctx.probe_spec(dims, 1, cuda(col), m, 0, 0, 1, "real_z2", False)
    op = ctx.operator(dims, 1, m2, None)
    disps = [-2, -1, 0, 1, 2, 3, 4]
    res = ctx.trace_multi(op, ps, disps, ctx.opts(tol=1e-13, rhs_block=64))
    for r, n in zip(res, disps):
        exact, _ = workloads.free_field_trace(dims, m2, n)
        assert abs(r["T"] - exact) < 1e-11 * abs(exact), (n, r["T"], exact)
    T = {r["p"]: r["T"] for r in res}
    for n in (1, 2):
        assert abs(T[-n] - np.conj(T[n])) < 1e-12 * abs(T[n])
    # P_4 on a 4-periodic dimension is the identity: Tr(P_4 A^-1) = Tr(A^-1)
    assert abs(T[4] - T[0]) < 1e-12 * abs(T[0])


def test_variance_and_speedup_from_gpu_samples(ctx):
    """4^4 free field, m2 = 0.5, p = 1, the distance-2 colouring (8 colours),
    real Rademacher noise: the sample variance of 3000 probed samples from the
    GPU matches the exact per-sample variance sum_{i<j same colour}(B_ij+B_ji)^2
    = 0.674371 of B = P A^-1 (dense inverse, oracle operator), plain Hutchinson
    (one colour) matches 13.9477, and eq. (11)'s speed-up follows."""
    from paper_2106_01275_amd import analysis
    _say("variance from GPU samples")
    dims, m2 = (4, 4, 4, 4), 0.5
    A = oracle.dense(dims, 1, m2, None)
    Ainv = np.linalg.inv(A).real
    idx = np.arange(256)
    x0 = idx // 64
    shifted = ((x0 + 1) % 4) * 64 + idx % 64
    B = Ainv[shifted, :]  # (P A^-1)[x, y] = A^-1[x + e0, y]
    col, n, _ = oracle.coloring(dims, 1, 2, oracle.NATURAL)

    def exact_var(c):
        same = c[:, None] == c[None, :]
        return float(((B + B.T) ** 2 * np.triu(same, 1)).sum())

    v_probed_exact, v_plain_exact = exact_var(col), exact_var(np.zeros(256, np.int64))
    op = ctx.operator(dims, 1, m2, None)
    ns = 3000
    o = ctx.opts(tol=1e-12, rhs_block=64)
    ps = ctx.probe_spec(dims, 1, cuda(col), n, 11, 0, ns, "real_z2", False)
    r = ctx.trace_estimate([op], [ps], [1], o)[0]
    one = np.zeros(256, dtype=np.int32)
    ps1 = ctx.probe_spec(dims, 1, cuda(one), 1, 12, 0, ns, "real_z2", False)
    r1 = ctx.trace_estimate([op], [ps1], [1], o)[0]
    v_p = analysis.sample_variance(r["per_sample"])
    v_h = analysis.sample_variance(r1["per_sample"])
    rel = 5 * np.sqrt(2.0 / ns)  # 5 standard deviations of a variance estimate (Gaussian-like tails)
    assert abs(v_p / v_probed_exact - 1) < rel, (v_p, v_probed_exact)
    assert abs(v_h / v_plain_exact - 1) < 2 * rel, (v_h, v_plain_exact)
    exact_speedup = analysis.speedup_over_hutchinson(v_plain_exact, v_probed_exact, n)
    assert abs(analysis.speedup_over_hutchinson(v_h, v_p, n) / exact_speedup - 1) < 3 * rel
    # the estimate itself is unbiased: within 5 standard errors of the exact trace
    exact = np.trace(B)
    assert abs(r["T"] - exact) < 5 * np.sqrt(v_probed_exact / ns)


def test_trace_multi_rejects_bad_arguments(ctx):
    dims = (4, 4, 4, 4)
    col, m, _ = oracle.coloring(dims, 1, 1, oracle.NATURAL)
    ps = ctx.probe_spec(dims, 1, cuda(col), m, 0, 0, 1, "real_z2", False)
    op = ctx.operator(dims, 1, 0.5, None)
    with pytest.raises(dp.DPError):
        ctx.trace_multi(op, ps, [], ctx.opts())
    ps_bad = ctx.probe_spec((4, 4, 4, 2), 1, cuda(col[:128]), m, 0, 0, 1, "real_z2", False)
    with pytest.raises(dp.DPError):
        ctx.trace_multi(op, ps_bad, [0, 1], ctx.opts())
