// extern "C" entry points of the dp library (declared in include/dp.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "context.h"

using namespace dp;

namespace {

thread_local std::string g_err;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

dp_status check_ctx(dp_ctx *ctx) {
    if (!ctx) {
        g_err = "null context";
        return DP_EINVAL;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->err = "hipSetDevice failed";
        return DP_EHIP;
    }
    return DP_OK;
}

dp_status solve_cfg(dp_ctx *ctx, const dp_solve_opts *o, SolveCfg &c) {
    if (!o) {
        ctx->err = "null solve options";
        return DP_EINVAL;
    }
    c.tol = o->tol;
    c.max_iter = o->max_iter > 0 ? o->max_iter : 100000;
    c.inner = o->inner;
    c.delta = o->reliable_delta > 0 ? o->reliable_delta : default_reliable_delta(c.inner);
    c.profile = o->profile;
    c.use_graph = o->use_graph;
    c.ru_gap = default_ru_gap(c.inner);
    if (!(c.tol > 0) || !(c.delta < 1)) {
        ctx->err = "tol must be > 0 and reliable_delta < 1";
        return DP_EINVAL;
    }
    if (c.inner != kF64 && c.inner != kF32 && c.inner != kBF16) {
        ctx->err = "unknown inner precision";
        return DP_EINVAL;
    }
    return DP_OK;
}

dp_status check_spec(dp_ctx *ctx, const dp_probe_spec &ps, const dp_operator *op) {
    for (int d = 0; d < 4; ++d)
        if (ps.dims[d] < 1 || (op && ps.dims[d] != op->dims[d])) {
            ctx->err = "probe spec dims invalid or not equal to the operator's";
            return DP_EINVAL;
        }
    if ((ps.nc != 1 && ps.nc != 3) || (op && ps.nc != op->nc)) {
        ctx->err = "probe spec nc invalid or not equal to the operator's";
        return DP_EINVAL;
    }
    if (!ps.colors_dev || ps.ncolors < 1 || ps.nsamples < 1 || ps.sample0 < 0 ||
        ps.noise < DP_NOISE_REAL_Z2 || ps.noise > DP_NOISE_Z4) {
        ctx->err = "probe spec: colors_dev, ncolors >= 1, nsamples >= 1, sample0 >= 0, noise kind";
        return DP_EINVAL;
    }
    return DP_OK;
}

ProbeGen make_gen(const dp_probe_spec &ps, long long rhs0, long long nvalid, int shift) {
    ProbeGen g{};
    g.colors = ps.colors_dev;
    g.seed = ps.seed;
    g.ncolors = ps.ncolors;
    g.sample0 = ps.sample0;
    g.noise = ps.noise;
    g.dilute = ps.dilute ? 1 : 0;
    g.rhs0 = rhs0;
    g.nvalid = nvalid;
    g.shift = shift;
    return g;
}

double noise_norm(int kind) { return kind == DP_NOISE_Z2_COMPLEX ? 0.5 : 1.0; }

dp_status batch_inst(dp_ctx *ctx, const dp_operator &op, BatchInst &I) {
    for (int d = 0; d < 4; ++d)
        if (op.dims[d] < 1) {
            ctx->err = "operator dims must be >= 1";
            return DP_EINVAL;
        }
    if (op.nc != 1 && op.nc != 3) {
        ctx->err = "operator nc must be 1 or 3";
        return DP_EINVAL;
    }
    const long long N = (long long)op.dims[0] * op.dims[1] * op.dims[2] * op.dims[3];
    if (N > (1LL << 30) / 8) {
        ctx->err = "lattice too large";
        return DP_EUNSUPPORTED;
    }
    if (!std::isfinite(op.m2)) {
        ctx->err = "m2 must be finite";
        return DP_EINVAL;
    }
    for (int d = 0; d < 4; ++d) I.lat.D[d] = op.dims[d];
    I.lat.N = (int)N;
    I.nc = op.nc;
    I.m2 = op.m2;
    I.links = op.links != nullptr;
    I.links_abi = op.links;
    return DP_OK;
}

// The multi-instance engine needs one nc and either links everywhere or nowhere.
bool batchable(int ninst, const dp_operator *ops) {
    if (ninst < 2) return false;
    for (int i = 1; i < ninst; ++i)
        if (ops[i].nc != ops[0].nc || (ops[i].links == nullptr) != (ops[0].links == nullptr)) return false;
    return true;
}

dp_status final_status(const dp_solve_stats &st) {
    if (st.nbreakdown > 0) return DP_EBREAKDOWN;
    if (st.nconverged < st.nrhs) return DP_ENOCONV;
    return DP_OK;
}

}  // namespace

// host-only colouring utilities: exceptions become status codes
template <typename F>
static dp_status host_call(const char *name, F f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        g_err = std::string(name) + ": out of host memory";
        return DP_ENOMEM;
    } catch (...) {
        g_err = std::string(name) + ": internal error";
        return DP_EINVAL;
    }
}

extern "C" {

dp_status dp_create(dp_ctx **out, int32_t hip_device) {
    if (!out) {
        g_err = "dp_create: null output";
        return DP_EINVAL;
    }
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
        g_err = "dp_create: no such HIP device";
        return DP_EHIP;
    }
    if (hipSetDevice(hip_device) != hipSuccess) {
        g_err = "dp_create: hipSetDevice failed";
        return DP_EHIP;
    }
    if (noalloc_attach(hip_device, g_err) != DP_OK) return DP_EHIP;
    dp_ctx *ctx = new (std::nothrow) dp_ctx();
    if (!ctx) {
        g_err = "dp_create: out of host memory";
        return DP_ENOMEM;
    }
    ctx->device = hip_device;
    // DP_STENCIL: unset or "tune" (time the stencil launches per shape),
    // "rule" (the built-in choice), or "m,n" (mode, workgroups)
    if (const char *e = std::getenv("DP_STENCIL")) {
        int m = -1, n = 0;
        if (std::strcmp(e, "rule") == 0) {
            ctx->stencil_policy = 1;
        } else if (std::sscanf(e, "%d,%d", &m, &n) == 2) {
            ctx->stencil_policy = 2;
            ctx->stencil_forced = {{m, n}};
        }
    }
    if (hipHostMalloc((void **)&ctx->ctrl_host, 64, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->state_host, state_bytes(), hipHostMallocDefault) != hipSuccess) {
        g_err = "dp_create: pinned allocation failed";
        dp_destroy(ctx);
        return DP_ENOMEM;
    }
    if (hipHostGetDevicePointer((void **)&ctx->ctrl_dev, ctx->ctrl_host, 0) != hipSuccess) {
        g_err = "dp_create: hipHostGetDevicePointer failed";
        dp_destroy(ctx);
        return DP_EHIP;
    }
    *out = ctx;
    return DP_OK;
}

void dp_destroy(dp_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (int s = 0; s < kNumSlots; ++s)
        if (ctx->slot[s]) (void)hipFree(ctx->slot[s]);
    for (auto &b : ctx->pool) (void)hipFree(b.first);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto &pr : ctx->ev_pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    ctx->drop_graphs();
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->ctrl_host) (void)hipHostFree(ctx->ctrl_host);
    if (ctx->state_host) (void)hipHostFree(ctx->state_host);
    delete ctx;
}

const char *dp_last_error(const dp_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

dp_status dp_build_coloring(const int32_t dims[4], int32_t p, const int32_t *ks, int32_t nlevels, int32_t order,
                            int32_t *colors, int32_t *ncolors, int32_t *order_used) {
    if (!dims) {
        g_err = "build_coloring: null dims";
        return DP_EINVAL;
    }
    try {
        return build_coloring(dims, p, ks, nlevels, order, colors, ncolors, order_used, g_err);
    } catch (const std::bad_alloc &) {
        g_err = "build_coloring: out of host memory";
        return DP_ENOMEM;
    } catch (...) {
        g_err = "build_coloring: internal error";
        return DP_EINVAL;
    }
}

dp_status dp_build_coloring_multi(const int32_t dims[4], const int32_t *disp, int32_t ndisp, const int32_t *ks,
                                  int32_t nlevels, int32_t order, int32_t *colors, int32_t *ncolors,
                                  int32_t *order_used) {
    if (!dims) {
        g_err = "build_coloring_multi: null dims";
        return DP_EINVAL;
    }
    return host_call("build_coloring_multi", [&] {
        return build_coloring_multi(dims, disp, ndisp, ks, nlevels, order, colors, ncolors, order_used, g_err);
    });
}

dp_status dp_tile_shape(const int32_t dims[4], int32_t p, int32_t k, int32_t tile[4]) {
    if (!dims || !tile || p < 0 || k < 0) {
        g_err = "tile_shape: bad arguments";
        return DP_EINVAL;
    }
    for (int d = 0; d < 4; ++d)
        if (dims[d] < 1) {
            g_err = "tile_shape: dims must be >= 1";
            return DP_EINVAL;
        }
    tile_shape(dims, p, k, tile);
    return DP_OK;
}

dp_status dp_build_coloring_tiled(const int32_t dims[4], int32_t p, int32_t k, int32_t order, int32_t *colors,
                                  int32_t *ncolors, int32_t *order_used, int32_t tile[4]) {
    if (!dims) {
        g_err = "build_coloring_tiled: null dims";
        return DP_EINVAL;
    }
    return host_call("build_coloring_tiled", [&] {
        return build_coloring_tiled(dims, p, k, order, colors, ncolors, order_used, tile, g_err);
    });
}

dp_status dp_clearance(const int32_t dims[4], const int32_t *colors, int32_t p, int32_t kmax, double *pct) {
    if (!dims) {
        g_err = "clearance: null dims";
        return DP_EINVAL;
    }
    return host_call("clearance", [&] { return clearance(dims, colors, p, kmax, pct, g_err); });
}

dp_status dp_make_probes(dp_ctx *ctx, const dp_probe_spec *ps, int64_t rhs0, int64_t nrhs, void *out,
                         hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!ps || (!out && nrhs > 0) || rhs0 < 0 || nrhs < 0) {
        ctx->err = "make_probes: bad arguments";
        return DP_EINVAL;
    }
    DP_TRY(check_spec(ctx, *ps, nullptr));
    if (nrhs == 0) return DP_OK;
    Lat lat{};
    long long N = 1;
    for (int d = 0; d < 4; ++d) {
        lat.D[d] = ps->dims[d];
        N *= ps->dims[d];
    }
    lat.N = (int)N;
    launch_make_probes_abi(lat, ps->nc, make_gen(*ps, rhs0, nrhs, 0), nrhs, (double *)out, stream);
    DP_HIP(hipGetLastError());
    return DP_OK;
}

dp_status dp_solve_batch(dp_ctx *ctx, int32_t ninst, const dp_operator *ops, const void *const *b, void *const *x,
                         const int64_t *nrhs, const dp_solve_opts *o, dp_solve_stats *st, hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (ninst < 1 || !ops || !b || !x || !nrhs) {
        ctx->err = "solve_batch: bad arguments";
        return DP_EINVAL;
    }
    SolveCfg cfg;
    DP_TRY(solve_cfg(ctx, o, cfg));
    WorkStream ws_;
    DP_TRY(ws_.enter(ctx, stream, cfg.use_graph));
    struct Leave {
        WorkStream &w;
        ~Leave() { (void)w.leave(); }
    } leave_{ws_};
    stream = ws_.s;
    dp_status worst = DP_OK;
    if (batchable(ninst, ops)) {
        const double t0 = now_s();
        std::vector<BatchInst> in(ninst);
        long long maxr = 0;
        for (int i = 0; i < ninst; ++i) {
            if (nrhs[i] < 0 || (nrhs[i] > 0 && (!b[i] || !x[i]))) {
                ctx->err = "solve_batch: bad right-hand sides";
                return DP_EINVAL;
            }
            DP_TRY(batch_inst(ctx, ops[i], in[i]));
            in[i].nrhs = nrhs[i];
            in[i].babi = (const double *)b[i];
            in[i].xabi = (double *)x[i];
            maxr = std::max<long long>(maxr, nrhs[i]);
        }
        int W = 1;
        {
            // the width is tuned on the largest instance
            int imax = 0;
            for (int i = 1; i < ninst; ++i)
                if ((long long)ops[i].dims[0] * ops[i].dims[1] * ops[i].dims[2] * ops[i].dims[3] >
                    (long long)ops[imax].dims[0] * ops[imax].dims[1] * ops[imax].dims[2] * ops[imax].dims[3])
                    imax = i;
            // (the width model reads the shape only: nothing is prepared)
            OpPrep opm;
            opm.lat = in[imax].lat;
            opm.nc = ops[imax].nc;
            opm.links = ops[imax].links != nullptr;
            opm.m2 = ops[imax].m2;
            opm.inner = cfg.inner;
            std::vector<std::pair<long long, long long>> work;
            for (auto &I : in) work.emplace_back(I.nrhs, (long long)I.lat.N);
            DP_TRY(choose_width(ctx, opm, cfg, maxr, o->rhs_block, stream, W, &work));
        }
        DP_TRY(run_batch(ctx, in, cfg, W, false, stream));
        for (int i = 0; i < ninst; ++i) {
            in[i].st.rhs_block = W;
            in[i].st.seconds = now_s() - t0;
            if (st) st[i] = in[i].st;
            dp_status fs = final_status(in[i].st);
            if (fs != DP_OK && worst == DP_OK) worst = fs;
        }
        if (worst == DP_ENOCONV) ctx->err = "solve_batch: some right-hand sides did not converge";
        if (worst == DP_EBREAKDOWN) ctx->err = "solve_batch: CG breakdown (operator not positive definite?)";
        return worst;
    }
    for (int i = 0; i < ninst; ++i) {
        const double t0 = now_s();
        dp_solve_stats s{};
        if (nrhs[i] < 0 || (nrhs[i] > 0 && (!b[i] || !x[i]))) {
            ctx->err = "solve_batch: bad right-hand sides";
            return DP_EINVAL;
        }
        OpPrep op;
        DP_TRY(prepare_operator(ctx, ops[i], cfg.inner, op, stream));
        int W = 1;
        DP_TRY(choose_width(ctx, op, cfg, nrhs[i], o->rhs_block, stream, W));
        s.rhs_block = W;
        Launch L;
        Red rd{};
        CgState cs{};
        DP_TRY(make_launch(ctx, op, W, stream, L, rd, cs, cfg));
        for (long long r0 = 0; r0 < nrhs[i]; r0 += W) {
            const long long nv = std::min<long long>(W, nrhs[i] - r0);
            BlockStats bs;
            bs.nvalid = (int)nv;
            InitAbi init{&L, cfg.inner, (const double *)b[i], r0, nv, &rd, &cs, ctx};
            double *x64 = (double *)ctx->at(kSlotX64);
            DP_TRY(solve_block(ctx, op, cfg, L, rd, cs, x64, init, bs, &s));
            launch_to_abi(L, x64, (double *)x[i], r0, nv);
            DP_HIP(hipGetLastError());
        }
        DP_HIP(hipStreamSynchronize(stream));
        s.seconds = now_s() - t0;
        if (st) st[i] = s;
        dp_status fs = final_status(s);
        if (fs != DP_OK && worst == DP_OK) worst = fs;
    }
    if (worst == DP_ENOCONV) ctx->err = "solve_batch: some right-hand sides did not converge";
    if (worst == DP_EBREAKDOWN) ctx->err = "solve_batch: CG breakdown (operator not positive definite?)";
    return worst;
}

// T_s, T and stderr from the per-right-hand-side contractions
static void combine(const dp_probe_spec &ps, const std::vector<double> &tj, dp_trace_result &out) {
    const int ndil = ps.dilute ? ps.nc : 1;
    const long long nrhs = (long long)ps.nsamples * ps.ncolors * ndil;
    const double norm = noise_norm(ps.noise);
    const long long per = (long long)ps.ncolors * ndil;
    std::vector<double> Ts(2 * ps.nsamples, 0.0);
    for (long long j = 0; j < nrhs; ++j) {
        Ts[2 * (j / per)] += norm * tj[2 * j];
        Ts[2 * (j / per) + 1] += norm * tj[2 * j + 1];
    }
    double Tr = 0, Ti = 0;
    for (int s_ = 0; s_ < ps.nsamples; ++s_) {
        Tr += Ts[2 * s_];
        Ti += Ts[2 * s_ + 1];
    }
    Tr /= ps.nsamples;
    Ti /= ps.nsamples;
    double var = 0;
    for (int s_ = 0; s_ < ps.nsamples; ++s_) {
        const double dr = Ts[2 * s_] - Tr, di = Ts[2 * s_ + 1] - Ti;
        var += dr * dr + di * di;
    }
    out.tr[0] = Tr;
    out.tr[1] = Ti;
    out.stderr_ = ps.nsamples > 1 ? std::sqrt(var / (ps.nsamples - 1) / ps.nsamples) : NAN;
    if (out.per_sample) std::memcpy(out.per_sample, Ts.data(), Ts.size() * sizeof(double));
    if (out.per_rhs) std::memcpy(out.per_rhs, tj.data(), tj.size() * sizeof(double));
}

// The probes of ps solved once; every solution contracted with each of the
// ndisp displacements (any sign).  outs[n] gets the estimate for disp[n].
// Pinned staging of a call's per-block results: every block's states (for
// its statistics) and its contractions are copied there in stream order and
// read after a synchronisation once per kChunk blocks (and at the end), so
// consecutive blocks follow each other on the device without a host round
// trip while the staging stays small.
struct Staging {
    static constexpr long long kChunk = 256;
    char *base = nullptr;
    size_t sb = 0, per_block = 0;
    int states = 1;
    long long chunk = 1;
    std::vector<BlockStats> bss;  // host-side counts (reliable updates) of the chunk's solves
    dp_status init(dp_ctx *ctx, long long nblocks, int states_per_block, size_t result_doubles_per_block) {
        sb = (state_bytes() + 255) / 256 * 256;
        states = states_per_block;
        per_block = result_doubles_per_block;
        chunk = std::max(1LL, std::min(nblocks, kChunk));
        bss.assign((size_t)chunk * states, BlockStats());
        return ctx->host_pinned((size_t)chunk * (states * sb + per_block * sizeof(double)), (void **)&base);
    }
    void *state(long long k, int i = 0) const { return base + ((size_t)(k % chunk) * states + i) * sb; }
    BlockStats &stats(long long k, int i, int nvalid) {
        BlockStats &b = bss[(size_t)(k % chunk) * states + i];
        if (nvalid >= 0) {
            b = BlockStats();
            b.nvalid = nvalid;
        }
        return b;
    }
    double *result(long long k) const {
        return (double *)(base + (size_t)chunk * states * sb) + (size_t)(k % chunk) * per_block;
    }
    bool drain_after(long long k, long long nblocks) const { return k % chunk == chunk - 1 || k == nblocks - 1; }
};

// colors[n], cmaps[n] (optional, per contraction): contract each solution
// with the probe of colour cmap[c] of the colouring colors[n] instead of its
// own (the parent class on a coarser nested level).
static dp_status trace_displacements(dp_ctx *ctx, const dp_operator &opd, const int32_t *disp, int ndisp,
                                     const dp_probe_spec &ps, const dp_solve_opts *o, const SolveCfg &cfg,
                                     dp_trace_result *outs, hipStream_t stream,
                                     const int32_t *const *colors = nullptr, const int *const *cmaps = nullptr) {
    const double t0 = now_s();
    DP_TRY(check_spec(ctx, ps, &opd));
    OpPrep op;
    DP_TRY(prepare_operator(ctx, opd, cfg.inner, op, stream));
    const int ndil = ps.dilute ? ps.nc : 1;
    const long long nrhs = (long long)ps.nsamples * ps.ncolors * ndil;
    int W = 1;
    DP_TRY(choose_width(ctx, op, cfg, nrhs, o->rhs_block, stream, W));
    Launch L;
    Red rd{};
    CgState cs{};
    DP_TRY(make_launch(ctx, op, W, stream, L, rd, cs, cfg));
    dp_solve_stats s{};
    s.rhs_block = W;
    const long long nblocks = (nrhs + W - 1) / W;
    Staging stg;
    DP_TRY(stg.init(ctx, nblocks, 1, (size_t)ndisp * 2 * W));
    std::vector<std::vector<double>> tj(ndisp, std::vector<double>(2 * nrhs, 0.0));
    long long k0 = 0;  // first block not yet drained
    for (long long k = 0; k < nblocks; ++k) {
        const long long r0 = k * W, nv = std::min<long long>(W, nrhs - r0);
        BlockStats &bs = stg.stats(k, 0, (int)nv);
        InitProbe init{&L, cfg.inner, make_gen(ps, r0, nv, 0), &rd, &cs, ctx};
        double *x64 = (double *)ctx->at(kSlotX64);
        DP_TRY(solve_block(ctx, op, cfg, L, rd, cs, x64, init, bs, &s, stg.state(k)));
        for (int n = 0; n < ndisp; ++n) {
            // each contraction reads x only at the probe's sites shifted by disp[n]
            ProbeGen g = make_gen(ps, r0, nv, 0);
            if (colors && colors[n]) g.colors = colors[n];
            if (cmaps) g.cmap = cmaps[n];
            launch_displaced_dot(L, g, disp[n], x64, rd, cs);
            DP_HIP(hipGetLastError());
            DP_HIP(hipMemcpyAsync(stg.result(k) + (size_t)n * 2 * W, cs.tj, 2 * nv * sizeof(double),
                                  hipMemcpyDeviceToHost, stream));
        }
        if (stg.drain_after(k, nblocks)) {
            DP_HIP(hipStreamSynchronize(stream));
            for (; k0 <= k; ++k0) {
                const long long b0 = k0 * W, bn = std::min<long long>(W, nrhs - b0);
                block_stats(stg.state(k0), stg.stats(k0, 0, -1), &s);
                for (int n = 0; n < ndisp; ++n)
                    std::memcpy(tj[n].data() + 2 * b0, stg.result(k0) + (size_t)n * 2 * W, 2 * bn * sizeof(double));
            }
        }
    }
    DP_TRY(finish_profile(ctx, &s));
    s.seconds = now_s() - t0;
    for (int n = 0; n < ndisp; ++n) {
        combine(ps, tj[n], outs[n]);
        outs[n].solve = s;
    }
    return final_status(s);
}

static dp_status trace_one(dp_ctx *ctx, const dp_operator &opd, int32_t p, const dp_probe_spec &ps,
                           const dp_solve_opts *o, const SolveCfg &cfg, dp_trace_result &out, hipStream_t stream) {
    if (p < 0) {
        ctx->err = "trace_estimate: p must be >= 0";
        return DP_EINVAL;
    }
    return trace_displacements(ctx, opd, &p, 1, ps, o, cfg, &out, stream);
}

dp_status dp_trace_estimate(dp_ctx *ctx, int32_t ninst, const dp_operator *ops, const int32_t *p,
                            const dp_probe_spec *ps, const dp_solve_opts *o, dp_trace_result *out,
                            hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (ninst < 1 || !ops || !p || !ps || !out) {
        ctx->err = "trace_estimate: bad arguments";
        return DP_EINVAL;
    }
    SolveCfg cfg;
    DP_TRY(solve_cfg(ctx, o, cfg));
    WorkStream ws_;
    DP_TRY(ws_.enter(ctx, stream, cfg.use_graph));
    struct Leave {
        WorkStream &w;
        ~Leave() { (void)w.leave(); }
    } leave_{ws_};
    stream = ws_.s;
    dp_status worst = DP_OK;
    if (batchable(ninst, ops)) {
        const double t0 = now_s();
        std::vector<BatchInst> in(ninst);
        long long maxr = 0;
        for (int i = 0; i < ninst; ++i) {
            DP_TRY(check_spec(ctx, ps[i], &ops[i]));
            if (p[i] < 0) {
                ctx->err = "trace_estimate: p must be >= 0";
                return DP_EINVAL;
            }
            DP_TRY(batch_inst(ctx, ops[i], in[i]));
            const int ndil = ps[i].dilute ? ps[i].nc : 1;
            in[i].nrhs = (long long)ps[i].nsamples * ps[i].ncolors * ndil;
            in[i].ps = ps[i];
            in[i].disp = p[i];
            in[i].tj.assign(2 * in[i].nrhs, 0.0);
            maxr = std::max<long long>(maxr, in[i].nrhs);
        }
        int W = 1;
        {
            // the width is tuned on the largest instance
            int imax = 0;
            for (int i = 1; i < ninst; ++i)
                if ((long long)ops[i].dims[0] * ops[i].dims[1] * ops[i].dims[2] * ops[i].dims[3] >
                    (long long)ops[imax].dims[0] * ops[imax].dims[1] * ops[imax].dims[2] * ops[imax].dims[3])
                    imax = i;
            // (the width model reads the shape only: nothing is prepared)
            OpPrep opm;
            opm.lat = in[imax].lat;
            opm.nc = ops[imax].nc;
            opm.links = ops[imax].links != nullptr;
            opm.m2 = ops[imax].m2;
            opm.inner = cfg.inner;
            std::vector<std::pair<long long, long long>> work;
            for (auto &I : in) work.emplace_back(I.nrhs, (long long)I.lat.N);
            DP_TRY(choose_width(ctx, opm, cfg, maxr, o->rhs_block, stream, W, &work));
        }
        DP_TRY(run_batch(ctx, in, cfg, W, true, stream));
        for (int i = 0; i < ninst; ++i) {
            combine(ps[i], in[i].tj, out[i]);
            in[i].st.rhs_block = W;
            in[i].st.seconds = now_s() - t0;
            out[i].solve = in[i].st;
            dp_status fs = final_status(in[i].st);
            if (fs != DP_OK && worst == DP_OK) worst = fs;
        }
        if (worst == DP_ENOCONV) ctx->err = "trace_estimate: some right-hand sides did not converge";
        if (worst == DP_EBREAKDOWN) ctx->err = "trace_estimate: CG breakdown";
        return worst;
    }
    for (int i = 0; i < ninst; ++i) {
        dp_status s = trace_one(ctx, ops[i], p[i], ps[i], o, cfg, out[i], stream);
        if (s == DP_EINVAL || s == DP_ENOMEM || s == DP_EHIP || s == DP_EUNSUPPORTED) return s;
        if (s != DP_OK && worst == DP_OK) worst = s;
    }
    if (worst == DP_ENOCONV) ctx->err = "trace_estimate: some right-hand sides did not converge";
    if (worst == DP_EBREAKDOWN) ctx->err = "trace_estimate: CG breakdown";
    return worst;
}

dp_status dp_trace_multi(dp_ctx *ctx, const dp_operator *op, const int32_t *disp, int32_t ndisp,
                         const dp_probe_spec *ps, const dp_solve_opts *o, dp_trace_result *out, hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!op || !disp || ndisp < 1 || !ps || !out) {
        ctx->err = "trace_multi: bad arguments";
        return DP_EINVAL;
    }
    SolveCfg cfg;
    DP_TRY(solve_cfg(ctx, o, cfg));
    WorkStream ws_;
    DP_TRY(ws_.enter(ctx, stream, cfg.use_graph));
    struct Leave {
        WorkStream &w;
        ~Leave() { (void)w.leave(); }
    } leave_{ws_};
    dp_status st = trace_displacements(ctx, *op, disp, ndisp, *ps, o, cfg, out, ws_.s);
    if (st == DP_ENOCONV) ctx->err = "trace_multi: some right-hand sides did not converge";
    if (st == DP_EBREAKDOWN) ctx->err = "trace_multi: CG breakdown";
    return st;
}

dp_status dp_trace_levels(dp_ctx *ctx, const dp_operator *op, int32_t p, const dp_probe_spec *ps, int32_t ncoarse,
                          const int32_t *const *coarse_colors, const int32_t *coarse_ncolors, const dp_solve_opts *o,
                          dp_trace_result *out, hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!op || !ps || !out || p < 0 || ncoarse < 0 || (ncoarse > 0 && (!coarse_colors || !coarse_ncolors))) {
        ctx->err = "trace_levels: bad arguments";
        return DP_EINVAL;
    }
    for (int l = 0; l < ncoarse; ++l)
        if (!coarse_colors[l] || coarse_ncolors[l] < 1) {
            ctx->err = "trace_levels: a coarse colouring is missing or has no colours";
            return DP_EINVAL;
        }
    SolveCfg cfg;
    DP_TRY(solve_cfg(ctx, o, cfg));
    DP_TRY(check_spec(ctx, *ps, op));
    WorkStream ws_;
    DP_TRY(ws_.enter(ctx, stream, cfg.use_graph));
    struct Leave {
        WorkStream &w;
        ~Leave() { (void)w.leave(); }
    } leave_{ws_};
    const int N = ps->dims[0] * ps->dims[1] * ps->dims[2] * ps->dims[3];
    const size_t nmap = (size_t)ncoarse * ps->ncolors;
    std::vector<const int32_t *> cols(ncoarse + 1, nullptr);
    std::vector<const int *> maps(ncoarse + 1, nullptr);
    if (ncoarse > 0) {
        // fine colour -> parent colour on each coarse level, checked nested
        DP_TRY(ctx->ensure(kSlotCmap, (nmap + ncoarse) * sizeof(int)));
        int *cm = (int *)ctx->at(kSlotCmap), *bad = cm + nmap;
        for (int l = 0; l < ncoarse; ++l)
            launch_level_map(N, ps->colors_dev, ps->ncolors, coarse_colors[l], coarse_ncolors[l],
                             cm + (size_t)l * ps->ncolors, bad + l, ws_.s);
        DP_HIP(hipGetLastError());
        std::vector<int> hbad(ncoarse, 0);
        DP_HIP(hipMemcpyAsync(hbad.data(), bad, ncoarse * sizeof(int), hipMemcpyDeviceToHost, ws_.s));
        DP_HIP(hipStreamSynchronize(ws_.s));
        for (int l = 0; l < ncoarse; ++l) {
            if (hbad[l]) {
                ctx->err = "trace_levels: coarse colouring " + std::to_string(l) +
                           " is not nested in the fine one, or a colour is out of range";
                return DP_EINVAL;
            }
            cols[l + 1] = coarse_colors[l];
            maps[l + 1] = cm + (size_t)l * ps->ncolors;
        }
    }
    std::vector<int32_t> disp(ncoarse + 1, p);
    dp_status st = trace_displacements(ctx, *op, disp.data(), ncoarse + 1, *ps, o, cfg, out, ws_.s, cols.data(),
                                       maps.data());
    if (st == DP_ENOCONV) ctx->err = "trace_levels: some right-hand sides did not converge";
    if (st == DP_EBREAKDOWN) ctx->err = "trace_levels: CG breakdown";
    return st;
}

dp_status dp_trace_grad(dp_ctx *ctx, const dp_operator *opd, int32_t p, const dp_probe_spec *ps,
                        const dp_solve_opts *o, dp_trace_result *out, double dT_dm2[2], void *dT_dU,
                        void *dT_dUbar, hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!opd || !ps || !out || !dT_dm2 || p < 0) {
        ctx->err = "trace_grad: bad arguments";
        return DP_EINVAL;
    }
    const double t0 = now_s();
    SolveCfg cfg;
    DP_TRY(solve_cfg(ctx, o, cfg));
    DP_TRY(check_spec(ctx, *ps, opd));
    WorkStream ws_;
    DP_TRY(ws_.enter(ctx, stream, cfg.use_graph));
    struct Leave {
        WorkStream &w;
        ~Leave() { (void)w.leave(); }
    } leave_{ws_};
    stream = ws_.s;

    OpPrep op;
    DP_TRY(prepare_operator(ctx, *opd, cfg.inner, op, stream));
    const int ndil = ps->dilute ? ps->nc : 1;
    const long long nrhs = (long long)ps->nsamples * ps->ncolors * ndil;
    int W = 1;
    DP_TRY(choose_width(ctx, op, cfg, nrhs, o->rhs_block, stream, W));
    Launch L;
    Red rd{};
    CgState cs{};
    DP_TRY(make_launch(ctx, op, W, stream, L, rd, cs, cfg));
    DP_TRY(ctx->ensure(kSlotX64b, (size_t)op.lat.N * op.nc * W * 16));
    double *xsol = (double *)ctx->at(kSlotX64b);
    double *lsol = (double *)ctx->at(kSlotX64);
    const double norm = noise_norm(ps->noise) / ps->nsamples;
    dp_solve_stats s{};
    s.rhs_block = W;
    const long long nblocks = (nrhs + W - 1) / W;
    Staging stg;
    DP_TRY(stg.init(ctx, nblocks, 2, 4 * (size_t)W));
    std::vector<double> tj(2 * nrhs, 0.0), lx(2 * nrhs, 0.0);
    long long k0 = 0;  // first block not yet drained
    for (long long k = 0; k < nblocks; ++k) {
        const long long r0 = k * W, nv = std::min<long long>(W, nrhs - r0);
        BlockStats &bs1 = stg.stats(k, 0, (int)nv), &bs2 = stg.stats(k, 1, (int)nv);
        InitProbe ix{&L, cfg.inner, make_gen(*ps, r0, nv, 0), &rd, &cs, ctx};
        DP_TRY(solve_block(ctx, op, cfg, L, rd, cs, xsol, ix, bs1, &s, stg.state(k, 0)));
        launch_displaced_dot(L, make_gen(*ps, r0, nv, 0), p, xsol, rd, cs);
        DP_HIP(hipMemcpyAsync(stg.result(k), cs.tj, 2 * nv * sizeof(double), hipMemcpyDeviceToHost, stream));
        InitProbe il{&L, cfg.inner, make_gen(*ps, r0, nv, p), &rd, &cs, ctx};
        DP_TRY(solve_block(ctx, op, cfg, L, rd, cs, lsol, il, bs2, &s, stg.state(k, 1)));
        launch_dot(L, lsol, xsol, rd, cs);
        DP_HIP(hipMemcpyAsync(stg.result(k) + 2 * W, cs.tj, 2 * nv * sizeof(double), hipMemcpyDeviceToHost,
                              stream));
        if (dT_dU || dT_dUbar)
            launch_force(L, xsol, lsol, op.nbr, norm, r0 == 0, (double *)dT_dU, (double *)dT_dUbar);
        DP_HIP(hipGetLastError());
        if (stg.drain_after(k, nblocks)) {
            DP_HIP(hipStreamSynchronize(stream));
            for (; k0 <= k; ++k0) {
                const long long b0 = k0 * W, bn = std::min<long long>(W, nrhs - b0);
                for (int i = 0; i < 2; ++i) block_stats(stg.state(k0, i), stg.stats(k0, i, -1), &s);
                std::memcpy(tj.data() + 2 * b0, stg.result(k0), 2 * bn * sizeof(double));
                std::memcpy(lx.data() + 2 * b0, stg.result(k0) + 2 * W, 2 * bn * sizeof(double));
            }
        }
    }
    DP_TRY(finish_profile(ctx, &s));
    double Tr = 0, Ti = 0, gr = 0, gi = 0;
    for (long long j = 0; j < nrhs; ++j) {
        Tr += tj[2 * j];
        Ti += tj[2 * j + 1];
        gr += lx[2 * j];
        gi += lx[2 * j + 1];
    }
    out->tr[0] = norm * Tr;
    out->tr[1] = norm * Ti;
    out->stderr_ = NAN;
    if (out->per_rhs) std::memcpy(out->per_rhs, tj.data(), tj.size() * sizeof(double));
    dT_dm2[0] = -norm * gr;
    dT_dm2[1] = -norm * gi;
    s.seconds = now_s() - t0;
    out->solve = s;
    dp_status fs = final_status(s);
    if (fs == DP_ENOCONV) ctx->err = "trace_grad: some right-hand sides did not converge";
    if (fs == DP_EBREAKDOWN) ctx->err = "trace_grad: CG breakdown";
    return fs;
}

dp_status dp_apply(dp_ctx *ctx, const dp_operator *opd, int32_t prec, const void *v, void *y, int64_t nrhs,
                   hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!opd || nrhs < 0 || (nrhs > 0 && (!v || !y))) {
        ctx->err = "apply: bad arguments";
        return DP_EINVAL;
    }
    if (nrhs == 0) return DP_OK;
    OpPrep op;
    DP_TRY(prepare_operator(ctx, *opd, prec, op, stream));
    SolveCfg cfg;
    cfg.inner = prec;
    int W = 1;
    while (W < nrhs && W < 64) W *= 2;
    Launch L;
    Red rd{};
    CgState cs{};
    DP_TRY(make_launch(ctx, op, W, stream, L, rd, cs, cfg));
    for (long long r0 = 0; r0 < nrhs; r0 += W) {
        const long long nv = std::min<long long>(W, nrhs - r0);
        launch_abi_to_internal(L, prec, (const double *)v, r0, nv, ctx->at(kSlotP));
        StencilArgs sa;
        sa.links = op.links;
        sa.diag = op.m2 + 8.0;
        sa.pin = ctx->at(kSlotP);
        sa.q = ctx->at(kSlotQ);
        sa.U = op.U8;
        sa.nbr = op.nbr;
        launch_stencil(L, prec, sa);
        launch_internal_to_abi_prec(L, prec, ctx->at(kSlotQ), (double *)y, r0, nv);
        DP_HIP(hipGetLastError());
    }
    DP_HIP(hipStreamSynchronize(stream));
    return DP_OK;
}

// ------------------------------------------------------------ deflation

dp_status dp_deflation_create(dp_ctx *ctx, const dp_operator *op, int32_t nvec, const dp_eig_opts *o,
                              dp_deflation **out, hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!op || !out) {
        ctx->err = "deflation_create: bad arguments";
        return DP_EINVAL;
    }
    *out = nullptr;
    dp_eig_opts eo{};
    if (o) eo = *o;
    if (eo.degree < 0 || eo.max_outer < 0 || !(eo.tol >= 0) || eo.degree > 200) {
        ctx->err = "deflation_create: bad options";
        return DP_EINVAL;
    }
    dp_deflation *d = new dp_deflation;
    d->device = ctx->device;
    const dp_status st = deflation_build(ctx, *op, nvec, eo, *d, stream);
    if (st != DP_OK && st != DP_ENOCONV) {
        dp_deflation_destroy(d);
        return st;
    }
    if (st == DP_ENOCONV) ctx->err = "deflation_create: Ritz residuals above tol after max_outer iterations";
    *out = d;
    return st;
}

dp_status dp_deflation_info(const dp_deflation *d, double *evals, double *resid, int32_t *outer,
                            int32_t *subspace) {
    if (!d) return DP_EINVAL;
    if (evals) std::memcpy(evals, d->theta.data(), d->theta.size() * sizeof(double));
    if (resid) std::memcpy(resid, d->resid.data(), d->resid.size() * sizeof(double));
    if (outer) *outer = d->outer;
    if (subspace) *subspace = d->W;
    return DP_OK;
}

dp_status dp_deflation_vectors(dp_ctx *ctx, const dp_deflation *d, void *out, hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!d || !out) {
        ctx->err = "deflation_vectors: bad arguments";
        return DP_EINVAL;
    }
    if (d->device != ctx->device) {
        ctx->err = "deflation_vectors: the deflation lives on another device than the context";
        return DP_EINVAL;
    }
    return deflation_vectors(ctx, *d, (double *)out, stream);
}

void dp_deflation_destroy(dp_deflation *d) {
    if (!d) return;
    (void)hipSetDevice(d->device);
    if (d->V) (void)hipFree(d->V);
    if (d->Z) (void)hipFree(d->Z);
    if (d->scratch) (void)hipFree(d->scratch);
    delete d;
}

dp_status dp_trace_deflated(dp_ctx *ctx, const dp_operator *opd, const dp_deflation *d, int32_t p,
                            const dp_probe_spec *ps, const dp_solve_opts *o, dp_trace_result *out,
                            double tr_defl[2], hipStream_t stream) {
    DP_TRY(check_ctx(ctx));
    if (!opd || !d || !ps || !out || p < 0) {
        ctx->err = "trace_deflated: bad arguments";
        return DP_EINVAL;
    }
    bool same = opd->nc == d->nc && opd->m2 == d->m2 && (opd->links != nullptr) == d->links;
    for (int k = 0; k < 4; ++k) same = same && opd->dims[k] == d->lat.D[k];
    if (!same) {
        ctx->err = "trace_deflated: the deflation was built for another operator";
        return DP_EINVAL;
    }
    if (d->device != ctx->device) {
        ctx->err = "trace_deflated: the deflation lives on another device than the context";
        return DP_EINVAL;
    }
    const double t0 = now_s();
    SolveCfg cfg;
    DP_TRY(solve_cfg(ctx, o, cfg));
    DP_TRY(check_spec(ctx, *ps, opd));
    WorkStream ws_;
    DP_TRY(ws_.enter(ctx, stream, cfg.use_graph));
    struct Leave {
        WorkStream &w;
        ~Leave() { (void)w.leave(); }
    } leave_{ws_};
    stream = ws_.s;
    double td[2] = {0.0, 0.0};
    DP_TRY(deflation_trace_part(ctx, *d, p, stream, td));
    OpPrep op;
    DP_TRY(prepare_operator(ctx, *opd, cfg.inner, op, stream));
    const int ndil = ps->dilute ? ps->nc : 1;
    const long long nrhs = (long long)ps->nsamples * ps->ncolors * ndil;
    int W = 1;
    DP_TRY(choose_width(ctx, op, cfg, nrhs, o->rhs_block, stream, W));
    Launch L;
    Red rd{};
    CgState cs{};
    DP_TRY(make_launch(ctx, op, W, stream, L, rd, cs, cfg));
    dp_solve_stats s{};
    s.rhs_block = W;
    const long long nblocks = (nrhs + W - 1) / W;
    Staging stg;
    DP_TRY(stg.init(ctx, nblocks, 1, 2 * (size_t)W));
    std::vector<double> tj(2 * nrhs, 0.0);
    dp_status proj = DP_OK;
    long long k0 = 0;  // first block not yet drained
    for (long long k = 0; k < nblocks; ++k) {
        const long long r0 = k * W, nv = std::min<long long>(W, nrhs - r0);
        BlockStats &bs = stg.stats(k, 0, (int)nv);
        InitDeflated init{&L, cfg.inner, make_gen(*ps, r0, nv, 0), &rd, &cs, ctx, d, &proj};
        double *x64 = (double *)ctx->at(kSlotX64);
        DP_TRY(solve_block(ctx, op, cfg, L, rd, cs, x64, init, bs, &s, stg.state(k)));
        DP_TRY(proj);
        launch_displaced_dot(L, make_gen(*ps, r0, nv, 0), p, x64, rd, cs);
        DP_HIP(hipGetLastError());
        DP_HIP(hipMemcpyAsync(stg.result(k), cs.tj, 2 * nv * sizeof(double), hipMemcpyDeviceToHost, stream));
        if (stg.drain_after(k, nblocks)) {
            DP_HIP(hipStreamSynchronize(stream));
            for (; k0 <= k; ++k0) {
                const long long b0 = k0 * W, bn = std::min<long long>(W, nrhs - b0);
                block_stats(stg.state(k0), stg.stats(k0, 0, -1), &s);
                std::memcpy(tj.data() + 2 * b0, stg.result(k0), 2 * bn * sizeof(double));
            }
        }
    }
    DP_TRY(finish_profile(ctx, &s));
    s.seconds = now_s() - t0;
    combine(*ps, tj, *out);
    out->tr[0] += td[0];
    out->tr[1] += td[1];
    if (out->per_sample)
        for (int k = 0; k < ps->nsamples; ++k) {
            out->per_sample[2 * k] += td[0];
            out->per_sample[2 * k + 1] += td[1];
        }
    out->solve = s;
    if (tr_defl) {
        tr_defl[0] = td[0];
        tr_defl[1] = td[1];
    }
    const dp_status fs = final_status(s);
    if (fs == DP_ENOCONV) ctx->err = "trace_deflated: some right-hand sides did not converge";
    if (fs == DP_EBREAKDOWN) ctx->err = "trace_deflated: CG breakdown";
    return fs;
}

}  // extern "C"
