// Solver driver: operator preparation, workspace, the batched CG loop with
// FP64 reliable updates, and the right-hand-side block width choice.
//
// CG (x0 = 0) runs on a block of W right-hand sides at once; every
// right-hand side keeps its own scalars on the device (alpha, beta, |r|^2),
// and right-hand sides that have converged are frozen (alpha = 0) while the
// others continue.  One iteration is three kernels and one reduction:
//   stencil   q = A p; p^H q, |q|^2 (BF16 storage: r^H q, r^H p too)
//   finish    alpha = |r|^2 / p^H q, the new |r|^2 from the recurrence
//             |r - alpha q|^2 = |r|^2 - 2 alpha Re r^H q + alpha^2 |q|^2 with
//             Re r^H q = Re p^H q - beta Re q_prev^H p (BF16: alpha from the
//             direct r^H p, the line search along p), beta, convergence flags
//   update    x += alpha p, r -= alpha q, p = r + beta p; |r|^2 and
//             Re q^H p of the new p as stored
// The host reads a control word after groups of iterations whose length is
// predicted from the residual decay.
//
// Mixed precision (inner = F32 or BF16): x, r, p, q are stored in the inner
// precision and the stencil accumulates in FP32; the solution is kept in
// FP64 (x64) and the residual is replaced by the FP64 true residual b - A x64
// (FP64 links) whenever it has dropped by reliable_delta since the last
// replacement, or when every active right-hand side believes it has
// converged.  Convergence is then decided on the FP64 true residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"

dp_status dp_ctx::ensure(int s, size_t bytes, bool zero) {
    if (bytes == 0) bytes = 256;
    if (slot_bytes[s] >= bytes) return DP_OK;
    if (no_alloc) {
        err = "internal: workspace slot " + std::to_string(s) + " needs " + std::to_string(bytes) +
              " bytes beyond the static scratch layout";
        return DP_ENOMEM;
    }
    dp_ctx *ctx = this;
    if (slot[s]) DP_HIP(hipFree(slot[s]));
    slot[s] = nullptr;
    slot_bytes[s] = 0;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        err = "out of device memory (" + std::to_string(bytes) + " bytes)";
        return DP_ENOMEM;
    }
    if (zero) DP_HIP(hipMemset(p, 0, bytes));
    slot[s] = p;
    slot_bytes[s] = bytes;
    return DP_OK;
}

dp_status dp_ctx::pool_get(size_t bytes, void **out, size_t *got) {
    if (bytes == 0) bytes = 256;
    if (no_alloc) {
        err = "internal: pooled buffer requested by a call that may not allocate";
        return DP_ENOMEM;
    }
    size_t best = pool.size();
    for (size_t i = 0; i < pool.size(); ++i)
        if (pool[i].second >= bytes && (best == pool.size() || pool[i].second < pool[best].second)) best = i;
    if (best < pool.size()) {
        *out = pool[best].first;
        *got = pool[best].second;
        pool.erase(pool.begin() + (long)best);
        return DP_OK;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        // release the pooled buffers and try once more
        for (auto &b : pool) (void)hipFree(b.first);
        pool.clear();
        if (hipMalloc(&p, bytes) != hipSuccess) {
            err = "out of device memory (" + std::to_string(bytes) + " bytes)";
            return DP_ENOMEM;
        }
    }
    *out = p;
    *got = bytes;
    return DP_OK;
}

void dp_ctx::pool_put(void *p, size_t bytes) { pool.emplace_back(p, bytes ? bytes : 256); }

dp_status dp_ctx::host_pinned(size_t bytes, void **out) {
    if (pinned_bytes < bytes) {
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        pinned_bytes = 0;
        if (hipHostMalloc(&pinned, bytes, hipHostMallocDefault) != hipSuccess) {
            pinned = nullptr;
            err = "pinned host allocation failed";
            return DP_ENOMEM;
        }
        pinned_bytes = bytes;
    }
    *out = pinned;
    return DP_OK;
}

dp_status dp_ctx::harvest_events(size_t n) {
    dp_ctx *ctx = this;
    n = std::min(n, ev_pending.size());
    for (size_t i = 0; i < n; ++i) {
        auto &pr = ev_pending[i];
        DP_HIP(hipEventSynchronize(pr.second));
        float ms = 0;
        DP_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        ev_ms += ms;
        ++ev_done;
        ev_pool.push_back(pr.first);
        ev_pool.push_back(pr.second);
    }
    ev_pending.erase(ev_pending.begin(), ev_pending.begin() + (long)n);
    return DP_OK;
}

void dp_ctx::drop_graphs() {
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
}

namespace dp {

dp_status WorkStream::enter(dp_ctx *c, hipStream_t u, bool graph) {
    ctx = c;
    user = u;
    s = u;
    if (!graph) return DP_OK;
    if (!ctx->gstream) {
        DP_HIP(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
        DP_HIP(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
        DP_HIP(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
    }
    DP_HIP(hipEventRecord(ctx->ev_in, u));
    DP_HIP(hipStreamWaitEvent(ctx->gstream, ctx->ev_in, 0));
    s = ctx->gstream;
    own = true;
    ctx->drop_graphs();
    return DP_OK;
}

dp_status WorkStream::leave() {
    if (!own) return DP_OK;
    own = false;
    DP_HIP(hipEventRecord(ctx->ev_out, s));
    DP_HIP(hipStreamWaitEvent(user, ctx->ev_out, 0));
    ctx->drop_graphs();
    return DP_OK;
}

static size_t prec_bytes(int prec) { return prec == kF64 ? 16 : (prec == kF32 ? 8 : 4); }

// work units of a launch: site tiles, or for one right-hand side groups of
// eight sites (the stencil splits a site over 32 threads, eight sites per
// workgroup, so the launch takes up to N / 8 workgroups; the other kernels
// leave the extra ones idle)
static int launch_units(const Lat &lat, int W) {
    int logW = 0;
    while ((1 << logW) < W) ++logW;
    const int ntiles = (lat.N + (kBlock >> logW) - 1) / (kBlock >> logW);
    return W == 1 ? std::max(ntiles, (lat.N + 7) / 8) : ntiles;
}

int launch_blocks(const Lat &lat, int W) { return grid_blocks(launch_units(lat, W)); }

// grids the stencil tuner times: the default and 256 .. 2048 workgroups
// (multiples of 8, not above the work units)
static std::vector<int> grid_candidates(const Lat &lat, int W) {
    const int units = launch_units(lat, W), base = launch_blocks(lat, W);
    std::vector<int> out{base};
    if (units <= 8) return out;
    for (int n : {256, 512, 1024, 2048})
        if (n < units && n != base) out.push_back(n);
    return out;
}

int max_launch_blocks(const Lat &lat, int W) {
    int m = 0;
    for (int n : grid_candidates(lat, W)) m = std::max(m, n);
    return m;
}

size_t slot_size(int slot, const Lat &lat, int nc, bool links, int inner, int W) {
    const size_t N = (size_t)lat.N, vec = N * nc * W, lo = vec * prec_bytes(inner);
    switch (slot) {
        case kSlotNbr: return N * 8 * sizeof(int);
        case kSlotU8: return links ? 2 * N * 4 * nc * nc * prec_bytes(inner) : 0;
        case kSlotU8x: return links && inner != kF64 ? 2 * N * 4 * nc * nc * 16 : 0;
        case kSlotQ64: return inner != kF64 ? vec * 16 : 0;
        case kSlotB64:
        case kSlotX64: return vec * 16;
        case kSlotR:
        case kSlotP:
        case kSlotQ: return lo;
        case kSlotXLo: return inner != kF64 ? lo : 0;
        case kSlotPart1: return (size_t)max_launch_blocks(lat, W) * W * 6 * sizeof(double);  // part1 [.][4], part2 [.][2]
        case kSlotState: return state_bytes();
        default: return 0;
    }
}

dp_status prepare_operator(dp_ctx *ctx, const dp_operator &op, int inner, OpPrep &out, hipStream_t s) {
    for (int d = 0; d < 4; ++d)
        if (op.dims[d] < 1) {
            ctx->err = "operator dims must be >= 1";
            return DP_EINVAL;
        }
    if (op.nc != 1 && op.nc != 3) {
        ctx->err = "operator nc must be 1 or 3";
        return DP_EINVAL;
    }
    if (inner != kF64 && inner != kF32 && inner != kBF16) {
        ctx->err = "unknown precision";
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
    out.lat.N = (int)N;
    for (int d = 0; d < 4; ++d) out.lat.D[d] = op.dims[d];
    out.nc = op.nc;
    out.m2 = op.m2;
    out.links = op.links != nullptr;
    out.inner = inner;
    auto sz = [&](int slot) { return slot_size(slot, out.lat, op.nc, out.links, inner, 1); };
    DP_TRY(ctx->ensure(kSlotNbr, sz(kSlotNbr)));
    out.nbr = (const int *)ctx->at(kSlotNbr);
    if (out.links) {
        DP_TRY(ctx->ensure(kSlotU8, sz(kSlotU8)));
        if (inner != kF64) DP_TRY(ctx->ensure(kSlotU8x, sz(kSlotU8x)));
        out.U8 = ctx->at(kSlotU8);
        out.U8x = inner != kF64 ? ctx->at(kSlotU8x) : out.U8;
    }
    prepare_links(out.lat, op.nc, op.links, (int *)out.nbr, nullptr, inner, (void *)out.U8,
                  inner != kF64 ? (double *)out.U8x : nullptr, s);
    DP_HIP(hipGetLastError());
    return DP_OK;
}

// ---------------------------------------------------------------- stencil tuner
//
// The stencil launch of a shape (lattice, nc, precision, links, W) is chosen
// by timing: every admissible mode (kernels.hip: per-lane links, LDS tiles,
// wave-uniform sites, x0 pairs, x0 x x3 quads, x0 lines) on every grid of
// grid_candidates, each over four CG iterations of a block of dense probes
// (the workgroup count is that of the whole iteration); the built-in
// choice stands unless another is 2% faster.  Choices are cached per shape in the context and
// with the block widths in the DP_TUNE_CACHE file.  DP_STENCIL=rule (at
// context creation) takes the built-in rule instead, DP_STENCIL=m,n forces
// mode m and n workgroups (-1 / 0 keep the rule's), where the shape admits
// them.
static std::string stencil_key(const OpPrep &op, int inner, int W) {
    char k[160];
    std::snprintf(k, sizeof k, "stencil gfx950 dims=%dx%dx%dx%d nc=%d prec=%d links=%d W=%d", op.lat.D[0],
                  op.lat.D[1], op.lat.D[2], op.lat.D[3], op.nc, inner, op.links ? 1 : 0, W);
    return k;
}

static void load_tune_file(dp_ctx *ctx);
static void save_tune_file(dp_ctx *ctx);

static void apply_choice(const std::array<int, 2> &c, const Lat &lat, int inner, Launch &L) {
    // any grid up to the largest candidate (the partial sums are sized for it)
    if (c[1] > 0 && c[1] <= max_launch_blocks(lat, L.W)) L.nblk = c[1];
    if (c[0] >= 0 && stencil_mode_valid(L, inner, c[0])) L.smode = c[0];
}

// Mean time of one CG iteration (stencil, finish, update) of the block in
// the workspace under launch shape Lc: the block is initialised with dense
// probes, one iteration runs untimed, four are timed.
static dp_status time_iterations(dp_ctx *ctx, const OpPrep &op, int inner, const Launch &Lc, const CgState &cs,
                                 hipEvent_t e0, hipEvent_t e1, float &ms) {
    Red rd;
    rd.part1 = (double *)ctx->at(kSlotPart1);
    rd.part2 = rd.part1 + (size_t)Lc.nblk * Lc.W * 4;
    rd.nblk = Lc.nblk;
    const bool mixed = inner != kF64;
    void *xlo = mixed ? ctx->at(kSlotXLo) : ctx->at(kSlotX64);
    ProbeGen g{};
    g.colors = (const int *)ctx->at(kSlotColors);  // one colour: dense noise
    g.seed = 12345;
    g.ncolors = 1;
    g.noise = DP_NOISE_Z2_COMPLEX;
    g.nvalid = Lc.W;
    launch_init_probe(Lc, inner, g, (double *)ctx->at(kSlotB64), ctx->at(kSlotR), ctx->at(kSlotP), xlo,
                      (double *)ctx->at(kSlotX64), mixed ? 1 : 0, rd, cs);
    StencilArgs a;
    a.links = op.links;
    a.diag = op.m2 + 8.0;
    a.pin = ctx->at(kSlotP);
    a.rin = ctx->at(kSlotR);
    a.q = ctx->at(kSlotQ);
    a.U = op.U8;
    a.nbr = op.nbr;
    a.cg = 1;
    a.rd = rd;
    a.cs = cs;
    // the solve's paired x updates (xmode 1 then 2) where it takes them
    const bool xdefer = cs.xdef != nullptr && xdefer_enabled();
    auto iter = [&](int xm) {
        launch_stencil(Lc, inner, a);
        launch_update(Lc, inner, xlo, ctx->at(kSlotR), ctx->at(kSlotP), ctx->at(kSlotQ), rd, cs, xm);
    };
    iter(0);
    DP_HIP(hipEventRecord(e0, Lc.stream));
    for (int k = 0; k < 4; ++k) iter(xmode_of(k, 4, xdefer));
    DP_HIP(hipEventRecord(e1, Lc.stream));
    DP_HIP(hipEventSynchronize(e1));
    DP_HIP(hipEventElapsedTime(&ms, e0, e1));
    DP_HIP(hipGetLastError());
    return DP_OK;
}

static dp_status tune_stencil(dp_ctx *ctx, const OpPrep &op, int inner, Launch &L, const CgState &cs,
                              std::array<int, 2> &best) {
    DP_TRY(ctx->ensure(kSlotColors, (size_t)L.lat.N * sizeof(int), true));
    hipEvent_t e0, e1;
    DP_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    DP_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    // the built-in choice and every valid (mode, workgroups), each timed twice,
    // in one order and then in the reverse one (a drift of the clock over the
    // sweep then favours no end of it); the least time of each counts
    std::vector<std::array<int, 2>> cand{{{-1, L.nblk}}};
    for (int n : grid_candidates(L.lat, L.W)) {
        Launch Lc = L;
        Lc.nblk = n;
        for (int mode = 0; mode <= 6; ++mode)
            if (stencil_mode_valid(Lc, inner, mode)) cand.push_back({{mode, n}});
    }
    std::vector<float> least(cand.size(), 1e30f);
    dp_status st = DP_OK;
    for (int pass = 0; pass < 2 && st == DP_OK; ++pass)
        for (size_t k = 0; k < cand.size() && st == DP_OK; ++k) {
            const size_t i = pass == 0 ? k : cand.size() - 1 - k;
            Launch Lc = L;
            if (cand[i][0] >= 0) {
                Lc.nblk = cand[i][1];
                Lc.smode = cand[i][0];
            }
            float ms = 0;
            st = time_iterations(ctx, op, inner, Lc, cs, e0, e1, ms);
            if (st == DP_OK) least[i] = std::min(least[i], ms);
        }
    // another choice has to beat the built-in one by 2% (timing noise is about 1%)
    best = cand[0];
    float best_ms = 0.98f * least[0];
    for (size_t i = 1; i < cand.size(); ++i)
        if (least[i] < best_ms) {
            best_ms = least[i];
            best = cand[i];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

dp_status pick_stencil(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, Launch &L, const CgState &cs) {
    const int inner = cfg.inner;
    if (ctx->stencil_policy == 1) return DP_OK;
    if (ctx->stencil_policy == 2) {
        apply_choice(ctx->stencil_forced, L.lat, inner, L);
        return DP_OK;
    }
    load_tune_file(ctx);
    const std::string key = stencil_key(op, inner, L.W);
    auto it = ctx->tuned_st.find(key);
    if (it == ctx->tuned_st.end()) {
        if (ctx->no_alloc) return DP_OK;  // (timing takes events: the built-in rule)
        std::array<int, 2> best;
        DP_TRY(tune_stencil(ctx, op, inner, L, cs, best));
        it = ctx->tuned_st.emplace(key, best).first;
        save_tune_file(ctx);
    }
    apply_choice(it->second, L.lat, inner, L);
    return DP_OK;
}

bool block_fits(const Lat &lat, int nc, int W, int inner) {
    return (double)lat.N * nc * W * (double)prec_bytes(inner) < 4294967296.0;
}

dp_status make_launch(dp_ctx *ctx, const OpPrep &op, int W, hipStream_t s, Launch &L, Red &rd, CgState &cs,
                      const SolveCfg &cfg) {
    if (!block_fits(op.lat, op.nc, W, cfg.inner)) {
        ctx->err = "rhs_block too wide for this lattice: a block vector (N * nc * rhs_block elements) must stay "
                   "under 4 GiB";
        return DP_EINVAL;
    }
    int logW = 0;
    while ((1 << logW) < W) ++logW;
    L.lat = op.lat;
    L.nc = op.nc;
    L.W = W;
    L.logW = logW;
    L.ntiles = (op.lat.N + (kBlock >> logW) - 1) / (kBlock >> logW);
    L.nblk = launch_blocks(op.lat, W);
    L.stream = s;
    L.smode = -1;
    for (int slot : {kSlotB64, kSlotX64, kSlotR, kSlotP, kSlotQ, kSlotQ64, kSlotXLo, kSlotPart1, kSlotState}) {
        const size_t b = slot_size(slot, op.lat, op.nc, op.links, cfg.inner, W);
        if (b) DP_TRY(ctx->ensure(slot, b));
    }
    const size_t nd = kStateDoubles;
    double *d = (double *)ctx->at(kSlotState);
    cs.rr = d;
    cs.qp = d + kMaxW;
    cs.rr_ref = d + 2 * kMaxW;
    cs.bb = d + 3 * kMaxW;
    cs.alpha = d + 4 * kMaxW;
    cs.beta = d + 5 * kMaxW;
    cs.true_rr = d + 6 * kMaxW;
    cs.tj = d + 7 * kMaxW;
    cs.xdef = cfg.inner != kF64 ? d + 9 * kMaxW : nullptr;
    // the control word lives in pinned host memory: k_ctrl writes it there
    // and the host reads it after the synchronisation, no copy
    cs.ctrld = (double *)(ctx->ctrl_dev + 4);
    int *iv = (int *)(d + nd);
    cs.active = iv;
    cs.iters = iv + kMaxW;
    cs.flags = iv + 2 * kMaxW;
    cs.ctrl = ctx->ctrl_dev;
    cs.tol2 = cfg.tol * cfg.tol;
    cs.delta2 = cfg.delta * cfg.delta;
    cs.hold = cfg.inner == kBF16;
    cs.rq_direct = cfg.inner == kBF16;  // see the finishing kernel
    cs.exact = cfg.inner == kF64;
    DP_TRY(pick_stencil(ctx, op, cfg, L, cs));
    rd.part1 = (double *)ctx->at(kSlotPart1);
    rd.part2 = rd.part1 + (size_t)L.nblk * W * 4;
    rd.nblk = L.nblk;
    return DP_OK;
}

static dp_status read_ctrl(dp_ctx *ctx, const Red &rd, const CgState &cs, int W, hipStream_t s) {
    launch_ctrl(rd, cs, W, s);
    DP_HIP(hipStreamSynchronize(s));
    return DP_OK;
}

int next_check(int dflt, double ratio, double ratio_prev, int dit, double ru_ratio) {
    int next = dflt;
    if (ratio_prev > 0 && ratio > 1.0 && ratio < ratio_prev && dit > 0) {
        const double per_it = std::log(ratio_prev / ratio) / dit;
        next = (int)std::ceil(std::log(ratio) / per_it);
        if (ru_ratio > 1.0) next = std::min(next, (int)std::ceil(std::log(ru_ratio) / per_it));
    }
    return std::min(16, std::max(2, next));
}

// Update mode of iteration c of a group of n: pairs (1, 2) of a deferred
// and a completing x update, and a plain last one when n is odd, so that x
// is whole at the end of every group (where a reliable update or the caller
// may read it).
int xmode_of(int c, int n, bool defer) {
    if (!defer) return 0;
    if (c & 1) return 2;
    return c + 1 < n ? 1 : 0;
}

// Default residual drop between reliable updates: about the unit roundoff
// of BF16 storage (2^-9; the fastest drop measured on the 16^4 single
// instance and the uneven batch, where 0.05 took 1.4x the time), and 1e-3
// for FP32, where the drop hardly matters.
double default_reliable_delta(int inner) { return inner == kBF16 ? 0.002 : 1e-3; }

// A reliable update at least every ru_gap iterations (mixed precision).
int default_ru_gap(int inner) { return inner == kBF16 ? 24 : 100; }

// DP_XDEFER=0 takes every x update at once (for comparison)
bool xdefer_enabled() {
    const char *e = std::getenv("DP_XDEFER");
    return !(e && std::strcmp(e, "0") == 0);
}

double stencil_alg_bytes(const Lat &lat, int nc, int W, int prec, bool links) {
    const double c = (double)prec_bytes(prec);  // one complex number
    return (double)lat.N * (2.0 * W * nc * c + (links ? 4.0 * nc * nc * c : 0.0));
}

static dp_status timed_stencil(dp_ctx *ctx, const SolveCfg &cfg, const Launch &L, const StencilArgs &a) {
    // the launches of one block are equal: below 256 MB of algorithmic
    // traffic per launch, time every 8th
    const double bytes = stencil_alg_bytes(L.lat, L.nc, L.W, cfg.inner, a.links);
    return timed_launch(ctx, cfg.profile != 0, bytes,
                        [&](hipEvent_t e0, hipEvent_t e1) {
                            StencilArgs ta = a;
                            ta.ev0 = e0;
                            ta.ev1 = e1;
                            launch_stencil(L, cfg.inner, ta);
                        }, bytes < 256e6 ? 8u : 1u);
}

dp_status finish_profile(dp_ctx *ctx, dp_solve_stats *st) {
    DP_TRY(ctx->harvest_events(ctx->ev_pending.size()));
    if (st) {
        st->stencil_ms += ctx->ev_ms;
        st->stencil_launches += ctx->ev_done;
        st->stencil_bytes += ctx->ev_bytes;
        st->stencil_bytes_all += ctx->ev_bytes_all;
    }
    ctx->ev_bytes_all = 0;
    ctx->ev_ms = 0;
    ctx->ev_done = 0;
    ctx->ev_bytes = 0;
    return DP_OK;
}

size_t state_bytes() { return kStateDoubles * sizeof(double) + (3 * kMaxW + 8) * sizeof(int); }

void block_stats(const void *state, BlockStats &bs, dp_solve_stats *acc) {
    // the layout of make_launch: doubles rr .. tj, then the ints active, iters, flags
    const double *d = (const double *)state;
    const double *true_rr = d + 6 * kMaxW, *bbv = d + 3 * kMaxW;
    const int *iv = (const int *)(d + kStateDoubles);
    const int *iters = iv + kMaxW, *flags = iv + 2 * kMaxW;
    for (int j = 0; j < bs.nvalid; ++j) {
        const double bb = bbv[j];
        const double rel = bb > 0 ? std::sqrt(true_rr[j] / bb) : 0.0;
        bs.max_rel = std::max(bs.max_rel, rel);
        bs.iters_sum += iters[j];
        bs.iters_max = std::max(bs.iters_max, iters[j]);
        if (flags[j] & kFlagBreakdown) ++bs.nbreak;
        else if (flags[j] & kFlagConverged) ++bs.nconv;
    }
    if (acc) {
        acc->rhs_iters += bs.iters_sum;
        acc->max_iters = std::max(acc->max_iters, bs.iters_max);
        acc->nconverged += bs.nconv;
        acc->nbreakdown += bs.nbreak;
        acc->reliable_updates += bs.ru;
        acc->max_true_resid = std::max(acc->max_true_resid, bs.max_rel);
        acc->nrhs += bs.nvalid;
    }
}

// Every argument a captured iteration group passes to its kernels, as a
// lookup key of the graph cache.
static std::string graph_key(int steps, int inner, const Launch &L, const StencilArgs &a, const void *xlo) {
    std::string k;
    auto put = [&k](const void *v, size_t n) { k.append((const char *)v, n); };
    auto val = [&put](auto v) { put(&v, sizeof v); };
    val(steps);
    val(inner);
    for (int d = 0; d < 4; ++d) val(L.lat.D[d]);
    val(L.lat.N);
    val(L.nc);
    val(L.W);
    val(L.logW);
    val(L.nblk);
    val(L.ntiles);
    val((const void *)L.stream);
    val(a.links);
    val(a.diag);
    val(a.pin);
    val(a.q);
    val(a.U);
    val((const void *)a.nbr);
    val(a.cg);
    val(a.rin);
    val((const void *)a.rd.part1);
    val((const void *)a.rd.part2);
    val(a.rd.nblk);
    const CgState &c = a.cs;
    for (const void *ptr : {(const void *)c.rr, (const void *)c.qp, (const void *)c.rr_ref,
                            (const void *)c.bb, (const void *)c.alpha, (const void *)c.beta,
                            (const void *)c.true_rr, (const void *)c.tj, (const void *)c.active,
                            (const void *)c.iters, (const void *)c.flags, (const void *)c.ctrl,
                            (const void *)c.ctrld})
        val(ptr);
    val(c.tol2);
    val(c.delta2);
    val(c.exact);
    val(c.hold);
    val(c.rq_direct);
    val(xlo);
    return k;
}

// The FP64 true residual r = b - A x64 of the block (ru: with the residual
// replacement; else statistics only): the FP64 stencil on x64 into an FP64
// q, then an element-wise pass that forms r,
// continues p and sums |r|^2.  With FP64 storage q itself is the scratch
// (its contents are dead whenever this runs).
static void true_residual(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, const Launch &L, const Red &rd,
                          const CgState &cs, const double *b64, double *x64, int ru, const ProbeGen *gen) {
    const bool mixed = cfg.inner != kF64;
    double *q64 = (double *)ctx->at(mixed ? kSlotQ64 : kSlotQ);
    StencilArgs a;
    a.links = op.links;
    a.diag = op.m2 + 8.0;
    a.pin = x64;
    a.q = q64;
    a.U = op.U8x;
    a.nbr = op.nbr;
    a.cg = 0;
    // the built-in choice, the fastest measured: 16^4, W = 32: FP64 quads
    // 100 us (although they hold 177 registers: two waves per SIMD), the LDS
    // tile 105, x0 pairs 108, per-lane links 157; 32^4: x0 lines 1504 us,
    // pairs 1672, the LDS tile 1756, per-lane links 2417
    Launch L64 = L;
    L64.smode = -1;
    launch_stencil(L64, kF64, a);
    launch_resid_q(L, cfg.inner, b64, q64, ctx->at(kSlotR), ctx->at(kSlotP), ctx->at(kSlotQ), ru, rd, cs, gen);
}

template <typename Init>
dp_status solve_block(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, const Launch &L, const Red &rd,
                      const CgState &cs, double *x64, Init init, BlockStats &bs, dp_solve_stats *acc,
                      void *defer) {
    const bool mixed = cfg.inner != kF64;
    void *xlo = mixed ? ctx->at(kSlotXLo) : (void *)x64;
    void *r = ctx->at(kSlotR), *p = ctx->at(kSlotP), *q = ctx->at(kSlotQ);
    const double *b64 = (const double *)ctx->at(kSlotB64);
    const double diag = op.m2 + 8.0;
    init(xlo, x64);  // b, r = p = b, xlo = 0 (x64 = 0)
    DP_HIP(hipGetLastError());
    int nactive = bs.nvalid;
    if (!Init::kLanesNonzero) {
        DP_TRY(read_ctrl(ctx, rd, cs, L.W, L.stream));
        nactive = ctx->ctrl_host[0];
    }
    int it = 0;
    StencilArgs a;
    a.links = op.links;
    a.diag = diag;
    a.pin = p;
    a.rin = r;
    a.q = q;
    a.U = op.U8;
    a.nbr = op.nbr;
    a.cg = 1;
    a.rd = rd;
    a.cs = cs;
    // Iterations between host checks: start with check_every, then predict
    // from the decay of the slowest lane's residual since the last check.
    int steps_next = std::max(1, ctx->check_every);
    // mixed precision takes the x updates of an iteration group in pairs
    // (the update kernel's deferred mode)
    const bool xdefer = cs.xdef != nullptr && xdefer_enabled();
    double ratio_prev = -1.0;
    int it_prev = 0, it_ru = 0;
    while (nactive > 0 && it < cfg.max_iter) {
        const int steps = std::min(steps_next, cfg.max_iter - it);
        if (cfg.use_graph && !cfg.profile) {
            // the group [stencil, finish, update] x steps replayed from a
            // graph; a graph holds the kernel arguments it was captured with,
            // so it is looked up by all of them (two solves of one call, say
            // the forward and adjoint solves of a gradient, or instances of
            // different shapes, never share a graph)
            const std::string key = graph_key(2 * steps + (xdefer ? 1 : 0), cfg.inner, L, a, xlo);
            auto g = ctx->graphs.find(key);
            if (g == ctx->graphs.end()) {
                if (ctx->graphs.size() >= 64) ctx->drop_graphs();
                hipGraph_t graph = nullptr;
                hipGraphExec_t exec = nullptr;
                DP_HIP(hipStreamBeginCapture(L.stream, hipStreamCaptureModeThreadLocal));
                for (int c = 0; c < steps; ++c) {
                    launch_stencil(L, cfg.inner, a);
                    launch_update(L, cfg.inner, xlo, r, p, q, rd, cs, xmode_of(c, steps, xdefer));
                }
                DP_HIP(hipStreamEndCapture(L.stream, &graph));
                const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                DP_HIP(ie);
                g = ctx->graphs.emplace(key, exec).first;
            }
            DP_HIP(hipGraphLaunch(g->second, L.stream));
        } else {
            for (int c = 0; c < steps; ++c) {
                DP_TRY(timed_stencil(ctx, cfg, L, a));
                launch_update(L, cfg.inner, xlo, r, p, q, rd, cs, xmode_of(c, steps, xdefer));
            }
        }
        DP_HIP(hipGetLastError());
        it += steps;
        DP_TRY(read_ctrl(ctx, rd, cs, L.W, L.stream));
        nactive = ctx->ctrl_host[0];
        {
            double ratio, ru_ratio;
            std::memcpy(&ratio, ctx->ctrl_host + 4, sizeof(double));
            std::memcpy(&ru_ratio, ctx->ctrl_host + 6, sizeof(double));
            steps_next = next_check(std::max(1, ctx->check_every), ratio, ratio_prev, it - it_prev,
                                    cfg.inner == kBF16 ? ru_ratio : 0.0);
            ratio_prev = ratio;
            it_prev = it;
        }
        if (mixed && nactive > 0 &&
            (ctx->ctrl_host[2] > 0 || ctx->ctrl_host[1] == nactive || it >= cfg.max_iter ||
             it - it_ru >= cfg.ru_gap)) {
            it_ru = it;
            // reliable update: x64 += xlo, r = b - A x64 in FP64 (p continued
            // from it), the residual norms restart from it
            launch_fold(L, cfg.inner, x64, xlo);
            true_residual(ctx, op, cfg, L, rd, cs, b64, x64, 1, init.probe());
            DP_HIP(hipGetLastError());
            ++bs.ru;
            DP_TRY(read_ctrl(ctx, rd, cs, L.W, L.stream));
            nactive = ctx->ctrl_host[0];
        }
    }
    // Mixed precision: lanes stop only at a reliable update, which folded
    // x and left the FP64 true residual of the final x64 in true_rr, so
    // with no lane active there is nothing left to do.  Otherwise (FP64, or
    // max_iter reached) fold what is left (mixed) and take the final true
    // residual (statistics).
    if (!(mixed && nactive == 0)) {
        if (mixed) launch_fold(L, cfg.inner, x64, xlo);
        true_residual(ctx, op, cfg, L, rd, cs, b64, x64, 0, init.probe());
        DP_HIP(hipGetLastError());
    }
    // the block's state (one copy); deferred: the caller reads it after its
    // next synchronisation, so the next block's work queues behind this one
    // without a host round trip
    if (defer) {
        DP_HIP(hipMemcpyAsync(defer, cs.rr, state_bytes(), hipMemcpyDeviceToHost, L.stream));
        return DP_OK;
    }
    void *h = ctx->state_host;
    DP_HIP(hipMemcpyAsync(h, cs.rr, state_bytes(), hipMemcpyDeviceToHost, L.stream));
    DP_HIP(hipStreamSynchronize(L.stream));
    DP_TRY(finish_profile(ctx, acc));
    block_stats(h, bs, acc);
    return DP_OK;
}

// Autotuner of the right-hand-side block width W (one instance): for each
// candidate W (powers of two from 8 to 256, not above the next power of two
// of nrhs, within a memory budget) a block of dense random right-hand sides
// runs 2 + 6 CG iterations of the real kernels, each width with its own
// tuned stencil launch; the 6 are timed with HIP events.  The chosen W
// solves all nrhs right-hand sides in the least time per iteration,
// ceil(nrhs / W) blocks times the time of one (the padding of the last block
// is paid for: 96 right-hand sides take 3 blocks of 32 or 2 of 64).  The
// time per width is cached per (dims, nc, precision, links, W) in the
// context, and in the JSON file named by DP_TUNE_CACHE when that variable is
// set.  A batch of instances is not timed: its width comes from a traffic
// model (see choose_width).
static std::string width_key(const OpPrep &op, const SolveCfg &cfg, int W) {
    char k[160];
    std::snprintf(k, sizeof k, "width gfx950 dims=%dx%dx%dx%d nc=%d prec=%d links=%d W=%d", op.lat.D[0],
                  op.lat.D[1], op.lat.D[2], op.lat.D[3], op.nc, cfg.inner, op.links ? 1 : 0, W);
    return k;
}

static void load_tune_file(dp_ctx *ctx) {
    const char *path = std::getenv("DP_TUNE_CACHE");
    if (!path || ctx->tune_loaded) return;
    ctx->tune_loaded = true;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        // lines of the form   "<width key>": <ms>,   or   "<stencil key>": "<mode>,<workgroups>",
        char *a = std::strchr(line, '"');
        char *b = a ? std::strchr(a + 1, '"') : nullptr;
        char *c = b ? std::strchr(b, ':') : nullptr;
        if (!c) continue;
        const std::string key(a + 1, b);
        const char *v = c + 1;
        while (*v == ' ') ++v;
        if (*v == '"') {
            std::array<int, 2> ch{{-1, 0}};
            if (std::sscanf(v + 1, "%d,%d", &ch[0], &ch[1]) == 2) ctx->tuned_st[key] = ch;
        } else {
            ctx->tuned_w[key] = std::strtod(v, nullptr);
        }
    }
    std::fclose(f);
}

static void save_tune_file(dp_ctx *ctx) {
    const char *path = std::getenv("DP_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    const size_t n = ctx->tuned_w.size() + ctx->tuned_st.size();
    size_t i = 0;
    for (auto &kv : ctx->tuned_w)
        std::fprintf(f, "  \"%s\": %.6g%s\n", kv.first.c_str(), kv.second, ++i < n ? "," : "");
    for (auto &kv : ctx->tuned_st)
        std::fprintf(f, "  \"%s\": \"%d,%d\"%s\n", kv.first.c_str(), kv.second[0], kv.second[1], ++i < n ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
}

static dp_status time_width(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, int W, hipStream_t s,
                            float &ms) {
    Launch L;
    Red rd{};
    CgState cs{};
    DP_TRY(make_launch(ctx, op, W, s, L, rd, cs, cfg));
    DP_TRY(ctx->ensure(kSlotColors, (size_t)op.lat.N * sizeof(int), true));
    ProbeGen g{};
    g.colors = (const int *)ctx->at(kSlotColors);  // one colour: dense noise
    g.seed = 12345;
    g.ncolors = 1;
    g.noise = DP_NOISE_Z2_COMPLEX;
    g.rhs0 = 0;
    g.nvalid = W;
    const bool mixed = cfg.inner != kF64;
    void *xlo = mixed ? ctx->at(kSlotXLo) : ctx->at(kSlotX64);
    launch_init_probe(L, cfg.inner, g, (double *)ctx->at(kSlotB64), ctx->at(kSlotR), ctx->at(kSlotP), xlo,
                      (double *)ctx->at(kSlotX64), mixed ? 1 : 0, rd, cs);
    StencilArgs a;
    a.links = op.links;
    a.diag = op.m2 + 8.0;
    a.pin = ctx->at(kSlotP);
    a.rin = ctx->at(kSlotR);
    a.q = ctx->at(kSlotQ);
    a.U = op.U8;
    a.nbr = op.nbr;
    a.cg = 1;
    a.rd = rd;
    a.cs = cs;
    // the solve's paired x updates (xmode 1 then 2) where it takes them
    const bool xdefer = cs.xdef != nullptr && xdefer_enabled();
    auto iter = [&](int xm) {
        launch_stencil(L, cfg.inner, a);
        launch_update(L, cfg.inner, xlo, ctx->at(kSlotR), ctx->at(kSlotP), ctx->at(kSlotQ), rd, cs, xm);
    };
    iter(xmode_of(0, 2, xdefer));
    iter(xmode_of(1, 2, xdefer));
    hipEvent_t e0, e1;
    DP_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    DP_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
    // two timed runs of 6 iterations, the lesser counting (one run alone
    // once ranked W = 16 above W = 32 on the 32^4 gradient, whose solves
    // then took 6% longer)
    for (int rep = 0; rep < 2; ++rep) {
        float t = 0;
        DP_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < 6; ++i) iter(xmode_of(i, 6, xdefer));
        DP_HIP(hipEventRecord(e1, s));
        DP_HIP(hipEventSynchronize(e1));
        DP_HIP(hipEventElapsedTime(&t, e0, e1));
        ms = rep == 0 ? t : std::min(ms, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    DP_HIP(hipGetLastError());
    return DP_OK;
}

dp_status choose_width(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, long long nrhs, int requested,
                       hipStream_t s, int &W, const std::vector<std::pair<long long, long long>> *work) {
    if (requested != 0) {
        if (requested < 0 || requested > kMaxW || (requested & (requested - 1))) {
            ctx->err = "rhs_block must be a power of two <= 256";
            return DP_EINVAL;
        }
        W = requested;
        return DP_OK;
    }
    if (nrhs <= 1) {
        W = 1;
        return DP_OK;
    }
    if (work) {
        // Many instances in one launch: the slots keep thousands of lanes in
        // flight at every width, so a width costs what its CG iteration moves
        // per lane-site, 10 vector passes plus the eight hop links of a site
        // shared by the W lanes (stencil: p, r read, q written; update: x, r,
        // p, q read, x, r, p written), times the padding of every instance's last
        // block (its lanes and blocks over the useful lane-sites sum n_i N_i).  Timing one instance
        // alone instead rewards wide blocks that fill the GPU by themselves
        // (64 uneven lattices: this ranks W = 16/32/64/128 as the measured
        // 133/123/141/159 ms per step; the timed single instance picked 128).
        // Widths below 16 (per-lane link loads) only when no instance has
        // more right-hand sides.
        const double c = (double)prec_bytes(cfg.inner);
        double useful = 0;
        long long most = 1;
        for (auto &nw : *work) {
            useful += (double)nw.first * nw.second;
            most = std::max(most, nw.first);
        }
        int wmax = 1;
        while (wmax < most && wmax < 128) wmax *= 2;
        double best = 1e300;
        int best_w = wmax;
        for (int w = std::min(16, wmax); w <= wmax; w *= 2) {
            // lane-sites and block-sites of the instances' blocks (a last
            // block at most half full runs half as wide where the engine
            // allows it: batch_narrow_last)
            double lanes = 0, blocks = 0;
            for (auto &nw : *work) {
                const long long full = nw.first / w, rem = nw.first % w;
                const int last = rem == 0 ? 0 : (batch_narrow_last(w, rem) ? w / 2 : w);
                lanes += (double)(full * w + last) * nw.second;
                blocks += (double)(full + (rem ? 1 : 0)) * nw.second;
            }
            const double bytes = lanes * 10.0 * op.nc * c + (op.links ? blocks * 8.0 * op.nc * op.nc * c : 0.0);
            const double cost = useful > 0 ? bytes / useful : bytes;
            if (cost < best * (1 - 1e-9)) {
                best = cost;
                best_w = w;
            }
        }
        W = best_w;
        return DP_OK;
    }
    load_tune_file(ctx);
    const size_t bytes_per_w = (size_t)op.lat.N * op.nc * (2 * 16 + 4 * (cfg.inner == kF64 ? 16 : 8));
    double best = 1e300;
    int best_w = 1;
    bool timed = false;
    for (int w = 8; w <= kMaxW; w *= 2) {
        if (w > 8 && w / 2 >= nrhs) break;
        if (bytes_per_w * w > ((size_t)32 << 30) || !block_fits(op.lat, op.nc, w, cfg.inner)) break;
        const std::string key = width_key(op, cfg, w);
        auto it = ctx->tuned_w.find(key);
        if (it == ctx->tuned_w.end()) {
            float ms = 0;
            DP_TRY(time_width(ctx, op, cfg, w, s, ms));
            timed = true;
            it = ctx->tuned_w.emplace(key, (double)ms / 6.0).first;
        }
        const double cost = (double)((nrhs + w - 1) / w) * it->second;
        if (cost < best) {
            best = cost;
            best_w = w;
        }
    }
    W = best_w;
    if (timed) save_tune_file(ctx);
    return DP_OK;
}

// explicit instantiations used by api.cpp
template dp_status solve_block<InitProbe>(dp_ctx *, const OpPrep &, const SolveCfg &, const Launch &, const Red &,
                                          const CgState &, double *, InitProbe, BlockStats &, dp_solve_stats *,
                                          void *);
template dp_status solve_block<InitAbi>(dp_ctx *, const OpPrep &, const SolveCfg &, const Launch &, const Red &,
                                        const CgState &, double *, InitAbi, BlockStats &, dp_solve_stats *,
                                        void *);
template dp_status solve_block<InitDeflated>(dp_ctx *, const OpPrep &, const SolveCfg &, const Launch &, const Red &,
                                        const CgState &, double *, InitDeflated, BlockStats &, dp_solve_stats *,
                                        void *);

}  // namespace dp
