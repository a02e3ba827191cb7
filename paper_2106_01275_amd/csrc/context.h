// The dp_ctx object and the solver driver shared by the ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <string>
#include <vector>

#include "dp_internal.h"

#define DP_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);         \
            return DP_EHIP;                                                       \
        }                                                                         \
    } while (0)

#define DP_TRY(expr)                  \
    do {                              \
        dp_status s_ = (expr);        \
        if (s_ != DP_OK) return s_;   \
    } while (0)

namespace dp {

enum Slot {
    kSlotNbr, kSlotU8, kSlotU8x, kSlotB64, kSlotX64, kSlotX64b, kSlotR, kSlotP, kSlotQ, kSlotQ64,
    kSlotXLo, kSlotPart1, kSlotState, kSlotColors, kSlotVec, kSlotCmap, kNumSlots
};

// A prepared operator: neighbour table and links in the internal layout.
struct OpPrep {
    Lat lat{};
    int nc = 1;
    double m2 = 0;
    bool links = false;
    const void *U8 = nullptr;   // hop links of the inner precision [N][8][nc][nc]: U_mu(x), then U_mu(x-mu)
    const void *U8x = nullptr;  // FP64 hop links (the true residual's FP64 stencil; U8 itself for FP64)
    const int *nbr = nullptr;
    int inner = kF64;
};

struct BlockStats {
    long long iters_sum = 0;
    int iters_max = 0, nconv = 0, nbreak = 0, nvalid = 0, ru = 0;
    double max_rel = 0;
};

}  // namespace dp

struct dp_ctx {
    int device = 0;
    std::string err;
    void *slot[dp::kNumSlots] = {};
    size_t slot_bytes[dp::kNumSlots] = {};
    int *ctrl_host = nullptr;        // pinned [16]: 4 counts, then 2 doubles at [4] and [6]
    int *ctrl_dev = nullptr;         // the same memory as the device sees it (k_ctrl writes it)
    double *state_host = nullptr;    // pinned staging of per-lane results
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    double ev_bytes = 0;                      // algorithmic bytes of the timed launches not yet reported
    double ev_ms = 0;                         // summed durations of the harvested timed launches
    int ev_done = 0;                          // number of those
    unsigned ev_seq = 0;                      // timed-launch candidates so far (sampling)
    double ev_bytes_all = 0;                  // algorithmic bytes of every profiled launch
    dp_status harvest_events(size_t n);       // reads and recycles the n oldest pending event pairs
    std::map<std::string, double> tuned_w;    // ms per CG iteration at a block width
    // autotuned stencil launches: mode, workgroups per (shape, precision, W)
    std::map<std::string, std::array<int, 2>> tuned_st;
    // DP_STENCIL at context creation: 0 tune (default), 1 the built-in rule,
    // 2 forced to stencil_forced (mode, workgroups; -1 / 0 keep the rule's)
    int stencil_policy = 0;
    std::array<int, 2> stencil_forced{{-1, 0}};
    bool tune_loaded = false;
    int check_every = 8;
    hipStream_t gstream = nullptr;            // library stream for graph capture
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::map<std::string, hipGraphExec_t> graphs;  // iteration groups by length and kernel arguments
    // device buffers of the multi-instance engine, kept for the next call
    // (hipMalloc / hipFree synchronise the device and cost far more than a
    // small batch's solves)
    std::vector<std::pair<void *, size_t>> pool;
    void *pinned = nullptr;                   // pinned host staging of the multi-instance engine
    size_t pinned_bytes = 0;
    dp_status host_pinned(size_t bytes, void **out);  // at least `bytes`, kept for later calls

    // set while a call runs on the static scratch array (dp_solve_noalloc):
    // ensure() and pool_get() then fail instead of allocating or freeing
    bool no_alloc = false;

    void drop_graphs();
    // smallest pooled buffer of at least `bytes`, else a new one; *got = its size
    dp_status pool_get(size_t bytes, void **out, size_t *got);
    void pool_put(void *p, size_t bytes);

    dp_status ensure(int s, size_t bytes, bool zero = false);
    void *at(int s) const { return slot[s]; }
};

namespace dp {

struct SolveCfg {
    int use_graph = 0;
    double tol = 1e-10;
    int max_iter = 100000;
    int inner = kF64;
    double delta = 0.1;
    int ru_gap = 100;     // a reliable update at least every ru_gap iterations (mixed)
    int profile = 0;
    int W = 0, logW = 0;
};

dp_status prepare_operator(dp_ctx *ctx, const dp_operator &op, int inner, OpPrep &out, hipStream_t s);
// Looks up (once per device, with `device` current) the device address of
// the static scratch array of dp_solve_noalloc.
dp_status noalloc_attach(int device, std::string &err);
// workgroups of a single-instance launch at width W (the default), and the
// largest number the stencil tuner may pick (partial-sum buffers are sized
// for it)
int launch_blocks(const Lat &lat, int W);
// update mode (launch_update's xmode) of iteration c of a group of n
int xmode_of(int c, int n, bool defer);
bool xdefer_enabled();
// The solve options' defaults shared by every entry point: the residual drop
// between reliable updates (reliable_delta = 0) and the longest run of
// iterations without one.
double default_reliable_delta(int inner);
int default_ru_gap(int inner);
int max_launch_blocks(const Lat &lat, int W);
// bytes of workspace slot `slot` that prepare_operator and make_launch need
// for this operator, inner precision and width (0: the slot is not used)
size_t slot_size(int slot, const Lat &lat, int nc, bool links, int inner, int W);
dp_status make_launch(dp_ctx *ctx, const OpPrep &op, int W, hipStream_t s, Launch &L, Red &rd, CgState &cs,
                      const SolveCfg &cfg);
// the stencil launch (mode, workgroups) of L's shape: cached,
// else timed (solver.cpp), or as DP_STENCIL says
dp_status pick_stencil(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, Launch &L, const CgState &cs);
// Runs CG on the block initialised by `init` (a callable launching the init
// kernel).  On return the FP64 solution is in x64_dst (internal layout).
// With `defer` (pinned host memory of state_bytes()) the block's state is
// copied there without a synchronisation and block_stats() is left to the
// caller; otherwise the statistics are added to bs and acc before return.
template <typename Init>
dp_status solve_block(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, const Launch &L, const Red &rd,
                      const CgState &cs, double *x64_dst, Init init, BlockStats &bs, dp_solve_stats *acc,
                      void *defer = nullptr);
size_t state_bytes();
void block_stats(const void *state, BlockStats &bs, dp_solve_stats *acc);
// whether a block vector of W right-hand sides stays under 4 GiB (the stencil
// kernels address it through 32-bit byte offsets)
bool block_fits(const Lat &lat, int nc, int W, int inner);
// For a batch, `work` lists (right-hand sides, sites) of every instance: the
// width then comes from the traffic per lane-site of a CG iteration times the
// padded lanes of each instance's last block (no timing).
dp_status choose_width(dp_ctx *ctx, const OpPrep &op, const SolveCfg &cfg, long long nrhs, int requested,
                       hipStream_t s, int &W, const std::vector<std::pair<long long, long long>> *work = nullptr);
dp_status finish_profile(dp_ctx *ctx, dp_solve_stats *st);
// runs launch(ev0, ev1); when profiling, with two events from the pool that
// the launch attaches to the kernel's own start and stop (finish_profile()
// later adds their interval and the launch's algorithmic bytes to the stats),
// otherwise with null events
// `stride`: only every stride-th launch carries the events (two events per
// launch cost host time that a short, launch-bound solve pays in full; a
// regular sample of equal launches gives the same average).
template <typename F>
dp_status timed_launch(dp_ctx *ctx, bool profile, double bytes, F launch, unsigned stride = 1) {
    if (profile) ctx->ev_bytes_all += bytes;
    if (!profile || (ctx->ev_seq++ % stride) != 0) {
        launch(hipEvent_t(nullptr), hipEvent_t(nullptr));
        return DP_OK;
    }
    if (ctx->ev_pool.size() < 2 && ctx->ev_pending.size() >= 256) DP_TRY(ctx->harvest_events(128));
    if (ctx->ev_pool.size() < 2) {
        for (int i = 0; i < 64; ++i) {
            // timing only: no system-scope fence (no L2 writeback around the timed launch)
            hipEvent_t e;
            DP_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            ctx->ev_pool.push_back(e);
        }
    }
    hipEvent_t e0 = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    hipEvent_t e1 = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    launch(e0, e1);
    ctx->ev_pending.emplace_back(e0, e1);
    ctx->ev_bytes += bytes;
    return DP_OK;
}
double stencil_alg_bytes(const Lat &lat, int nc, int W, int prec, bool links);
// Iterations until the next host check (2..16): what the slowest lane needs
// to reach tol and, with ru_ratio > 1 (mixed precision), what the first lane
// needs to be due a reliable update, both from the slowest lane's decay of
// |r|^2 over the last dit iterations (ratio_prev -> ratio); dflt without one.
int next_check(int dflt, double ratio, double ratio_prev, int dit, double ru_ratio);

// Work stream of a call: the caller's stream, or (graph replay requested)
// the library's own stream, ordered after the caller's stream on entry and
// before it on exit.
struct WorkStream {
    dp_ctx *ctx;
    hipStream_t user, s;
    bool own = false;
    dp_status enter(dp_ctx *c, hipStream_t u, bool graph);
    dp_status leave();
};

// One instance of a multi-instance batch (batch.cpp).
struct BatchInst {
    Lat lat{};
    int nc = 3;
    double m2 = 0;
    bool links = false;
    const void *links_abi = nullptr;   // caller's complex128 [4][N][nc][nc]
    void *U64 = nullptr, *U8 = nullptr;
    int *nbr = nullptr;
    long long nrhs = 0;
    dp_probe_spec ps{};                // trace mode
    int disp = 0;
    const double *babi = nullptr;      // solve mode
    double *xabi = nullptr;
    std::vector<double> tj;            // [2 * nrhs] contractions (trace mode)
    dp_solve_stats st{};
};
dp_status run_batch(dp_ctx *ctx, std::vector<BatchInst> &in, const SolveCfg &cfg, int W, bool trace_mode,
                    hipStream_t s);

// Initialisers of a block: probes generated on the device, or ABI vectors.
struct InitProbe {
    const Launch *L;
    int prec;
    ProbeGen g;
    const Red *rd;
    const CgState *cs;
    dp_ctx *ctx;
    void operator()(void *xlo, double *x64) const {
        launch_init_probe(*L, prec, g, (double *)ctx->at(kSlotB64), ctx->at(kSlotR), ctx->at(kSlotP), xlo, x64,
                          prec != kF64, *rd, *cs);
    }
    const ProbeGen *probe() const { return &g; }  // b is these probes
    static constexpr bool kLanesNonzero = true;     // a probe has a site of its colour
};

struct InitAbi {
    const Launch *L;
    int prec;
    const double *babi;
    long long rhs0, nvalid;
    const Red *rd;
    const CgState *cs;
    dp_ctx *ctx;
    void operator()(void *xlo, double *x64) const {
        launch_init_abi(*L, prec, babi, rhs0, nvalid, (double *)ctx->at(kSlotB64), ctx->at(kSlotR),
                        ctx->at(kSlotP), xlo, x64, prec != kF64, *rd, *cs);
    }
    const ProbeGen *probe() const { return nullptr; }  // b is read back from b64
    static constexpr bool kLanesNonzero = false;       // the caller's b may be zero
};

// deflation.cpp: the eigensolve, b64 -= Z (V^H b64) for one block of W
// right-hand sides, Tr(P A^{-1} Q), and the vectors in the ABI layout
dp_status deflation_build(dp_ctx *ctx, const dp_operator &op, int nvec, const dp_eig_opts &eo, dp_deflation &d,
                          hipStream_t s);
dp_status deflate_rhs(dp_ctx *ctx, const dp_deflation &d, const Launch &L, double *b64);
dp_status deflation_trace_part(dp_ctx *ctx, const dp_deflation &d, int p, hipStream_t s, double out[2]);
dp_status deflation_vectors(dp_ctx *ctx, const dp_deflation &d, double *out, hipStream_t s);

// Probes with the deflation applied: z is generated into b64, projected
// there, and the CG vectors are initialised from the result; the true
// residual then reads b64 (the probes are no longer the right-hand sides).
struct InitDeflated {
    const Launch *L;
    int prec;
    ProbeGen g;
    const Red *rd;
    const CgState *cs;
    dp_ctx *ctx;
    const dp_deflation *d;
    dp_status *status;  // set when the projection fails
    void operator()(void *xlo, double *x64) const {
        double *b64 = (double *)ctx->at(kSlotB64);
        launch_init_probe(*L, prec, g, b64, ctx->at(kSlotR), ctx->at(kSlotP), xlo, x64, prec != kF64, *rd, *cs);
        const dp_status e = deflate_rhs(ctx, *d, *L, b64);
        if (e != DP_OK) *status = e;
        launch_init_b64(*L, prec, b64, ctx->at(kSlotR), ctx->at(kSlotP), xlo, x64, prec != kF64, *rd, *cs);
    }
    const ProbeGen *probe() const { return nullptr; }
    static constexpr bool kLanesNonzero = true;  // (assumed; a zero lane only costs one group)
};

}  // namespace dp

// Deflation vectors of one operator (Sec. Deflation), device memory owned here.
struct dp_deflation {
    int device = 0;
    int nvec = 0, W = 0, outer = 0;
    dp::Lat lat{};
    int nc = 1;
    double m2 = 0;
    bool links = false;
    double *V = nullptr;  // Ritz vectors, internal layout [N][nc][W] (FP64 complex)
    double *Z = nullptr;  // A V Theta^{-1} in the kept lanes, zero in the others
    double *scratch = nullptr;  // device: tj [2W], true_rr [W], alpha [W], partial sums
    std::vector<double> theta, resid;
};
