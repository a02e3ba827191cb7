// dp_solve_noalloc: the single-instance solve of dp_solve_batch with every
// workspace buffer carved from one static device array, for callers that
// cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).
//
// The array below is a host-side stand-in in host code: its device address
// on each GPU is looked up once per device with hipGetSymbolAddress when a
// context is created (noalloc_attach) and only that address is used after.
// Every call on one GPU shares that GPU's array, which keeps the last call's
// contents; calls that overlap on one GPU (two host threads, two contexts)
// race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>

#include "context.h"

namespace dp {

namespace {

constexpr size_t kScratchBytes = DP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Points the context's workspace slots at pieces of the scratch array for
// the duration of one call (ensure() then finds them large enough and,
// with no_alloc set, never allocates); the previous slots come back after.
struct ScratchSlots {
    dp_ctx *ctx;
    void *saved[kNumSlots];
    size_t saved_bytes[kNumSlots];
    ScratchSlots(dp_ctx *c, char *base, const size_t (&bytes)[kNumSlots]) : ctx(c) {
        std::memcpy(saved, ctx->slot, sizeof saved);
        std::memcpy(saved_bytes, ctx->slot_bytes, sizeof saved_bytes);
        size_t off = 0;
        for (int s = 0; s < kNumSlots; ++s) {
            ctx->slot[s] = bytes[s] ? base + off : nullptr;
            ctx->slot_bytes[s] = bytes[s];
            off += align256(bytes[s]);
        }
        ctx->no_alloc = true;
    }
    ~ScratchSlots() {
        std::memcpy(ctx->slot, saved, sizeof saved);
        std::memcpy(ctx->slot_bytes, saved_bytes, sizeof saved_bytes);
        ctx->no_alloc = false;
    }
};

// Scratch bytes of a solve at width W (the slots that prepare_operator and
// make_launch take; the colour slot of the autotuner is never used here).
size_t layout(const Lat &lat, int nc, bool links, int inner, int W, size_t (&bytes)[kNumSlots]) {
    size_t tot = 0;
    for (int s = 0; s < kNumSlots; ++s) {
        bytes[s] = slot_size(s, lat, nc, links, inner, W);
        tot += align256(bytes[s]);
    }
    return tot;
}

}  // namespace

// Device address of the scratch array on the current device (which is
// `device`), looked up once per device.
dp_status noalloc_attach(int device, std::string &err) {
    if (device < 0 || device >= kMaxDevices) {
        err = "no-alloc scratch: device index out of range";
        return DP_EHIP;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return DP_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return DP_EHIP;
    }
    g_ptr[device] = ptr;
    return DP_OK;
}

}  // namespace dp

using namespace dp;

extern "C" dp_status dp_solve_noalloc(dp_ctx *ctx, const dp_operator *op, const void *b, void *x, int64_t nrhs,
                                      const dp_solve_opts *o, dp_solve_stats *st, hipStream_t stream) {
    if (!ctx) return DP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->err = "hipSetDevice failed";
        return DP_EHIP;
    }
    if (!op || !o || nrhs < 0 || (nrhs > 0 && (!b || !x))) {
        ctx->err = "solve_noalloc: bad arguments";
        return DP_EINVAL;
    }
    if (o->use_graph || o->profile) {
        ctx->err = "solve_noalloc: use_graph and profile need allocations; set both to 0";
        return DP_EINVAL;
    }
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        base = ctx->device < kMaxDevices ? g_ptr[ctx->device] : nullptr;
    }
    if (!base) {
        ctx->err = "solve_noalloc: no scratch address for this device (context creation failed?)";
        return DP_EHIP;
    }
    SolveCfg cfg;
    cfg.tol = o->tol;
    cfg.max_iter = o->max_iter > 0 ? o->max_iter : 100000;
    cfg.inner = o->inner;
    cfg.delta = o->reliable_delta > 0 ? o->reliable_delta : default_reliable_delta(cfg.inner);
    cfg.ru_gap = default_ru_gap(cfg.inner);
    if (!(cfg.tol > 0) || !(cfg.delta < 1) || (cfg.inner != kF64 && cfg.inner != kF32 && cfg.inner != kBF16)) {
        ctx->err = "solve_noalloc: tol must be > 0, reliable_delta < 1, inner a DP_PREC_* value";
        return DP_EINVAL;
    }
    for (int d = 0; d < 4; ++d)
        if (op->dims[d] < 1) {
            ctx->err = "operator dims must be >= 1";
            return DP_EINVAL;
        }
    if (op->nc != 1 && op->nc != 3) {
        ctx->err = "operator nc must be 1 or 3";
        return DP_EINVAL;
    }
    const long long N = (long long)op->dims[0] * op->dims[1] * op->dims[2] * op->dims[3];
    if (N > (1LL << 30) / 8) {
        ctx->err = "lattice too large";
        return DP_EUNSUPPORTED;
    }
    Lat lat{};
    for (int d = 0; d < 4; ++d) lat.D[d] = op->dims[d];
    lat.N = (int)N;
    const bool links = op->links != nullptr;
    // width: the caller's, else the widest power of two <= 32 (and <= the
    // next power of two of nrhs) whose workspace fits the array
    int W = o->rhs_block;
    size_t bytes[kNumSlots];
    if (W != 0) {
        if (W < 0 || W > kMaxW || (W & (W - 1))) {
            ctx->err = "rhs_block must be a power of two <= 256";
            return DP_EINVAL;
        }
        const size_t need = layout(lat, op->nc, links, cfg.inner, W, bytes);
        if (need > kScratchBytes) {
            ctx->err = "solve_noalloc: this lattice at rhs_block " + std::to_string(W) + " needs " +
                       std::to_string(need) + " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                       " of DP_NOALLOC_SCRATCH_BYTES";
            return DP_EINVAL;
        }
    } else {
        W = 1;
        while (W < 32 && W < nrhs) W *= 2;
        while (W > 1 && layout(lat, op->nc, links, cfg.inner, W, bytes) > kScratchBytes) W /= 2;
        const size_t need = layout(lat, op->nc, links, cfg.inner, W, bytes);
        if (need > kScratchBytes) {
            ctx->err = "solve_noalloc: this lattice needs " + std::to_string(need) +
                       " bytes of scratch even at rhs_block 1, more than the " + std::to_string(kScratchBytes) +
                       " of DP_NOALLOC_SCRATCH_BYTES";
            return DP_EINVAL;
        }
    }
    const double t0 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    dp_solve_stats s{};
    s.rhs_block = W;
    {
        ScratchSlots scope(ctx, (char *)base, bytes);
        OpPrep opp;
        DP_TRY(prepare_operator(ctx, *op, cfg.inner, opp, stream));
        Launch L;
        Red rd{};
        CgState cs{};
        DP_TRY(make_launch(ctx, opp, W, stream, L, rd, cs, cfg));
        // every buffer of the layout is written before it is read: the init
        // kernel writes b, r, p, x (and the FP64 copies) at every site and
        // lane, the finishing kernels the whole per-lane state, and each
        // reduction all of its partial sums, so nothing left by an earlier
        // call on this GPU needs clearing
        for (long long r0 = 0; r0 < nrhs; r0 += W) {
            const long long nv = std::min<long long>(W, nrhs - r0);
            BlockStats bs;
            bs.nvalid = (int)nv;
            InitAbi init{&L, cfg.inner, (const double *)b, r0, nv, &rd, &cs, ctx};
            double *x64 = (double *)ctx->at(kSlotX64);
            DP_TRY(solve_block(ctx, opp, cfg, L, rd, cs, x64, init, bs, &s));
            launch_to_abi(L, x64, (double *)x, r0, nv);
            DP_HIP(hipGetLastError());
        }
        DP_HIP(hipStreamSynchronize(stream));
    }
    s.seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count() - t0;
    if (st) *st = s;
    if (s.nbreakdown > 0) {
        ctx->err = "solve_noalloc: CG breakdown (operator not positive definite?)";
        return DP_EBREAKDOWN;
    }
    if (s.nconverged < s.nrhs) {
        ctx->err = "solve_noalloc: some right-hand sides did not converge";
        return DP_ENOCONV;
    }
    return DP_OK;
}
