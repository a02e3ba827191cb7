// Multi-instance engine: many independent lattice instances (each with its
// own operator, displacement and probes) solved together.  The work is a
// list of jobs, one per block of W right-hand sides of an instance, ordered
// longest first.  Up to kMaxSlots jobs are resident at once, each in a slot
// with its own buffers and CG state; every kernel of a CG iteration is ONE
// launch over all slots (a device-side slot table maps workgroups to slots),
// so small lattices share the GPU instead of each underfilling it.  The
// workgroups of a launch are shared among the busy slots in proportion to
// their site tiles, so a launch is not as long as its largest lattice needs
// with an equal share.  At each host check the finished slots are contracted
// and refilled with the next jobs; the slot table is rewritten in device
// memory, so the captured graph of an iteration group stays valid for the
// whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "context.h"

namespace dp {

namespace {

constexpr int kMaxSlots = 256;
constexpr int kSlotMaxBlk = 2048;           // workgroups of one slot (partial sums per lane)
constexpr int kLaunchBlk = 2048 * 8;        // workgroups of one multi-instance launch
constexpr size_t kSlotBudget = 48ull << 30;  // device bytes of all slot buffers

// Buffers of one call, taken from the context's pool and returned to it at
// the end of the call (the stream is synchronised before that).
struct DevBuf {
    dp_ctx *ctx;
    hipStream_t s;
    std::vector<std::pair<void *, size_t>> ptrs;
    DevBuf(dp_ctx *c, hipStream_t st) : ctx(c), s(st) {}
    ~DevBuf() {
        (void)hipStreamSynchronize(s);
        for (auto &b : ptrs) ctx->pool_put(b.first, b.second);
    }
    dp_status alloc(dp_ctx *, void **out, size_t bytes, bool zero = false) {
        void *p = nullptr;
        size_t got = 0;
        DP_TRY(ctx->pool_get(bytes, &p, &got));
        ptrs.emplace_back(p, got);
        if (zero) DP_HIP(hipMemsetAsync(p, 0, bytes ? bytes : 256, s));
        *out = p;
        return DP_OK;
    }
};

size_t prec_bytes(int prec) { return prec == kF64 ? 16 : (prec == kF32 ? 8 : 4); }

struct Job {
    int inst;
    long long r0;
    int nv;
    double cost;
};

}  // namespace

dp_status run_batch(dp_ctx *ctx, std::vector<BatchInst> &in, const SolveCfg &cfg, int W, bool trace_mode,
                    hipStream_t s) {
    const int ninst = (int)in.size();
    const bool mixed = cfg.inner != kF64;
    const int nc = in[0].nc;
    const bool links = in[0].links;
    for (auto &I : in)
        if (!block_fits(I.lat, nc, W, cfg.inner)) {
            ctx->err = "rhs_block too wide for an instance: a block vector (N * nc * rhs_block elements) must "
                       "stay under 4 GiB";
            return DP_EINVAL;
        }
    int logW = 0;
    while ((1 << logW) < W) ++logW;
    DevBuf mem(ctx, s);

    // per-instance operator data: neighbour table and converted links
    int maxN = 0;
    for (auto &I : in) {
        maxN = std::max(maxN, I.lat.N);
        DP_TRY(mem.alloc(ctx, (void **)&I.nbr, (size_t)I.lat.N * 8 * sizeof(int)));
        // hop links in the storage precision, and in FP64 for the true
        // residual (the same array when the storage is FP64)
        if (I.links) {
            const size_t nh = (size_t)I.lat.N * 8 * nc * nc;
            DP_TRY(mem.alloc(ctx, &I.U8, nh * prec_bytes(cfg.inner)));
            if (cfg.inner != kF64) DP_TRY(mem.alloc(ctx, &I.U64, nh * 16));
            else I.U64 = I.U8;
        }
        prepare_links(I.lat, nc, I.links ? I.links_abi : nullptr, I.nbr, nullptr, cfg.inner, I.U8,
                      cfg.inner != kF64 ? (double *)I.U64 : nullptr, s);
    }
    DP_HIP(hipGetLastError());

    // jobs, longest first
    std::vector<Job> jobs;
    for (int i = 0; i < ninst; ++i)
        for (long long r0 = 0; r0 < in[i].nrhs; r0 += W) {
            const int nv = (int)std::min<long long>(W, in[i].nrhs - r0);
            jobs.push_back({i, r0, nv, (double)in[i].lat.N * nv * std::sqrt(9.0 / std::max(in[i].m2, 1e-6))});
        }
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job &a, const Job &b) { return a.cost > b.cost; });
    // resident slots: about 8192 right-hand sides in flight, within the
    // memory budget
    const size_t vec = (size_t)maxN * nc * W;
    const size_t lo = vec * prec_bytes(cfg.inner);
    // partial sums: the stencil's four per lane and workgroup, then |r|^2 and Re q^H p
    const size_t part_bytes = (size_t)W * kSlotMaxBlk * 6 * sizeof(double);
    const size_t slot_bytes = vec * 32 + lo * (mixed ? 4 : 3) + part_bytes;
    int slot_cap = std::min(kMaxSlots, std::max(64, 8192 / W));
    slot_cap = (int)std::min<size_t>(slot_cap, std::max<size_t>(1, kSlotBudget / slot_bytes));
    const int nslots = std::max(1, std::min<int>((int)jobs.size(), slot_cap));

    // workgroups of a launch: enough for every slot to run its largest
    // lattice with a full grid, at most kLaunchBlk, a multiple of 8
    const int spt = kBlock >> logW;
    const int maxtiles = (maxN + spt - 1) / spt;
    int gblk = (int)std::min<long long>(kLaunchBlk, (long long)nslots * grid_blocks(maxtiles));
    gblk = std::max(8 * nslots, gblk - gblk % 8);

    // slot buffers; descriptor nslots is an idle one for unused workgroups
    std::vector<SlotDesc> hsd(nslots + 1);
    std::memset(&hsd[nslots], 0, sizeof(SlotDesc));

    // CG state of all slots in one block (one stride per slot), mirrored in
    // pinned host memory for the read-back of finished slots
    const size_t st_doubles = kStateDoubles, st_ints = 3 * kMaxW + 8;
    const size_t st_stride = (st_doubles * sizeof(double) + st_ints * sizeof(int) + 255) / 256 * 256;
    char *st_all = nullptr;
    DP_TRY(mem.alloc(ctx, (void **)&st_all, st_stride * nslots));
    // Uploads of the slot table go through a ring of pinned staging buffers:
    // a copy from pageable memory waits for the stream's earlier work (one
    // hidden synchronisation per upload: 33 refills of the uneven batch cost
    // 190 us of idle GPU each).  A buffer is reused once the copy that last
    // read it has run (an event per buffer).
    constexpr int kRing = 4;
    const size_t sd_bytes = sizeof(SlotDesc) * (nslots + 1), sd_al = (sd_bytes + 255) / 256 * 256;
    const size_t so_bytes = sizeof(int) * (size_t)gblk;
    const size_t ring_stride = sd_al + (so_bytes + 255) / 256 * 256;
    const size_t ring_off = (st_stride * nslots + sizeof(int) * 16 * nslots + 255) / 256 * 256;
    char *st_host = nullptr;
    DP_TRY(ctx->host_pinned(ring_off + kRing * ring_stride, (void **)&st_host));
    char *ring_host = st_host + ring_off;
    struct Ring {
        hipEvent_t ev[kRing] = {};
        bool used[kRing] = {};
        int next = 0;
        ~Ring() {
            for (auto e : ev)
                if (e) (void)hipEventDestroy(e);
        }
    } ring;
    for (auto &e : ring.ev) DP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // control words of the slots: pinned host memory that k_b_ctrl writes
    // through its device alias (no copy before the host reads them)
    int *hctrl = (int *)(st_host + st_stride * nslots);
    std::memset(hctrl, 0, sizeof(int) * 16 * nslots);
    char *st_dev = nullptr;
    DP_HIP(hipHostGetDevicePointer((void **)&st_dev, st_host, 0));
    const char *ring_dev = st_dev + ring_off;
    int *ctrl_all = (int *)(st_dev + st_stride * nslots);
    // per slot: its active lanes as the last control kernel counted them
    int *live_all = nullptr;
    DP_TRY(mem.alloc(ctx, (void **)&live_all, sizeof(int) * nslots));
    for (int k = 0; k < nslots; ++k) {
        SlotDesc &d = hsd[k];
        std::memset(&d, 0, sizeof d);
        DP_TRY(mem.alloc(ctx, (void **)&d.b64, vec * 16));
        DP_TRY(mem.alloc(ctx, (void **)&d.x64, vec * 16));
        DP_TRY(mem.alloc(ctx, &d.r, lo));
        DP_TRY(mem.alloc(ctx, &d.p, lo));
        DP_TRY(mem.alloc(ctx, &d.q, lo));
        if (mixed)
            DP_TRY(mem.alloc(ctx, &d.xlo, lo));
        else
            d.xlo = d.x64;
        DP_TRY(mem.alloc(ctx, (void **)&d.rd.part1, part_bytes));
        d.rd.part2 = d.rd.part1 + (size_t)W * kSlotMaxBlk * 4;
        double *st = (double *)(st_all + st_stride * k);
        CgState &cs = d.cs;
        cs.rr = st;
        cs.qp = st + kMaxW;
        cs.rr_ref = st + 2 * kMaxW;
        cs.bb = st + 3 * kMaxW;
        cs.alpha = st + 4 * kMaxW;
        cs.beta = st + 5 * kMaxW;
        cs.true_rr = st + 6 * kMaxW;
        cs.tj = st + 7 * kMaxW;
        cs.xdef = mixed ? st + 9 * kMaxW : nullptr;
        int *iv = (int *)(st + st_doubles);
        cs.active = iv;
        cs.iters = iv + kMaxW;
        cs.flags = iv + 2 * kMaxW;
        cs.ctrl = ctrl_all + 16 * k;
        cs.ctrld = (double *)(ctrl_all + 16 * k + 8);
        cs.live = live_all + k;
        cs.tol2 = cfg.tol * cfg.tol;
        cs.delta2 = cfg.delta * cfg.delta;
        cs.hold = cfg.inner == kBF16;
        cs.rq_direct = cfg.inner == kBF16;
        cs.exact = !mixed;
    }
    std::vector<int> slot_of((size_t)gblk, nslots);
    SlotDesc *d_sd = nullptr;
    int *d_slot_of = nullptr;
    DP_TRY(mem.alloc(ctx, (void **)&d_sd, sizeof(SlotDesc) * (nslots + 1)));
    DP_TRY(mem.alloc(ctx, (void **)&d_slot_of, sizeof(int) * slot_of.size()));

    BatchLaunch B;
    B.sd = d_sd;
    B.slot_of = d_slot_of;
    B.nslots = nslots;
    B.nblocks = gblk;
    B.W = W;
    B.nc = nc;
    B.prec = cfg.inner;
    B.links = links;
    B.mode = W >= 64 ? 2 : (W >= 16 ? 1 : 0);
    B.stream = s;

    std::vector<int> slot_job(nslots, -1), slot_it(nslots, 0), slot_ru(nslots, 0);
    size_t next_job = 0;
    auto assign = [&](int k, int jidx) {
        const Job &jb = jobs[jidx];
        BatchInst &I = in[jb.inst];
        SlotDesc &d = hsd[k];
        d.L.lat = I.lat;
        d.L.nc = nc;
        const bool half = batch_narrow_last(W, jb.nv);
        d.L.W = half ? W / 2 : W;
        d.L.logW = half ? logW - 1 : logW;
        d.L.ntiles = (I.lat.N + (kBlock >> d.L.logW) - 1) / (kBlock >> d.L.logW);
        d.L.stream = s;
        d.diag = I.m2 + 8.0;
        d.U = I.U8;
        d.U64 = I.U64;
        d.nbr = I.nbr;
        ProbeGen g{};
        if (trace_mode) {
            g.colors = I.ps.colors_dev;
            g.seed = I.ps.seed;
            g.ncolors = I.ps.ncolors;
            g.sample0 = I.ps.sample0;
            g.noise = I.ps.noise;
            g.dilute = I.ps.dilute ? 1 : 0;
        }
        g.rhs0 = jb.r0;
        g.nvalid = jb.nv;
        d.g = g;
        d.gen_b = trace_mode ? 1 : 0;
        d.disp = I.disp;
        d.flags = kSlotInit;
        slot_job[k] = jidx;
        slot_it[k] = 0;
        slot_ru[k] = 0;
    };
    // Shares the workgroups among the slots that take part in any phase: 8
    // each, the rest in proportion to their site tiles, every share a
    // multiple of 8 (so b % 8 is still the XCD) and at most kSlotMaxBlk or
    // the slot's tiles; workgroups left over go to the idle descriptor.
    std::vector<int> share(nslots, 0);
    auto balance = [&]() -> bool {
        long long tot = 0;
        int nbusy = 0;
        for (int k = 0; k < nslots; ++k)
            if (hsd[k].flags) {
                tot += hsd[k].L.ntiles;
                ++nbusy;
            }
        const long long spare = gblk - 8LL * nbusy;
        bool changed = false;
        for (int k = 0; k < nslots; ++k) {
            int nb = 0;
            if (hsd[k].flags) {
                const int t = hsd[k].L.ntiles;
                const long long extra = spare * t / std::max(1LL, tot);
                nb = 8 + (int)(extra - extra % 8);
                const int cap = std::min(kSlotMaxBlk, std::max(8, (t + 7) / 8 * 8));
                nb = std::min(nb, cap);
            }
            changed |= nb != share[k];
            share[k] = nb;
        }
        if (!changed) return false;
        int b0 = 0;
        for (int k = 0; k < nslots; ++k) {
            SlotDesc &d = hsd[k];
            d.blk0 = b0;
            d.L.nblk = share[k];
            d.rd.nblk = share[k];
            for (int w = 0; w < share[k]; ++w) slot_of[b0 + w] = k;
            b0 += share[k];
        }
        for (int w = b0; w < gblk; ++w) slot_of[w] = nslots;
        return true;
    };
    // The |r|^2 partial sums of a slot's last vector update, which the next
    // CG iteration adds up, are laid out by its number of workgroups: when
    // the sharing changes they are rebuilt from the lane totals (cs.rr, set
    // by the check that preceded every change).
    auto upload = [&]() -> dp_status {
        const bool reshared = balance();
        const int i = ring.next;
        ring.next = (ring.next + 1) % kRing;
        if (ring.used[i]) DP_HIP(hipEventSynchronize(ring.ev[i]));
        char *buf = ring_host + ring_stride * i;
        const char *buf_dev = ring_dev + ring_stride * i;
        std::memcpy(buf, hsd.data(), sd_bytes);
        // copied by a kernel that reads the pinned buffer through its device
        // alias (a DMA copy per upload cost more: set-up latency on every call)
        if (reshared) {
            std::memcpy(buf + sd_al, slot_of.data(), so_bytes);
            launch_copy_in(d_slot_of, buf_dev + sd_al, so_bytes, s);
        }
        launch_copy_in(d_sd, buf_dev, sd_bytes, s);
        DP_HIP(hipGetLastError());
        DP_HIP(hipEventRecord(ring.ev[i], s));
        ring.used[i] = true;
        if (reshared) launch_b_reseed(B);
        return DP_OK;
    };
    // initialise the slots flagged kSlotInit, then make them iterate
    auto init_slots = [&]() -> dp_status {
        DP_TRY(upload());
        if (trace_mode) {
            launch_b_init(B, mixed ? 1 : 0);
        } else {
            for (int k = 0; k < nslots; ++k) {
                if (!(hsd[k].flags & kSlotInit)) continue;
                const Job &jb = jobs[slot_job[k]];
                launch_init_abi(hsd[k].L, cfg.inner, in[jb.inst].babi, jb.r0, jb.nv, hsd[k].b64, hsd[k].r,
                                hsd[k].p, hsd[k].xlo, hsd[k].x64, mixed ? 1 : 0, hsd[k].rd, hsd[k].cs);
            }
        }
        DP_HIP(hipGetLastError());
        for (auto &d : hsd)
            if (d.flags & kSlotInit) d.flags = kSlotIter;
        return upload();
    };
    auto read_ctrl_all = [&]() -> dp_status {
        launch_b_ctrl(B);
        DP_HIP(hipStreamSynchronize(s));
        if (cfg.profile) DP_TRY(finish_profile(ctx, &in[0].st));
        return DP_OK;
    };
    // contract / copy out the slots flagged kSlotFinal and record statistics
    // (their state blocks into the pinned mirror, one synchronisation)
    auto finish_slots = [&]() -> dp_status {
        DP_TRY(upload());
        // mixed precision: a slot finishes only after a reliable update
        // (which folded x and took the true residual of the final x64) or
        // with no active lane from the start; FP64: apply the deferred
        // solution update and take the true residual now
        if (!mixed) launch_b_ru(B, 1);
        if (trace_mode) launch_b_dot(B);
        DP_HIP(hipGetLastError());
        for (int k = 0; k < nslots; ++k) {
            if (!(hsd[k].flags & kSlotFinal)) continue;
            const Job &jb = jobs[slot_job[k]];
            if (!trace_mode) launch_to_abi(hsd[k].L, hsd[k].x64, in[jb.inst].xabi, jb.r0, jb.nv);
        }
        // the finished slots' state blocks into their pinned mirrors: one
        // kernel writing through the device alias, not one copy per slot
        launch_b_state_out(B, st_all, st_dev, st_stride);
        DP_HIP(hipGetLastError());
        DP_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < nslots; ++k) {
            if (!(hsd[k].flags & kSlotFinal)) continue;
            const Job &jb = jobs[slot_job[k]];
            BatchInst &I = in[jb.inst];
            // the slot's state block: doubles rr .. tj as laid out above, then the ints
            const double *hs = (const double *)(st_host + st_stride * k);
            const double *true_rr = hs + 6 * kMaxW, *bbv = hs + 3 * kMaxW, *tj = hs + 7 * kMaxW;
            const int *iv = (const int *)(hs + st_doubles);
            const int *iters = iv + kMaxW, *flags = iv + 2 * kMaxW;
            for (int j = 0; j < jb.nv; ++j) {
                const double bb = bbv[j];
                I.st.max_true_resid = std::max(I.st.max_true_resid, bb > 0 ? std::sqrt(true_rr[j] / bb) : 0.0);
                I.st.rhs_iters += iters[j];
                I.st.max_iters = std::max(I.st.max_iters, iters[j]);
                if (flags[j] & kFlagBreakdown) ++I.st.nbreakdown;
                else if (flags[j] & kFlagConverged) ++I.st.nconverged;
                if (trace_mode) {
                    I.tj[2 * (jb.r0 + j)] = tj[2 * j];
                    I.tj[2 * (jb.r0 + j) + 1] = tj[2 * j + 1];
                }
            }
            I.st.nrhs += jb.nv;
            hsd[k].flags = 0;
            slot_job[k] = -1;
        }
        return DP_OK;
    };

    for (int k = 0; k < nslots && next_job < jobs.size(); ++k) assign(k, (int)next_job++);
    DP_TRY(init_slots());

    int steps_next = std::max(1, ctx->check_every);
    // mixed precision: the x updates of an iteration group in pairs (as in
    // the single-instance solve)
    const bool xdefer = mixed && xdefer_enabled();
    std::vector<double> ratio_prev(nslots, -1.0);
    std::vector<int> it_prev(nslots, 0);
    ctx->drop_graphs();
    for (;;) {
        bool any = false;
        for (auto &d : hsd) any |= (d.flags & kSlotIter) != 0;
        if (!any) break;
        int steps = steps_next;
        for (int k = 0; k < nslots; ++k)
            if (hsd[k].flags & kSlotIter) steps = std::min(steps, std::max(1, cfg.max_iter - slot_it[k]));
        if (cfg.use_graph && !cfg.profile) {
            // B is fixed for the call, and the graphs are dropped before and after it
            const std::string key = "batch " + std::to_string(steps) + (xdefer ? " xdefer" : "");
            auto g = ctx->graphs.find(key);
            if (g == ctx->graphs.end()) {
                hipGraph_t graph = nullptr;
                hipGraphExec_t exec = nullptr;
                DP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                for (int c = 0; c < steps; ++c) launch_b_iteration(B, xmode_of(c, steps, xdefer));
                DP_HIP(hipStreamEndCapture(s, &graph));
                const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                DP_HIP(ie);
                g = ctx->graphs.emplace(key, exec).first;
            }
            DP_HIP(hipGraphLaunch(g->second, s));
        } else {
            double bytes = 0;
            for (int k = 0; k < nslots; ++k)
                if (hsd[k].flags & kSlotIter) bytes += stencil_alg_bytes(hsd[k].L.lat, nc, hsd[k].L.W, cfg.inner, B.links);
            for (int c = 0; c < steps; ++c) {
                DP_TRY(timed_launch(ctx, cfg.profile != 0, bytes,
                                    [&](hipEvent_t e0, hipEvent_t e1) { launch_b_stencil(B, e0, e1); }));
                launch_b_update(B, xmode_of(c, steps, xdefer));
            }
        }
        DP_HIP(hipGetLastError());
        for (int k = 0; k < nslots; ++k)
            if (hsd[k].flags & kSlotIter) slot_it[k] += steps;
        DP_TRY(read_ctrl_all());
        bool any_ru = false, any_fin = false;
        int next_steps = 16;
        for (int k = 0; k < nslots; ++k) {
            SlotDesc &d = hsd[k];
            if (!(d.flags & kSlotIter)) continue;
            const int *c = hctrl + 16 * k;
            double ratio, ru_ratio;
            std::memcpy(&ratio, c + 8, sizeof(double));
            std::memcpy(&ru_ratio, c + 10, sizeof(double));
            const int nactive = c[0];
            if (nactive == 0) {
                d.flags = kSlotFinal;
                any_fin = true;
                continue;
            }
            if (mixed && (c[2] > 0 || c[1] == nactive || slot_it[k] >= cfg.max_iter ||
                          slot_it[k] - slot_ru[k] >= cfg.ru_gap)) {
                d.flags = kSlotIter | kSlotRU;
                slot_ru[k] = slot_it[k];
                any_ru = true;
            } else if (slot_it[k] >= cfg.max_iter) {
                d.flags = kSlotFinal;
                any_fin = true;
                continue;
            }
            next_steps = std::min(next_steps, next_check(std::max(1, ctx->check_every), ratio, ratio_prev[k],
                                                         slot_it[k] - it_prev[k], cfg.inner == kBF16 ? ru_ratio : 0.0));
            ratio_prev[k] = ratio;
            it_prev[k] = slot_it[k];
        }
        steps_next = next_steps;
        if (any_ru) {
            DP_TRY(upload());
            launch_b_ru(B, 0);
            // no host round trip: the slots' lane counts are refreshed on the
            // device, a slot whose lanes all stopped at its update idles
            // (its iteration workgroups return at once) until the next check
            // retires it
            launch_b_count(B);
            DP_HIP(hipGetLastError());
            for (int k = 0; k < nslots; ++k) {
                SlotDesc &d = hsd[k];
                if (!(d.flags & kSlotRU)) continue;
                ++in[jobs[slot_job[k]].inst].st.reliable_updates;
                d.flags = kSlotIter;
                if (slot_it[k] >= cfg.max_iter) {
                    d.flags = kSlotFinal;
                    any_fin = true;
                }
            }
        }
        if (any_fin) {
            DP_TRY(finish_slots());
            bool any_init = false;
            for (int k = 0; k < nslots; ++k) {
                if (hsd[k].flags == 0 && next_job < jobs.size()) {
                    assign(k, (int)next_job++);
                    ratio_prev[k] = -1.0;
                    it_prev[k] = 0;
                    any_init = true;
                }
            }
            if (any_init) DP_TRY(init_slots());
            else DP_TRY(upload());
        }
        // (after a reliable update alone the device table keeps the slots'
        // update bit until the next upload, which precedes every launch that
        // reads it: the iteration kernels look at the iteration bit only)
    }
    DP_HIP(hipStreamSynchronize(s));
    if (cfg.profile) DP_TRY(finish_profile(ctx, &in[0].st));
    ctx->drop_graphs();
    return DP_OK;
}

}  // namespace dp
