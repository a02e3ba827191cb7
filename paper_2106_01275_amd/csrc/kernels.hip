// gfx950 kernels of the displaced-probing hot path (arXiv:2106.01275):
// probe generation (eqs. (3)-(4)), the gauge-covariant stencil A p, the CG
// vector updates with FP64 reductions, FP64 reliable updates, the displaced
// contraction z^H P x (Sec. 3) and the adjoint force.
//
// Data layout.  A block of W right-hand sides (W a power of two) is stored
// site-major with the right-hand side innermost: element (site, colour a,
// lane j) at ((site * nc + a) * W + j), complex.  A workgroup of 256 threads
// covers a tile of 256 / W sites; thread (site, j) = (tid / W, tid % W).  The
// W lanes of a site read consecutive addresses (coalesced) and share the
// site's links, which are staged once per tile in LDS (W >= 16) and reused by
// all W right-hand sides.  Consecutive tiles form one contiguous chunk per
// workgroup, and chunks are assigned so that each XCD owns a contiguous part
// of the lattice (its L2 then serves the x1/x2/x3 neighbour re-reads).
//
// Reductions (dot products per right-hand side) accumulate in FP64 across
// sites and workgroups; with FP32 or BF16 storage a thread first sums the
// few products of one site (its colours and hops) in FP32, or up to 24
// elements in the vector kernels, before adding them to its FP64 total.
// Every workgroup writes its partial sums, and a finishing kernel with one
// workgroup per right-hand side adds them in a fixed order (deterministic)
// and runs the CG scalar epilogue (alpha, beta, convergence flags) on the
// device, so the host only reads a control word now and then.  The kernel
// boundary makes the partials visible; no device-scope fence is used (on
// this multi-XCD part such a fence writes back the whole L2 of the XCD).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "dp_internal.h"

namespace dp {

// ============================================================ storage types

struct bf16x2 {
    uint32_t v;  // low half: real part, high half: imaginary part
};

typedef __bf16 bf16v2 __attribute__((ext_vector_type(2)));

// two FP32 values rounded to nearest even into one bf16x2 word (low = a)
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    bf16v2 v;
    v.x = (__bf16)a;
    v.y = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}

// c + a.lo * b.lo + a.hi * b.hi for bf16x2 words a, b (FP32 accumulation)
__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16v2, a), __builtin_bit_cast(bf16v2, b), c, false);
}

// Global-memory pointers.  A pointer that the compiler cannot trace to a
// kernel argument (one read from a slot descriptor) is a generic one to it,
// and generic (flat) accesses also count against the LDS wait counter, so
// that every wait for an LDS read waits for them too.  The accessors below
// cast to the global address space at each access (every vector, link and
// index array of this library is in global memory).
template <typename T>
using gp = __attribute__((address_space(1))) T *;

// (the value moves as raw bits: copying a class type binds a generic
// reference, which brings the flat access back)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T ldg(const T *p) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "4, 8 or 16 bytes");
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, *(gp<const uint32_t>)p);
    else if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, *(gp<const uint64_t>)p);
    else return __builtin_bit_cast(T, *(gp<const u32x4>)p);
}

template <typename T>
__device__ __forceinline__ void stg(T *p, const T &v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "4, 8 or 16 bytes");
    if constexpr (sizeof(T) == 4) *(gp<uint32_t>)p = __builtin_bit_cast(uint32_t, v);
    else if constexpr (sizeof(T) == 8) *(gp<uint64_t>)p = __builtin_bit_cast(uint64_t, v);
    else *(gp<u32x4>)p = __builtin_bit_cast(u32x4, v);
}

template <typename S>
struct St;

template <>
struct St<double2> {
    using R = double;
    __device__ static __forceinline__ void ld(const double2 *__restrict__ a, size_t i, R &re, R &im) {
        double2 v = ldg(a + i);
        re = v.x;
        im = v.y;
    }
    __device__ static __forceinline__ void st(double2 *__restrict__ a, size_t i, R re, R im) {
        stg(a + i, make_double2(re, im));
    }
    __device__ static __forceinline__ void round(R &, R &) {}
};

template <>
struct St<float2> {
    using R = float;
    __device__ static __forceinline__ void ld(const float2 *__restrict__ a, size_t i, R &re, R &im) {
        float2 v = ldg(a + i);
        re = v.x;
        im = v.y;
    }
    __device__ static __forceinline__ void st(float2 *__restrict__ a, size_t i, R re, R im) {
        stg(a + i, make_float2(re, im));
    }
    __device__ static __forceinline__ void round(R &, R &) {}
};

template <>
struct St<bf16x2> {
    using R = float;
    __device__ static __forceinline__ void ld(const bf16x2 *__restrict__ a, size_t i, R &re, R &im) {
        uint32_t v = ldg(a + i).v;
        re = __uint_as_float(v << 16);
        im = __uint_as_float(v & 0xffff0000u);
    }
    __device__ static __forceinline__ void st(bf16x2 *__restrict__ a, size_t i, R re, R im) {
        bf16x2 o;
        o.v = pack_bf16(re, im);
        stg(a + i, o);
    }
    // the value a store followed by a load would give
    __device__ static __forceinline__ void round(R &re, R &im) {
        const uint32_t v = pack_bf16(re, im);
        re = __uint_as_float(v << 16);
        im = __uint_as_float(v & 0xffff0000u);
    }
};

// ============================================================ helpers

// The workgroups working on one lattice: this workgroup's index b among
// them and their number nb.  A standalone launch uses (blockIdx, gridDim);
// in a multi-instance launch each slot owns a range of workgroups (starting
// at a multiple of 8, so b % 8 is still the XCD).
struct Blk {
    int b, nb;
};

__device__ __forceinline__ Blk own_blk() { return Blk{(int)blockIdx.x, (int)gridDim.x}; }

__device__ __forceinline__ int logical_block(const Blk &bk) {
    // Workgroups are dispatched round-robin over the 8 XCDs; renumber them so
    // that XCD x runs the contiguous range of logical blocks [x*n/8, (x+1)*n/8).
    const int n = bk.nb, b = bk.b;
    if (n % 8) return b;
    return (b % 8) * (n / 8) + b / 8;
}

__device__ __forceinline__ void tile_range(const Blk &bk, int ntiles, int &t0, int &t1) {
    const int lb = logical_block(bk), n = bk.nb;
    t0 = (int)(((long long)lb * ntiles) / n);
    t1 = (int)(((long long)(lb + 1) * ntiles) / n);
}

// Site traversal of the stencil kernels.  XCD x (workgroups with
// blockIdx % 8 == x) owns the x0-slices [x*D0/8, (x+1)*D0/8) when D0 is a
// multiple of 8 (otherwise one eighth of the site range); its workgroups
// walk the slab in steps, all together: step k covers consecutive work
// items, item w mapping to site (x0_lo + w % n0) * V3 + w / n0 (x0
// varies fastest).  The sites in flight then form a compact window whose
// neighbours (x0 ones included) are read at nearly the same time, so they
// hit in the XCD's L2.  (Taking the (x1, x2, x3) columns in blocks of a
// few x2-rows instead, so that the x1-neighbour planes of a window are
// those just read, cut the stencil's fetched bytes at 32^4 by a tenth but
// not its time, which is set by load latency rather than bytes.)
struct SiteWalk {
    int items;      // work items of this XCD
    int n0, x0_lo;  // x0-slices of the slab (n0 == 0: plain range)
    int base;       // first site (plain range)
    int V3;         // sites per x0-slice
    int first, stride;  // first tile of this workgroup and tile stride
    int n0s;            // log2 n0 if n0 is a power of two, else -1
};

__device__ __forceinline__ SiteWalk site_walk(const Launch &L, const Blk &bk) {
    const Lat &lat = L.lat;
    SiteWalk w;
    const int nb = bk.nb, b = bk.b;
    w.V3 = lat.D[1] * lat.D[2] * lat.D[3];
    if (nb >= 8 && nb % 8 == 0) {
        const int x = b % 8;
        w.first = b / 8;
        w.stride = nb / 8;
        if (lat.D[0] % 8 == 0) {
            w.n0 = lat.D[0] / 8;
            w.x0_lo = x * w.n0;
            w.items = w.n0 * w.V3;
            w.base = 0;
        } else {
            w.n0 = 0;
            w.x0_lo = 0;
            w.base = (int)(((long long)x * lat.N) / 8);
            w.items = (int)(((long long)(x + 1) * lat.N) / 8) - w.base;
        }
    } else {
        w.first = b;
        w.stride = nb;
        w.n0 = 0;
        w.x0_lo = 0;
        w.base = 0;
        w.items = lat.N;
    }
    w.n0s = w.n0 > 0 && (w.n0 & (w.n0 - 1)) == 0 ? __builtin_ctz(w.n0) : -1;
    return w;
}

// (a shift and a mask where n0 is a power of two: the walk is taken for
// every staged link element; 32^4, FP32, W = 32: 1.4% off the stencil)
__device__ __forceinline__ int walk_site(const SiteWalk &w, int item) {
    if (w.n0 == 0) return w.base + item;
    if (w.n0s >= 0) return (w.x0_lo + (item & (w.n0 - 1))) * w.V3 + (item >> w.n0s);
    return (w.x0_lo + item % w.n0) * w.V3 + item / w.n0;
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    // SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// noise value z0(s, site, b) as (re, im) in {-1, 0, 1}
__device__ __forceinline__ void noise(unsigned long long seedmix, long long s, int N, int site, int nc,
                                      int b, int kind, double &re, double &im) {
    const unsigned long long ctr =
        ((unsigned long long)s * (unsigned long long)N + (unsigned long long)site) * (unsigned long long)nc +
        (unsigned long long)b;
    const unsigned long long h = mix64(seedmix ^ ctr);
    const int top = (int)(h >> 63), nxt = (int)((h >> 62) & 1ull);
    if (kind == DP_NOISE_REAL_Z2) {
        re = top ? -1.0 : 1.0;
        im = 0.0;
    } else if (kind == DP_NOISE_Z2_COMPLEX) {
        re = top ? -1.0 : 1.0;
        im = nxt ? -1.0 : 1.0;
    } else {
        const int q = (int)(h >> 62);
        re = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
        im = q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0);
    }
}

__device__ __forceinline__ int shift0(const Lat &L, int site, int p) {
    // site + p e0 on the torus (p may be negative)
    const int stride0 = L.D[1] * L.D[2] * L.D[3];
    const int x0 = site / stride0;
    int y0 = (x0 + p) % L.D[0];
    if (y0 < 0) y0 += L.D[0];
    return site + (y0 - x0) * stride0;
}

// The sample s, colour c and dilution index a that lane-enumeration index J
// stands for (J = ((s - sample0) * ncolors + c) * n_dil + a); computed once
// per lane, outside the site loops (64-bit divisions).
struct ProbeLane {
    long long s;
    int c, a;
};

__device__ __forceinline__ ProbeLane probe_lane(const ProbeGen &g, int nc, long long J) {
    const int ndil = g.dilute ? nc : 1;
    ProbeLane pl;
    pl.s = g.sample0 + J / ((long long)g.ncolors * ndil);
    pl.c = (int)((J / ndil) % g.ncolors);
    pl.a = (int)(J % ndil);
    return pl;
}

// value of that lane's probe at (site, colour b); 0 outside its support
__device__ __forceinline__ void probe_at(const ProbeGen &g, unsigned long long seedmix, const Lat &L, int nc,
                                         const ProbeLane &pl, int site, int b, double &re, double &im) {
    re = 0.0;
    im = 0.0;
    const int x = g.shift ? shift0(L, site, -g.shift) : site;
    if (g.colors[x] != pl.c) return;
    if (g.dilute && b != pl.a) return;
    noise(seedmix, pl.s, L.N, x, nc, b, g.noise, re, im);
}

// probe value of lane-enumeration index J at (site, colour b); 0 outside
__device__ __forceinline__ void probe_value(const ProbeGen &g, unsigned long long seedmix, const Lat &L,
                                            int nc, long long J, int site, int b, double &re, double &im) {
    probe_at(g, seedmix, L, nc, probe_lane(g, nc, J), site, b, re, im);
}

// ------------------------------------------------------------ reductions

// Writes this workgroup's sums of NV values per lane to
// dst[(lane * nblk + b) * NV + v] (all threads call it once).
// Lane j = tid % W: the threads of one lane inside a wavefront are summed by
// a butterfly over the thread-index bits above log2 W, then the wavefronts
// in order through LDS (sm: NV * kBlock doubles); a fixed order.
template <int NV>
__device__ void block_partials_to(const Blk &bk, const double (&val)[NV], int W, int logW, double *dst, int nblk,
                                  double *sm) {
    const int tid = threadIdx.x;
    double v_[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        v_[v] = val[v];
        for (int off = W; off < 64; off <<= 1) v_[v] += __shfl_xor(v_[v], off, 64);
    }
    // per wavefront, threads 0 .. min(W, 64) - 1 hold the sums of their lanes
    const int per_wave = W < 64 ? W : 64;
    const int lane_in_wave = tid & 63;
    if (lane_in_wave < per_wave) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sm[v * kBlock + (tid >> 6) * per_wave + lane_in_wave] = v_[v];
    }
    __syncthreads();
    if (tid < W) {
        // lane tid's wavefront sums: W < 64: one per wavefront at
        // w * W + tid; W >= 64: the wavefronts w with w * 64 + (tid % 64) = tid
        // mod W, i.e. entries tid, tid + W, ... of the packed array
        const int nsum = W < 64 ? kBlock / 64 : kBlock / W;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
            for (int k = 0; k < nsum; ++k) s += sm[v * kBlock + k * W + tid];
            stg(dst + ((size_t)tid * nblk + bk.b) * NV + v, s);
        }
    }
}

// the same into rd.part1
template <int NV>
__device__ void block_partials(const Blk &bk, const double (&val)[NV], int W, int logW, const Red &rd, double *sm) {
    block_partials_to<NV>(bk, val, W, logW, rd.part1, rd.nblk, sm);
}

// Total over the nblk partial sums of one lane, src = the lane's [nblk][NV]
// block, in a fixed order (the same on every call): thread tid adds
// partials tid, tid + kBlock, ... (four loads in flight), then a butterfly
// in each wavefront and the wavefronts in order.  All threads call it; the
// totals are valid in thread 0.  sm: NV * kBlock / 64 doubles.
template <int NV>
__device__ __forceinline__ void lane_total(const double *src, int nblk, double (&tot)[NV], double *sm) {
    constexpr int kWaves = kBlock / 64;
    const int tid = threadIdx.x;
    double s[NV], s2[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = s2[v] = 0.0;
    int b = tid;
    for (; b + 3 * kBlock < nblk; b += 4 * kBlock) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double a0 = src[(size_t)b * NV + v], a1 = src[(size_t)(b + kBlock) * NV + v];
            const double a2 = src[(size_t)(b + 2 * kBlock) * NV + v], a3 = src[(size_t)(b + 3 * kBlock) * NV + v];
            s[v] += a0 + a1;
            s2[v] += a2 + a3;
        }
    }
    for (; b < nblk; b += kBlock) {
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] += src[(size_t)b * NV + v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double x = s[v] + s2[v];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if ((tid & 63) == 0) sm[v * kWaves + tid / 64] = x;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        tot[v] = 0.0;
        for (int w = 0; w < kWaves; ++w) tot[v] += sm[v * kWaves + w];
    }
}

// The same total by one wavefront alone (any wavefront of the workgroup;
// no LDS, no barrier): thread t adds partials t, t + 64, ..., then a
// butterfly; the totals are valid in every thread of the wavefront.  For the
// slots of the multi-instance engine, whose lanes have a few dozen partials
// each.
template <int NV>
__device__ __forceinline__ void lane_total_wave(const double *src, int nblk, double (&tot)[NV]) {
    const int t = threadIdx.x & 63;
#pragma unroll
    for (int v = 0; v < NV; ++v) tot[v] = 0.0;
    for (int b = t; b < nblk; b += 64) {
#pragma unroll
        for (int v = 0; v < NV; ++v) tot[v] += src[(size_t)b * NV + v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int off = 32; off > 0; off >>= 1) tot[v] += __shfl_xor(tot[v], off, 64);
}

// Epilogues of the finishing kernels.  Those marked (part2, NV = 2) total
// the |r|^2 and Re q^H p partials of the last vector update, initialisation
// or reliable update; kEpiTj and kEpiStatsP1 total rd.part1.
enum Epi { kEpiInit, kEpiCheck, kEpiRU, kEpiStats, kEpiStatsP1, kEpiTj };

// One workgroup per lane: total of the lane's partials (fixed order), then
// the scalar epilogue of that lane (thread 0; only this workgroup reads or
// writes lane j's state).
//   kEpiInit (part2)   |b|^2: the lane's CG state from scratch
//   kEpiCheck (part2)  |r|^2 of the latest residual into rr; FP64: lanes
//                      that meet tol stop (before a host check)
//   kEpiRU (part2)     the FP64 true residual of a reliable update
//   kEpiStats (part2), kEpiStatsP1 (part1)  a norm into true_rr only
//   kEpiTj (part1, NV = 2)  a complex dot product into tj
template <int NV, int EPI>
__device__ __forceinline__ void k_finish_body(int lane, const Red &rd, const CgState &cs) {
    __shared__ double sm[NV * kBlock / 64];
    const int tid = threadIdx.x;
    constexpr bool kPart2 = EPI == kEpiInit || EPI == kEpiCheck || EPI == kEpiRU || EPI == kEpiStats;
    static_assert(!kPart2 || NV == 2, "part2 holds two values per lane and workgroup");
    const double *src = (kPart2 ? rd.part2 : rd.part1) + (size_t)lane * rd.nblk * NV;
    const int j = lane;
    // the lane's state that the epilogue reads, loaded before the partials
    // so that the two loads' latencies overlap
    constexpr bool kState = EPI == kEpiCheck || EPI == kEpiRU;
    double st_ref = 0.0, st_bb = 0.0;
    int st_active = 0, st_flags = 0;
    if (kState && tid == 0) {
        st_ref = cs.rr_ref[j];
        st_bb = cs.bb[j];
        st_active = cs.active[j];
        st_flags = cs.flags[j];
    }
    double tot[NV];
    lane_total<NV>(src, rd.nblk, tot, sm);
    if (tid != 0) return;
    const double t = tot[0];
    if (EPI == kEpiInit) {
        cs.bb[j] = t;
        cs.rr[j] = t;
        cs.qp[j] = 0.0;
        cs.rr_ref[j] = t;
        cs.true_rr[j] = t;
        cs.alpha[j] = 0.0;
        cs.beta[j] = 0.0;
        cs.iters[j] = 0;
        cs.active[j] = t > 0.0;
        cs.flags[j] = t > 0.0 ? 0 : kFlagConverged;
        if (cs.live && j == 0) *cs.live = 1;  // iterate until a control kernel counts the lanes
    } else if (EPI == kEpiCheck) {
        cs.rr[j] = t;
        cs.qp[j] = tot[NV - 1];
        if (cs.exact && st_active && t <= cs.tol2 * st_bb) {
            cs.active[j] = 0;
            cs.flags[j] = st_flags | kFlagConverged;
        }
    } else if (EPI == kEpiRU) {
        // the residual is the true one from here on (the direction was
        // continued, kept or restarted by the kernel that wrote it)
        cs.true_rr[j] = t;
        if (st_active) {
            int flags = st_flags & ~(kFlagRestart | kFlagHold);
            cs.rr[j] = t;
            cs.qp[j] = tot[NV - 1];
            cs.rr_ref[j] = t;
            // a restarted direction is the residual itself (no previous one)
            if (st_flags & kFlagRestart) cs.beta[j] = 0.0;
            if (t <= cs.tol2 * st_bb) {
                cs.active[j] = 0;
                flags |= kFlagConverged;
            }
            cs.flags[j] = flags;
        }
    } else if (EPI == kEpiStats || EPI == kEpiStatsP1) {
        cs.true_rr[j] = t;
    } else {
        cs.tj[2 * j] = tot[0];
        cs.tj[2 * j + 1] = NV > 1 ? tot[NV - 1] : 0.0;
    }
}

template <int NV, int EPI>
__global__ __launch_bounds__(kBlock) void k_finish(Red rd, CgState cs) {
    k_finish_body<NV, EPI>(blockIdx.x, rd, cs);
}

// Finishing kernel of a CG iteration (single reduction), one workgroup per
// lane.  From the stencil's partials, pq = Re p^H q and qq = |q|^2 (q = A p
// as stored; with BF16 storage also rq = Re r^H q and rp = Re r^H p), and
// from the last update's, rr = |r|^2 (the residual as stored) and
// Re q_prev^H p:
//   FP64: a lane with rr <= tol^2 |b|^2 stops (converged);
//   BF16: a lane whose rr fell below delta^2 times its value at the last
//         reliable update holds (does not move) until that update;
//   alpha = rr / pq (BF16: rp / pq),
//   |r - alpha q|^2 = rr - 2 alpha rq + alpha^2 qq   (the new residual's
//         norm, known before the update that forms it; rq as below),
//   beta = |r - alpha q|^2 / rr,
// so that one kernel can then form x, r and p (the new |r|^2 is also summed
// there, exactly, for the next iteration: the expansion's cancellation
// never carries over from one iteration to the next).  pq <= 0: FP64 stops
// the lane (breakdown); mixed precision flags it to restart its direction
// at the next reliable update (FP32 takes a steepest-descent step
// meanwhile, BF16 holds).
// The lane's state as the finishing kernel reads it (loaded before the
// partials, so that the two latencies overlap).
struct LaneState {
    double ref = 0.0, bb = 0.0, beta = 0.0;
    int active = 0, flags = 0, iters = 0;
};

__device__ __forceinline__ LaneState load_lane_state(int j, const CgState &cs) {
    LaneState st;
    st.ref = cs.rr_ref[j];
    st.bb = cs.bb[j];
    st.beta = cs.beta[j];
    st.active = cs.active[j];
    st.flags = cs.flags[j];
    st.iters = cs.iters[j];
    return st;
}

__device__ __forceinline__ void finish_cg_epilogue(int j, const CgState &cs, const LaneState &ls, const double (&d3)[4],
                                                   const double (&d2)[2]);

__device__ __forceinline__ void k_finish_cg_body(int lane, const Red &rd, const CgState &cs) {
    __shared__ double sm[6 * kBlock / 64];
    const int tid = threadIdx.x;
    LaneState ls;
    if (tid == 0) ls = load_lane_state(lane, cs);
    double d3[4], d2[2];
    lane_total<4>(rd.part1 + (size_t)lane * rd.nblk * 4, rd.nblk, d3, sm);
    lane_total<2>(rd.part2 + (size_t)lane * rd.nblk * 2, rd.nblk, d2, sm + 4 * kBlock / 64);
    if (tid == 0) finish_cg_epilogue(lane, cs, ls, d3, d2);
}

// The same with one wavefront per lane (the multi-instance engine: a few
// dozen partials per lane).
__device__ __forceinline__ void k_finish_cg_wave_body(int lane, const Red &rd, const CgState &cs) {
    LaneState ls;
    if ((threadIdx.x & 63) == 0) ls = load_lane_state(lane, cs);
    double d3[4], d2[2];
    lane_total_wave<4>(rd.part1 + (size_t)lane * rd.nblk * 4, rd.nblk, d3);
    lane_total_wave<2>(rd.part2 + (size_t)lane * rd.nblk * 2, rd.nblk, d2);
    if ((threadIdx.x & 63) == 0) finish_cg_epilogue(lane, cs, ls, d3, d2);
}

// alpha, beta, flags and counts of lane j from its totals (thread-local)
__device__ __forceinline__ void finish_cg_epilogue(int j, const CgState &cs, const LaneState &ls, const double (&d3)[4],
                                                   const double (&d2)[2]) {
    const double st_ref = ls.ref, st_bb = ls.bb, st_beta = ls.beta;
    const int st_active = ls.active, st_flags = ls.flags, st_iters = ls.iters;
    const double rr = d2[0], pq = d3[0], qq = d3[2];
    // r^H q: since the residual is r = p - beta p_prev (beta the one that
    // formed p), r^H q = p^H q - beta p_prev^H A p, and p_prev^H A p =
    // (A p_prev)^H p = q_prev^H p was summed by the update that formed p (A
    // Hermitian; no conjugacy assumed).  A reliable update replaces r by the
    // true residual and keeps p, so the relation then holds up to the drift
    // of the recursive residual, which with FP32 storage is a few 1e-5 of
    // |r| and with BF16 storage up to about a tenth: there (rq_direct) the
    // stencil sums r^H q itself, and also r^H p, so that alpha is the exact
    // line search along p, Re r^H p / p^H A p, instead of |r|^2 / p^H A p
    // (equal while r^H p_prev = 0; after a replacement the first step
    // restores that orthogonality).
    const double rq = cs.rq_direct ? d3[1] : pq - st_beta * d2[1];
    const double rp = cs.rq_direct ? d3[3] : rr;
    int active = st_active, flags = st_flags, iters = st_iters;
    // a held lane keeps its direction, and with it the beta that formed it
    double alpha = 0.0, beta = st_beta;
    if (active) {
        if (cs.exact && rr <= cs.tol2 * st_bb) {
            active = 0;
            flags |= kFlagConverged;
        } else if (cs.hold && !(rr >= cs.delta2 * st_ref)) {
            flags |= kFlagHold;  // due a reliable update (or not finite)
        }
    }
    if (!active) beta = 0.0;
    if (active && !(flags & kFlagHold)) {
        if (!(pq > 0.0) || !isfinite(pq)) {
            beta = 0.0;
            if (cs.exact) {
                flags |= kFlagBreakdown;
                active = 0;
            } else {
                flags |= kFlagRestart | (cs.hold ? kFlagHold : 0);
            }
        } else {
            alpha = rp / pq;
            const double rn = rr - 2.0 * alpha * rq + alpha * alpha * qq;
            beta = rn > 0.0 && isfinite(rn) ? rn / rr : 0.0;
            ++iters;
        }
    }
    cs.rr[j] = rr;
    cs.qp[j] = d2[1];
    cs.alpha[j] = alpha;
    cs.beta[j] = beta;
    cs.active[j] = active;
    cs.flags[j] = flags;
    cs.iters[j] = iters;
}

__global__ __launch_bounds__(kBlock) void k_finish_cg(Red rd, CgState cs) { k_finish_cg_body(blockIdx.x, rd, cs); }

// Control word for the host: [0] active lanes, [1] active lanes whose
// recursive residual meets tol, [2] active lanes due a reliable update,
// [3] lanes that broke down; ctrld[0] the largest |r|^2 / (tol^2 |b|^2) of
// an active lane (how far the slowest one still is from convergence);
// ctrld[1] (mixed precision) the smallest |r|^2 / (delta^2 |r_ref|^2) of an
// active lane not yet due a reliable update (how close the next one is;
// 0 if there is none).
__device__ __forceinline__ void k_ctrl_body(const CgState &cs, int W) {
    __shared__ int cnt[4][64];
    __shared__ double worst[64], first[64];
    const int t = threadIdx.x;
    int na = 0, nk = 0, nru = 0, nb = 0;
    double wr = 0.0, fr = 0.0;
    for (int k = t; k < W; k += 64) {
        nb += (cs.flags[k] & kFlagBreakdown) ? 1 : 0;
        if (!cs.active[k]) continue;
        ++na;
        const double goal = cs.tol2 * cs.bb[k];
        if (cs.rr[k] <= goal) ++nk;
        const bool due = !(cs.rr[k] >= cs.delta2 * cs.rr_ref[k]) || (cs.flags[k] & (kFlagRestart | kFlagHold));
        if (due) {
            ++nru;
        } else if (!cs.exact) {
            const double q = cs.rr[k] / (cs.delta2 * cs.rr_ref[k]);
            fr = fr == 0.0 ? q : fmin(fr, q);
        }
        wr = fmax(wr, cs.rr[k] / goal);
    }
    cnt[0][t] = na;
    cnt[1][t] = nk;
    cnt[2][t] = nru;
    cnt[3][t] = nb;
    worst[t] = wr;
    first[t] = fr;
    __syncthreads();
    if (t != 0) return;
    for (int i = 1; i < 64; ++i) {
        for (int c = 0; c < 4; ++c) cnt[c][0] += cnt[c][i];
        worst[0] = fmax(worst[0], worst[i]);
        if (first[i] > 0.0) first[0] = first[0] == 0.0 ? first[i] : fmin(first[0], first[i]);
    }
    for (int c = 0; c < 4; ++c) cs.ctrl[c] = cnt[c][0];
    cs.ctrld[0] = worst[0];
    cs.ctrld[1] = first[0];
    if (cs.live) *cs.live = cnt[0][0];
}

__global__ void k_ctrl(CgState cs, int W) { k_ctrl_body(cs, W); }

// ============================================================ kernels

// The operator's device tables in one pass over the hop-link elements
// e = ((site * 8 + dir) * nc + a) * nc + b: the neighbour table nbr[site][8]
// (x + mu for dir = mu < 4, then x - mu; written by the elements a = b = 0),
// the FP64 links [N][4][nc][nc] (from the forward elements; if u64), and
// the hop links [N][8][nc][nc], entry (x, mu) = U_mu(x) and (x, 4 + mu) =
// U_mu(x - mu) (not conjugated), in the storage LS (if u8) and in FP64 (if
// u8x), so that a site's eight hops are one contiguous record.  The ABI links
// are complex128 [4][N][nc][nc]; without links (abi null) only the
// neighbour table.
template <typename LS>
__global__ void k_prepare(Lat L, int nc, const double2 *__restrict__ abi, int *__restrict__ nbr,
                          double2 *__restrict__ u64, LS *__restrict__ u8, double2 *__restrict__ u8x) {
    const int ne = abi ? nc * nc : 1;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 8LL * L.N * ne) return;
    const int ab = (int)(e % ne);
    const long long t = e / ne;
    const int dir = (int)(t % 8), site = (int)(t / 8), mu = dir & 3;
    int r = site, x = 0, stride = 1;
    for (int d = 3; d >= mu; --d) {
        if (d == mu) x = r % L.D[d];
        else stride *= L.D[d];
        r /= L.D[d];
    }
    const int y = dir < 4 ? site + (x + 1 == L.D[mu] ? -(L.D[mu] - 1) : 1) * stride
                          : site + (x == 0 ? L.D[mu] - 1 : -1) * stride;
    if (ab == 0) stg(nbr + (size_t)site * 8 + dir, y);
    if (!abi) return;
    const double2 v = ldg(abi + ((size_t)mu * L.N + (dir < 4 ? site : y)) * nc * nc + ab);
    if (u8) St<LS>::st(u8, e, (typename St<LS>::R)v.x, (typename St<LS>::R)v.y);
    if (u8x) stg(u8x + e, v);
    if (u64 && dir < 4) stg(u64 + ((size_t)site * 4 + mu) * nc * nc + ab, v);
}

// Initialise one block of W right-hand sides: b (FP64), r = p = b (storage
// precision), x = 0, and |b|^2 per lane; the finishing workgroup sets up
// the CG scalars.  SRC 0: probes generated from ProbeGen; 1: from ABI b.
template <typename S, int SRC>
__device__ __forceinline__ void k_init_body(const Blk &bk, Launch L, ProbeGen g, const double2 *__restrict__ babi,
                                                 long long rhs0, long long nvalid, double2 *__restrict__ b64,
                                                 S *__restrict__ r, S *__restrict__ p, S *__restrict__ xlo,
                                                 double2 *__restrict__ x64, int mixed, Red rd, CgState cs) {
    __shared__ double sm[2 * kBlock];
    const int tid = threadIdx.x, W = L.W, logW = L.logW;
    const int j = tid & (W - 1);
    const int nc = L.nc;
    const unsigned long long seedmix = SRC == 0 ? mix64(g.seed) : 0ull;
    const ProbeLane pl = SRC == 0 ? probe_lane(g, nc, g.rhs0 + j) : ProbeLane{};
    double acc[2] = {0.0, 0.0};  // |b|^2, and 0 for q^H p (no previous direction)
    int t0, t1;
    tile_range(bk, L.ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const int site = t * (kBlock >> logW) + (tid >> logW);
        if (site >= L.lat.N) continue;
        for (int a = 0; a < nc; ++a) {
            double re = 0.0, im = 0.0;
            const size_t i = ((size_t)(site * nc + a) << logW) + j;
            if (SRC == 0) {
                if (j < g.nvalid) probe_at(g, seedmix, L.lat, nc, pl, site, a, re, im);
            } else if (SRC == 1) {
                if (j < nvalid) {
                    const double2 v = babi[((size_t)(rhs0 + j) * L.lat.N + site) * nc + a];
                    re = v.x;
                    im = v.y;
                }
            } else {
                const double2 v = b64[i];  // b already in place
                re = v.x;
                im = v.y;
            }
            if (SRC != 2) b64[i] = make_double2(re, im);
            St<S>::st(r, i, (typename St<S>::R)re, (typename St<S>::R)im);
            St<S>::st(p, i, (typename St<S>::R)re, (typename St<S>::R)im);
            St<S>::st(xlo, i, 0, 0);
            if (mixed) x64[i] = make_double2(0.0, 0.0);
            acc[0] += re * re + im * im;
        }
    }
    block_partials_to<2>(bk, acc, W, logW, rd.part2, rd.nblk, sm);
}

template <typename S, int SRC>
__global__ __launch_bounds__(kBlock) void k_init(Launch L, ProbeGen g, const double2 *__restrict__ babi,
                                                 long long rhs0, long long nvalid, double2 *__restrict__ b64,
                                                 S *__restrict__ r, S *__restrict__ p, S *__restrict__ xlo,
                                                 double2 *__restrict__ x64, int mixed, Red rd, CgState cs) {
    k_init_body<S, SRC>(own_blk(), L, g, babi, rhs0, nvalid, b64, r, p, xlo, x64, mixed, rd, cs);
}

// q = A p for one block of right-hand sides; with CG, also p^H q per lane
// and the other dot products of a CG iteration (k_finish_cg).
// STAGE: links of the tile's sites staged in LDS (W >= 16).
// ------------------------------------------------------------ stencil helpers

__device__ __forceinline__ float fmaR(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return fma(a, b, c); }

// Element i of a block vector, addressed by a 32-bit byte offset from the
// vector's base: with the base uniform (a kernel argument, or read from a
// slot descriptor by the whole workgroup) the access takes the scalar-base +
// 32-bit-offset form, with no 64-bit address arithmetic per element.  Every
// block vector of the stencil kernels is smaller than 4 GiB (the host
// rejects wider blocks).
template <typename T>
__device__ __forceinline__ const T *at32(const T *base, unsigned i) {
    return (const T *)((const char *)base + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T *at32(T *base, unsigned i) {
    return (T *)((char *)base + i * (unsigned)sizeof(T));
}

// p as an opaque uniform value (p must be the same in every thread of the
// wavefront): the compiler cannot then fold a colour row's offset into
// per-thread 64-bit address arithmetic, and every load of a site's colours
// shares the one 32-bit site offset, each from its own scalar base.
template <typename T>
__device__ __forceinline__ T *ubase(T *p) {
    const unsigned long long a = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    return (T *)(((unsigned long long)hi << 32) | lo);
}

// The colour-row bases v + b * W (b < NC) of a block vector.
template <typename T, int NC>
struct Rows {
    T *b[NC];
    __device__ __forceinline__ Rows(T *v, int logW) {
#pragma unroll
        for (int c = 0; c < NC; ++c) b[c] = ubase(v + ((size_t)c << logW));
    }
};

// element (site y, colour b, lane j) of a block vector
__device__ __forceinline__ unsigned vidx(int y, int nc, int b, int logW, int j) {
    return ((unsigned)(y * nc + b) << logW) + (unsigned)j;
}

// colour components of lane j at site y
template <typename S, int NC>
__device__ __forceinline__ void ld_site(const S *__restrict__ v, int y, int logW, int j,
                                        typename St<S>::R (&re)[NC], typename St<S>::R (&im)[NC]) {
    const S *row = v + ((size_t)(y * NC) << logW);
#pragma unroll
    for (int b = 0; b < NC; ++b) St<S>::ld(row, (unsigned)((b << logW) + j), re[b], im[b]);
}

// the same from colour-row bases, through one 32-bit site offset
template <typename S, int NC>
__device__ __forceinline__ void ld_rows(const Rows<const S, NC> &v, int y, int logW, int j,
                                        typename St<S>::R (&re)[NC], typename St<S>::R (&im)[NC]) {
    const unsigned i = vidx(y, NC, 0, logW, j);
#pragma unroll
    for (int b = 0; b < NC; ++b) St<S>::ld(at32(v.b[b], i), 0, re[b], im[b]);
}

// and stores colour components to colour-row bases
template <typename S, int NC>
__device__ __forceinline__ void st_rows(const Rows<S, NC> &v, int y, int logW, int j, int b,
                                        typename St<S>::R re, typename St<S>::R im) {
    St<S>::st(at32(v.b[b], vidx(y, NC, 0, logW, j)), 0, re, im);
}

// acc -= U v (DAG = false) or acc -= U^H v (DAG = true), u = 3x3 (or 1x1)
// complex matrix as (re, im) pairs in row-major order; four FMAs per
// complex multiply-subtract.
template <typename R, int NC, bool DAG>
__device__ __forceinline__ void mul_sub(const R *u, const R (&vr)[NC], const R (&vi)[NC], R (&ar)[NC], R (&ai)[NC]) {
#pragma unroll
    for (int a = 0; a < NC; ++a) {
#pragma unroll
        for (int b = 0; b < NC; ++b) {
            const int e = DAG ? b * NC + a : a * NC + b;
            const R ur = u[2 * e];
            const R ui = DAG ? -u[2 * e + 1] : u[2 * e + 1];
            ar[a] = fmaR(-ur, vr[b], ar[a]);
            ar[a] = fmaR(ui, vi[b], ar[a]);
            ai[a] = fmaR(-ur, vi[b], ai[a]);
            ai[a] = fmaR(-ui, vr[b], ai[a]);
        }
    }
}

// Stages the neighbour indices of the tile's sites in LDS (the bodies
// without links).  All threads of the workgroup call it; it ends with a
// barrier.
__device__ __forceinline__ void stage_nbr(int *snb, const SiteWalk &wk, int item0, int sites_per_tile,
                                          const int *__restrict__ nbr) {
    const int tid = threadIdx.x;
    __syncthreads();
    for (int e = tid; e < sites_per_tile * 8; e += kBlock)
        snb[e] = item0 + e / 8 < wk.items ? ldg(nbr + walk_site(wk, item0 + e / 8) * 8 + (e & 7)) : 0;
    __syncthreads();
}

// The packed products of one hop on bf16x2 words (low half real, high
// half imaginary), from the stored link word w = (Ur, Ui) and the vector
// word v = (vr, vi): re += dot(w, c1), im += dot(w, c2).  Forward hop
// (U v): c1 = (vr, -vi), c2 = (vi, vr).  Backward hop (U^H v, element (a, b)
// taken from U[b][a]): c1 = v, c2 = (vi, -vr).  The two words are formed once
// per vector word and used for the NC link elements that multiply it; the
// products are those of the complex multiplication, exactly.
__device__ __forceinline__ void hop_vec_words(uint32_t v, bool dag, uint32_t &c1, uint32_t &c2) {
    const uint32_t sw = (v >> 16) | (v << 16);  // (vi, vr)
    c1 = dag ? v : v ^ 0x80000000u;
    c2 = dag ? sw ^ 0x80000000u : sw;
}

// Orders this wavefront's LDS accesses before the call against those after
// it (LDS operations of one wavefront complete in issue order; the fences
// keep the compiler from moving accesses across).
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The tile items a wavefront stages and works on: n items from `first` (in
// the tile) into LDS slots from slot0.  With W <= 64 a wavefront holds 64 / W
// whole lane groups of G items each; with W > 64 a lane group spans W / 64
// wavefronts, which stage a copy each.  slot: the slot of member 0 of this
// thread's lane group.
struct WaveItems {
    int first, n, slot0, slot;
};

__device__ __forceinline__ WaveItems wave_items(int logW, int G) {
    const int tid = threadIdx.x, wv = tid >> 6, sl = tid >> logW;
    WaveItems w;
    if (logW <= 6) {
        w.n = G << (6 - logW);
        w.first = wv * w.n;
        w.slot0 = w.first;
        w.slot = G * sl;
    } else {
        w.n = G;
        w.first = G * sl;
        w.slot0 = wv * G;
        w.slot = w.slot0;
    }
    return w;
}

// Stages the hop links (converted to R) and neighbour indices of the
// wavefront's items item0 + wi.first .. + wi.n - 1 into its LDS slots, by
// that wavefront alone: each wavefront stages what its own threads read, so
// the tile loop takes no workgroup barrier.  Where the LDS layout is the
// memory layout (FP32 and FP64 links) the copy moves 16 bytes per thread.
template <typename LS, typename R, int NC, bool LINKS>
__device__ __forceinline__ void stage_hops_wave(R *su, int *snb, const SiteWalk &wk, int item0, const WaveItems &wi,
                                                const LS *__restrict__ U8, const int *__restrict__ nbr) {
    const int lane = threadIdx.x & 63;
    constexpr int kE = 8 * NC * NC;  // complex link elements of a site
    const int first = item0 + wi.first, n = wi.n;
    wave_fence();  // this wavefront's reads of the previous tile come first
    if (LINKS) {
        if constexpr (sizeof(LS) == 2 * sizeof(R)) {
            constexpr int kV = kE * (int)sizeof(LS) / 16;
            for (int e = lane; e < n * kV; e += 64) {
                const int i = e / kV, k = e - i * kV;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (first + i < wk.items) v = ldg((const uint4 *)(U8 + (size_t)walk_site(wk, first + i) * kE) + k);
                ((uint4 *)(su + (size_t)(wi.slot0 + i) * kE * 2))[k] = v;
            }
        } else {
            for (int e = lane; e < n * kE; e += 64) {
                const int i = e / kE, k = e - i * kE;
                typename St<LS>::R re = 0, im = 0;
                if (first + i < wk.items) St<LS>::ld(U8, (size_t)walk_site(wk, first + i) * kE + k, re, im);
                su[((size_t)(wi.slot0 + i) * kE + k) * 2] = (R)re;
                su[((size_t)(wi.slot0 + i) * kE + k) * 2 + 1] = (R)im;
            }
        }
    }
    for (int e = lane; e < n * 8; e += 64)
        snb[wi.slot0 * 8 + e] = first + e / 8 < wk.items ? ldg(nbr + walk_site(wk, first + e / 8) * 8 + (e & 7)) : 0;
    wave_fence();
}

// Starts the copy of one tile's hop links (as stored, [site][dir][a][b]) and
// neighbour indices into an LDS buffer laid out the same way: the links of
// the tile's sites, then their [site][8] indices.  16-byte loads that write
// LDS directly, without registers, issued by every wavefront for its share
// of the tile.  The copy is complete for this wavefront after its next
// `s_waitcnt vmcnt(0)`, for the workgroup after the barrier that follows it.
// Sites past the walk's end copy site 0 (their values are not used).
template <typename LS, int NC>
__device__ __forceinline__ void dma_tile(void *buf, const SiteWalk &wk, int item0, int sites_per_tile,
                                         const LS *__restrict__ U, const int *__restrict__ nbr) {
    constexpr int kSiteB = 8 * NC * NC * (int)sizeof(LS);  // bytes of a site's hop links
    static_assert(kSiteB % 16 == 0, "a site's hop links are whole 16-byte pieces");
    constexpr int kLC = kSiteB / 16;
    const int nlc = sites_per_tile * kLC, nch = nlc + sites_per_tile * 2;
    const int lane = threadIdx.x & 63;
    for (int c0 = (threadIdx.x >> 6) * 64; c0 < nch; c0 += kBlock) {
        const int c = c0 + lane;
        if (c >= nch) continue;
        const bool link = c < nlc;
        const int s_l = link ? c / kLC : (c - nlc) >> 1;
        const int k = link ? c - s_l * kLC : (c - nlc) & 1;
        const int site = item0 + s_l < wk.items ? walk_site(wk, item0 + s_l) : 0;
        const char *src = link ? (const char *)U + (size_t)site * kSiteB + 16 * k
                               : (const char *)(nbr + (size_t)site * 8) + 16 * k;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)((char *)buf + 16 * c0), 16, 0, 0);
    }
}

// dma_tile with the division of the pieces among the threads taken once:
// thread (wavefront w, lane) copies pieces 64 (w + 4 i) + lane, i < kN, of
// every tile, whose place in a site (piece of its links, or of its
// indices) does not change from tile to tile.
template <typename LS, int NC, int kN>
struct DmaPlan {
    static constexpr int kSiteB = 8 * NC * NC * (int)sizeof(LS);
    static constexpr int kLC = kSiteB / 16;
    int nch;          // pieces of a tile
    int s_l[kN];      // the piece's site in the tile
    int boff[kN];     // its byte offset in the site's links, or -1 - offset in its indices
    __device__ __forceinline__ DmaPlan(int sites_per_tile) {
        static_assert(kSiteB % 16 == 0, "a site's hop links are whole 16-byte pieces");
        const int nlc = sites_per_tile * kLC;
        nch = nlc + sites_per_tile * 2;
        const int c1 = (threadIdx.x >> 6) * 64 + (threadIdx.x & 63);
#pragma unroll
        for (int i = 0; i < kN; ++i) {
            const int c = c1 + i * kBlock;
            const bool link = c < nlc;
            s_l[i] = link ? c / kLC : (c - nlc) >> 1;
            boff[i] = link ? 16 * (c - (c / kLC) * kLC) : -1 - 16 * ((c - nlc) & 1);
        }
    }
    __device__ __forceinline__ void copy(void *buf, const SiteWalk &wk, int item0, const LS *__restrict__ U,
                                         const int *__restrict__ nbr) const {
        const int c1 = (threadIdx.x >> 6) * 64 + (threadIdx.x & 63);
#pragma unroll
        for (int i = 0; i < kN; ++i) {
            const int c0 = (threadIdx.x >> 6) * 64 + i * kBlock;  // uniform in the wavefront
            if (c0 >= nch) break;
            if (c1 + i * kBlock >= nch) continue;
            const int site = item0 + s_l[i] < wk.items ? walk_site(wk, item0 + s_l[i]) : 0;
            const char *src = boff[i] >= 0 ? (const char *)U + (size_t)site * kSiteB + boff[i]
                                           : (const char *)(nbr + (size_t)site * 8) + (-1 - boff[i]);
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)((char *)buf + 16 * c0), 16, 0,
                                             0);
        }
    }
};

// Waits for this wavefront's outstanding vector memory operations (the LDS
// copies above among them), then for the workgroup.
__device__ __forceinline__ void dma_wait_barrier() {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt not waited for
    __syncthreads();
}

// The stencil on BF16-stored vectors and links: every complex product of a
// hop is two packed bf16 dot products accumulated in FP32 (the loaded words
// are used as they are, no unpacking); the modes are those of the generic
// body below.
template <int NC, bool LINKS, int MODE>
__device__ __forceinline__ void k_stencil_bf16_body(const Blk &bk, Launch L, float diag, const bf16x2 *__restrict__ pin,
                                                    const bf16x2 *__restrict__ rin, bf16x2 *__restrict__ q,
                                                    const bf16x2 *__restrict__ U, const int *__restrict__ nbr, int cg,
                                                    Red rd) {
    constexpr bool STAGE = MODE == 1 && LINKS;
    constexpr int kMaxSites = kBlock / 16;
    // STAGE: two tile buffers, each [site][8 NC^2] link words then [site][8]
    // neighbour indices; the next tile is copied into one while the other is
    // read
    constexpr int kBuf = kMaxSites * 8 * NC * NC + kMaxSites * 8;
    constexpr bool kReuse = STAGE && 2 * kBuf * sizeof(uint32_t) >= 4 * kBlock * sizeof(double);
    __shared__ __align__(16) uint32_t su[STAGE ? 2 * kBuf : 1];
    __shared__ int snb[MODE == 1 && !STAGE ? kMaxSites * 8 : 1];
    __shared__ double sm_own[kReuse ? 1 : 4 * kBlock];
    double *sm = kReuse ? (double *)su : sm_own;
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1);
    const int sl = MODE == 2 ? __builtin_amdgcn_readfirstlane(tid >> logW) : tid >> logW;
    const int sites_per_tile = kBlock >> logW;
    const Rows<const bf16x2, NC> P(pin, logW), Rr(rin ? rin : pin, logW);
    const Rows<bf16x2, NC> Q(q, logW);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const SiteWalk wk = site_walk(L, bk);
    // STAGE: the copy of the next tile is in flight while this tile is worked
    // on, so that a tile waits for one round trip to memory rather than two
    // (at most 16 sites of 8 NC^2 + 8 words: two pieces per thread)
    const DmaPlan<bf16x2, NC, 2> plan(sites_per_tile);
    if (STAGE && wk.first * sites_per_tile < wk.items) plan.copy(su, wk, wk.first * sites_per_tile, U, nbr);
    // q of a tile is stored at the start of the next one, after the wait for
    // that tile's copy: the wait (for every outstanding vector memory
    // operation) then does not wait for the stores too
    uint32_t qw[NC];
    unsigned qi = 0;
    bool qpend = false;
    auto store_q = [&]() {
        if (!qpend) return;
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            bf16x2 o;
            o.v = qw[a];
            stg(at32(Q.b[a], qi), o);
        }
        qpend = false;
    };
    int cur = 0;
    for (int t = wk.first; t * sites_per_tile < wk.items; t += wk.stride, cur ^= 1) {
        const int item0 = t * sites_per_tile;
        const uint32_t *lw = su + cur * kBuf;                       // this tile's link words
        const int *tnb = (const int *)lw + sites_per_tile * 8 * NC * NC;  // and neighbour indices
        if (STAGE) {
            // this tile's copy is complete, and every wavefront is done with the other buffer
            dma_wait_barrier();
            store_q();
            const int next0 = (t + wk.stride) * sites_per_tile;
            if (next0 < wk.items) plan.copy(su + (cur ^ 1) * kBuf, wk, next0, U, nbr);
        } else {
            store_q();
            if (MODE == 1) stage_nbr(snb, wk, item0, sites_per_tile, nbr);
        }
        if (item0 + sl >= wk.items) continue;
        const int site = walk_site(wk, item0 + sl);
        int y[9];
        y[0] = site;
#pragma unroll
        for (int dir = 0; dir < 8; ++dir)
            y[dir + 1] = STAGE ? tnb[sl * 8 + dir] : (MODE == 1 ? snb[sl * 8 + dir] : ldg(nbr + site * 8 + dir));
        uint32_t v[9][NC];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const unsigned i = vidx(y[k], NC, 0, logW, j);
#pragma unroll
            for (int b = 0; b < NC; ++b) v[k][b] = ldg(at32(P.b[b], i)).v;
        }
        uint32_t rv[NC];  // the residual at the site (CG: r^H q and r^H p summed here)
        if (cg) {
            const unsigned i = vidx(site, NC, 0, logW, j);
#pragma unroll
            for (int b = 0; b < NC; ++b) rv[b] = ldg(at32(Rr.b[b], i)).v;
        }
        float hr[NC], hi[NC];  // sum of the hops
#pragma unroll
        for (int a = 0; a < NC; ++a) hr[a] = hi[a] = 0.0f;
#pragma unroll
        for (int dir = 0; dir < 8; ++dir) {
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                if (!LINKS) {
                    hr[b] += __uint_as_float(v[dir + 1][b] << 16);
                    hi[b] += __uint_as_float(v[dir + 1][b] & 0xffff0000u);
                    continue;
                }
                uint32_t c1, c2;
                hop_vec_words(v[dir + 1][b], dir >= 4, c1, c2);
#pragma unroll
                for (int a = 0; a < NC; ++a) {
                    const int el = dir < 4 ? a * NC + b : b * NC + a;
                    const uint32_t w = STAGE ? lw[(sl * 8 + dir) * NC * NC + el]
                                             : ldg(U + ((size_t)site * 8 + dir) * NC * NC + el).v;
                    hr[a] = dot2_bf16(w, c1, hr[a]);
                    hi[a] = dot2_bf16(w, c2, hi[a]);
                }
            }
        }
        float pqs = 0, rqs = 0, qqs = 0, rps = 0;
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            const float pr = __uint_as_float(v[0][a] << 16), pi = __uint_as_float(v[0][a] & 0xffff0000u);
            const float ar = fmaf(diag, pr, -hr[a]), ai = fmaf(diag, pi, -hi[a]);
            bf16x2 o;
            o.v = pack_bf16(ar, ai);
            qw[a] = o.v;
            if (cg) {
                // the real parts of the dot products of the stored words (the
                // rounded q): one packed dot each, the products exact in FP32
                pqs = dot2_bf16(v[0][a], o.v, pqs);
                qqs = dot2_bf16(o.v, o.v, qqs);
                rqs = dot2_bf16(rv[a], o.v, rqs);
                rps = dot2_bf16(rv[a], v[0][a], rps);
            }
        }
        qi = vidx(site, NC, 0, logW, j);
        qpend = true;
        acc[0] += (double)pqs;
        acc[1] += (double)rqs;
        acc[2] += (double)qqs;
        acc[3] += (double)rps;
    }
    store_q();
    if (!cg) return;
    if (kReuse) __syncthreads();  // every wavefront is done with the link tile
    block_partials<4>(bk, acc, W, logW, rd, sm);
}

// hop link dir of site from the hop-link array, converted to R
template <typename LS, typename R, int NC>
__device__ __forceinline__ void ld_hop(const LS *__restrict__ U8, int site, int dir, R *u) {
    const LS *base = U8 + ((size_t)site * 8 + dir) * NC * NC;
#pragma unroll
    for (int e = 0; e < NC * NC; ++e) {
        typename St<LS>::R re, im;
        St<LS>::ld(base, e, re, im);
        u[2 * e] = (R)re;
        u[2 * e + 1] = (R)im;
    }
}

// The stencil q = A p for one block of right-hand sides, with p^H q summed
// per lane when `cg` is set (the first kernel of a CG iteration).
//
// MODE 0 (W < 16): every lane loads its site's links itself (the lanes of a
// site read the same addresses); for W = 1 (FP64, FP32) MODE 5 instead
// splits a site over 32 threads (k_stencil_split_body).  MODE 1 (16 <= W < 64): the links of the
// tile's sites are staged in LDS once and shared by the W lanes.  MODE 2
// (W >= 64): a wavefront covers one site, so the site index is uniform and
// the links and neighbour indices come through scalar loads; no LDS and no
// barriers.  MODES 3 and 4 (16 <= W < 64 with even x0-slabs) are MODE 1
// with two or four neighbouring sites per thread (k_stencil_group_body).  In every mode the vector loads of the site and its eight
// neighbours are issued before any arithmetic, so they are in flight
// together.
template <typename S, typename LS, int NC, bool LINKS, int MODE>
__device__ __forceinline__ void k_stencil_body(const Blk &bk, Launch L, typename St<S>::R diag, const S *__restrict__ pin,
                                               const S *__restrict__ rin, S *__restrict__ q, const LS *__restrict__ U,
                                               const int *__restrict__ nbr, int cg, Red rd) {
    if constexpr (std::is_same<S, bf16x2>::value) {
        k_stencil_bf16_body<NC, LINKS, MODE>(bk, L, diag, pin, rin, q, U, nbr, cg, rd);
        return;
    }
    using R = typename St<S>::R;
    constexpr bool STAGE = MODE == 1 && LINKS;
    constexpr int kMaxSites = kBlock / 16;
    // the reduction at the end reuses the link tile when there is one
    constexpr bool kReuse = STAGE && kMaxSites * 8 * NC * NC * 2 * sizeof(R) >= 4 * kBlock * sizeof(double);
    __shared__ __align__(16) R su[STAGE ? kMaxSites * 8 * NC * NC * 2 : 1];
    __shared__ int snb[MODE == 1 ? kMaxSites * 8 : 1];
    __shared__ double sm_own[kReuse ? 1 : 4 * kBlock];
    double *sm = kReuse ? (double *)su : sm_own;
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1);
    const int sl = MODE == 2 ? __builtin_amdgcn_readfirstlane(tid >> logW) : tid >> logW;
    const int sites_per_tile = kBlock >> logW;
    const WaveItems wi = wave_items(logW, 1);
    const Rows<const S, NC> P(pin, logW);
    const Rows<S, NC> Q(q, logW);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const SiteWalk wk = site_walk(L, bk);
    for (int t = wk.first; t * sites_per_tile < wk.items; t += wk.stride) {
        const int item0 = t * sites_per_tile;
        if (MODE == 1) stage_hops_wave<LS, R, NC, LINKS>(su, snb, wk, item0, wi, U, nbr);
        if (item0 + sl >= wk.items) continue;
        const int site = walk_site(wk, item0 + sl);
        int y[9];
        y[0] = site;
#pragma unroll
        for (int dir = 0; dir < 8; ++dir) y[dir + 1] = MODE == 1 ? snb[wi.slot * 8 + dir] : ldg(nbr + site * 8 + dir);
        R vr[9][NC], vi[9][NC];
#pragma unroll
        for (int k = 0; k < 9; ++k) ld_rows<S, NC>(P, y[k], logW, j, vr[k], vi[k]);
        R ar[NC], ai[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            ar[a] = diag * vr[0][a];
            ai[a] = diag * vi[0][a];
        }
#pragma unroll
        for (int dir = 0; dir < 8; ++dir) {
            if (!LINKS) {
#pragma unroll
                for (int a = 0; a < NC; ++a) {
                    ar[a] -= vr[dir + 1][a];
                    ai[a] -= vi[dir + 1][a];
                }
                continue;
            }
            R u[2 * NC * NC];
            if (STAGE) {
#pragma unroll
                for (int e = 0; e < 2 * NC * NC; ++e) u[e] = su[(wi.slot * 8 + dir) * NC * NC * 2 + e];
            } else {
                ld_hop<LS, R, NC>(U, site, dir, u);
            }
            if (dir < 4)
                mul_sub<R, NC, false>(u, vr[dir + 1], vi[dir + 1], ar, ai);
            else
                mul_sub<R, NC, true>(u, vr[dir + 1], vi[dir + 1], ar, ai);
        }
        R pqs = 0, qqs = 0;
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            st_rows<S, NC>(Q, site, logW, j, a, ar[a], ai[a]);
            if (cg) {
                pqs = fmaR(vr[0][a], ar[a], fmaR(vi[0][a], ai[a], pqs));
                qqs = fmaR(ar[a], ar[a], fmaR(ai[a], ai[a], qqs));
            }
        }
        acc[0] += (double)pqs;
        acc[2] += (double)qqs;
    }
    if (!cg) return;
    if (kReuse) __syncthreads();  // every wavefront is done with the link tile
    block_partials<4>(bk, acc, W, logW, rd, sm);
}

// MODES 3 and 4: MODE 1 with G sites per thread that are each other's
// neighbours, so the shared neighbours are loaded once.  When every XCD's
// slab has an even number of x0-slices, the slab walk (x0 fastest) puts the
// x0-slices of a pair at consecutive items: with G = 2 a thread takes items
// 2i, 2i + 1, sites s and s + V3 (x0 neighbours): 16 site loads per pair
// instead of 18.  With two slices per slab and an even D3, items 4i .. 4i + 3
// are s, s + V3, s + 1, s + V3 + 1 (x0 and x3 neighbours; 4i / 2 is even,
// so x3 + 1 does not wrap): 28 loads per quad instead of 36.  16^4, FP32,
// W = 32: 45.1 us (G = 1), 41.6 (G = 2), 40.6 (G = 4).  With a multiple of
// four slices per slab (MODE 6, LINE), items 4i .. 4i + 3 are four
// consecutive x0-slices of one (x1, x2, x3): s + h V3, 30 loads per four
// sites instead of 32 with pairs.
template <int G, bool LINE>
__device__ __forceinline__ int group_nb(int h, int dir) {
    // the group member that is neighbour dir of member h, or -1
    if (LINE) return (dir == 0 && h < G - 1) ? h + 1 : (dir == 4 && h > 0) ? h - 1 : -1;
    if (G == 2) return (h == 0 && dir == 0) ? 1 : (h == 1 && dir == 4) ? 0 : -1;
    switch (h * 8 + dir) {
        case 0 * 8 + 0: return 1;
        case 0 * 8 + 3: return 2;
        case 1 * 8 + 4: return 0;
        case 1 * 8 + 3: return 3;
        case 2 * 8 + 0: return 3;
        case 2 * 8 + 7: return 0;
        case 3 * 8 + 4: return 2;
        case 3 * 8 + 7: return 1;
        default: return -1;
    }
}

template <typename S, typename LS, int NC, bool LINKS, int G, bool LINE = false>
__device__ __forceinline__ void k_stencil_group_body(const Blk &bk, Launch L, typename St<S>::R diag,
                                                     const S *__restrict__ pin, const S *__restrict__ rin,
                                                     S *__restrict__ q, const LS *__restrict__ U,
                                                     const int *__restrict__ nbr, int cg, Red rd) {
    using R = typename St<S>::R;
    // BF16 storage (FP32 arithmetic on the unpacked values here) sums r^H q
    // and r^H p itself, like the packed BF16 body
    constexpr bool kDirect = std::is_same<S, bf16x2>::value;
    // (pairs need W >= 16, quads and lines W >= 32: at most 32 items per tile)
    constexpr int kMaxItems = G == 2 ? 2 * (kBlock / 16) : 4 * (kBlock / 32);
    // the reduction at the end reuses the link tile when it is large enough
    constexpr bool kReuse = LINKS && kMaxItems * 8 * NC * NC * 2 * sizeof(R) >= 4 * kBlock * sizeof(double);
    __shared__ __align__(16) R su[LINKS ? kMaxItems * 8 * NC * NC * 2 : 1];
    __shared__ int snb[kMaxItems * 8];
    __shared__ double sm_own[kReuse ? 1 : 4 * kBlock];
    double *sm = kReuse ? (double *)su : sm_own;
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1);
    const int sl = tid >> logW;
    const int items_per_tile = G * (kBlock >> logW);
    const WaveItems wi = wave_items(logW, G);
    const Rows<const S, NC> P(pin, logW), Rr(kDirect && rin ? rin : pin, logW);
    const Rows<S, NC> Q(q, logW);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const SiteWalk wk = site_walk(L, bk);
    for (int t = wk.first; t * items_per_tile < wk.items; t += wk.stride) {
        const int item0 = t * items_per_tile;
        stage_hops_wave<LS, R, NC, LINKS>(su, snb, wk, item0, wi, U, nbr);
        if (item0 + G * sl >= wk.items) continue;
        const int s0 = walk_site(wk, item0 + G * sl);
        R vor[G][NC], voi[G][NC];  // the members' own vectors
#pragma unroll
        for (int h = 0; h < G; ++h)
            ld_rows<S, NC>(P, s0 + (LINE ? h * wk.V3 : (h & 1) * wk.V3 + (h >> 1)), logW, j, vor[h], voi[h]);
        R pqs = 0, qqs = 0, rqs = 0, rps = 0;
#pragma unroll
        for (int h = 0; h < G; ++h) {
            const int ls = wi.slot + h;
            const int site = s0 + (LINE ? h * wk.V3 : (h & 1) * wk.V3 + (h >> 1));
            R rr_[NC], ri_[NC];  // BF16 storage: the residual (r^H q, r^H p summed here)
            if (kDirect && cg) ld_rows<S, NC>(Rr, site, logW, j, rr_, ri_);
            R vr[8][NC], vi[8][NC];
#pragma unroll
            for (int dir = 0; dir < 8; ++dir) {
                const int m = group_nb<G, LINE>(h, dir);
                if (m >= 0) {
#pragma unroll
                    for (int b = 0; b < NC; ++b) {
                        vr[dir][b] = vor[m][b];
                        vi[dir][b] = voi[m][b];
                    }
                } else {
                    ld_rows<S, NC>(P, snb[ls * 8 + dir], logW, j, vr[dir], vi[dir]);
                }
            }
            R ar[NC], ai[NC];
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                ar[a] = diag * vor[h][a];
                ai[a] = diag * voi[h][a];
            }
#pragma unroll
            for (int dir = 0; dir < 8; ++dir) {
                if (!LINKS) {
#pragma unroll
                    for (int a = 0; a < NC; ++a) {
                        ar[a] -= vr[dir][a];
                        ai[a] -= vi[dir][a];
                    }
                    continue;
                }
                R u[2 * NC * NC];
#pragma unroll
                for (int e = 0; e < 2 * NC * NC; ++e) u[e] = su[(ls * 8 + dir) * NC * NC * 2 + e];
                if (dir < 4)
                    mul_sub<R, NC, false>(u, vr[dir], vi[dir], ar, ai);
                else
                    mul_sub<R, NC, true>(u, vr[dir], vi[dir], ar, ai);
            }
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                st_rows<S, NC>(Q, site, logW, j, a, ar[a], ai[a]);
                if (cg) {
                    R qr = ar[a], qi = ai[a];
                    St<S>::round(qr, qi);  // the dot products of the stored q
                    pqs = fmaR(vor[h][a], qr, fmaR(voi[h][a], qi, pqs));
                    qqs = fmaR(qr, qr, fmaR(qi, qi, qqs));
                    if (kDirect) {
                        rqs = fmaR(rr_[a], qr, fmaR(ri_[a], qi, rqs));
                        rps = fmaR(rr_[a], vor[h][a], fmaR(ri_[a], voi[h][a], rps));
                    }
                }
            }
        }
        acc[0] += (double)pqs;
        acc[1] += (double)rqs;
        acc[2] += (double)qqs;
        acc[3] += (double)rps;
    }
    if (!cg) return;
    if (kReuse) __syncthreads();  // every wavefront is done with the link tile
    block_partials<4>(bk, acc, W, logW, rd, sm);
}

// MODE 5 (W = 1): one right-hand side leaves a launch with one thread per
// site too few threads to fill the GPU (an 8^4 lattice: 16 workgroups), so
// a site takes 32 threads: thread (h, a) = (lane / 4, lane % 4) forms row a
// of hop h's product U v (rows a >= nc idle), the eight hops of a row are
// summed by a butterfly over lanes 4, 8 and 16 apart, and hop 0's threads
// write q.  Eight sites per workgroup pass.
template <typename S, typename LS, int NC, bool LINKS>
__device__ __forceinline__ void k_stencil_split_body(const Blk &bk, Launch L, typename St<S>::R diag,
                                                     const S *__restrict__ pin, const S *__restrict__ rin,
                                                     S *__restrict__ q, const LS *__restrict__ U,
                                                     const int *__restrict__ nbr, int cg, Red rd) {
    using R = typename St<S>::R;
    __shared__ double sm[4 * kBlock];
    const int tid = threadIdx.x, lane = tid & 31, h = lane >> 2, a = lane & 3;
    const int ngroups = (L.lat.N + 7) / 8;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = bk.b; g < ngroups; g += bk.nb) {
        const int site = g * 8 + (tid >> 5);
        const bool live = site < L.lat.N;
        R sr = 0, si = 0;
        if (live && a < NC) {
            const int y = nbr[site * 8 + h];
            if (LINKS) {
                // row a of U_mu(x) (h < 4) or of U_mu(x - mu)^H (h >= 4)
                const LS *u = U + ((size_t)site * 8 + h) * NC * NC;
#pragma unroll
                for (int b = 0; b < NC; ++b) {
                    typename St<LS>::R ur, ui;
                    St<LS>::ld(u, h < 4 ? a * NC + b : b * NC + a, ur, ui);
                    if (h >= 4) ui = -ui;
                    R vr, vi;
                    St<S>::ld(pin, (size_t)y * NC + b, vr, vi);
                    sr = fmaR((R)ur, vr, fmaR(-(R)ui, vi, sr));
                    si = fmaR((R)ur, vi, fmaR((R)ui, vr, si));
                }
            } else {
                St<S>::ld(pin, (size_t)y * NC + a, sr, si);
            }
        }
#pragma unroll
        for (int off = 4; off < 32; off <<= 1) {
            sr += __shfl_xor(sr, off, 64);
            si += __shfl_xor(si, off, 64);
        }
        if (live && h == 0 && a < NC) {
            R pr, pi;
            St<S>::ld(pin, (size_t)site * NC + a, pr, pi);
            R qr = fmaR(diag, pr, -sr), qi = fmaR(diag, pi, -si);
            St<S>::st(q, (size_t)site * NC + a, qr, qi);
            if (cg) {
                acc[0] += (double)fmaR(pr, qr, pi * qi);
                acc[2] += (double)fmaR(qr, qr, qi * qi);
            }
        }
    }
    if (!cg) return;
    block_partials<4>(bk, acc, 1, 0, rd, sm);
}

template <typename S, typename LS, int NC, bool LINKS, int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil(Launch L, typename St<S>::R diag, const S *__restrict__ pin,
                                                    const S *__restrict__ rin, S *__restrict__ q,
                                                    const LS *__restrict__ U, const int *__restrict__ nbr, int cg,
                                                    Red rd) {
    // the bodies are inlined once with cg = 1 and once with cg = 0: with a
    // run-time flag the compiler keeps the registers of both paths live
    // (the BF16 body went from 69 to 187 registers)
    auto body = [&](int cg_) {
        if constexpr (MODE == 3 || MODE == 4)
            k_stencil_group_body<S, LS, NC, LINKS, MODE == 3 ? 2 : 4>(own_blk(), L, diag, pin, rin, q, U, nbr, cg_,
                                                                      rd);
        else if constexpr (MODE == 6)
            k_stencil_group_body<S, LS, NC, LINKS, 4, true>(own_blk(), L, diag, pin, rin, q, U, nbr, cg_, rd);
        else if constexpr (MODE == 5)
            k_stencil_split_body<S, LS, NC, LINKS>(own_blk(), L, diag, pin, rin, q, U, nbr, cg_, rd);
        else
            k_stencil_body<S, LS, NC, LINKS, MODE>(own_blk(), L, diag, pin, rin, q, U, nbr, cg_, rd);
    };
    if (cg)
        body(1);
    else
        body(0);
}

// The vector update of a CG iteration (second kernel; alpha and beta from
// the finishing kernel): x += alpha p, r -= alpha q, p = r + beta p, and
// |r|^2 and Re q^H p of the new residual and direction as stored (the next
// finishing kernel adds the partials up).  A held or stopped lane keeps its
// direction (alpha = 0: x and r are unchanged too).
// The solution's update x += alpha p can be taken two iterations at a time
// (XM; FP32 or BF16 storage): an update with XM = 1 leaves x and records
// c = alpha_k / beta_k per lane; the next one (XM = 2) recovers the direction
// p_k it skipped from the two vectors it reads anyway, p_k = (p_{k+1} -
// r_{k+1}) / beta_k (the relation by which the skipped update formed p_{k+1}),
// and adds alpha_k p_k + alpha_{k+1} p_{k+1} in one read and write of x: six
// vector passes per iteration on average instead of seven.  The recovery
// divides by beta_k; its rounding error relative to alpha_k p_k is about
// eps / sqrt(beta_k) (|r_{k+1}| = sqrt(beta_k) |r_k| <= sqrt(beta_k) |p_k|),
// so a lane whose beta_k is below kDeferBetaMin (a restart has beta = 0)
// updates its x at once instead.  With BF16 storage the rounding of the
// stored p_{k+1} (2^-9 of it) enters the same way, about 2^-9 (1 + 1 /
// sqrt(beta_k)) of the step, against 2^-9 of the whole accumulated x that
// every BF16 write of x costs (and the pairs halve those writes); there the
// floor is 1/16 (at most 5 x 2^-9 of a step).  XM = 0 is the plain update.
// An XM = 1 update is always followed by an XM = 2 one before anything
// reads x.
template <typename S>
constexpr double kDeferBetaMin = std::is_same<S, bf16x2>::value ? 1.0 / 16 : 1.0 / 64;

template <typename S, int XM>
__device__ __forceinline__ void k_update_body(const Blk &bk, Launch L, S *__restrict__ x, S *__restrict__ r,
                                              S *__restrict__ p, const S *__restrict__ q, Red rd, CgState cs) {
    using R = typename St<S>::R;
    __shared__ double sm[2 * kBlock];
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1);
    const int sites_per_tile = kBlock >> logW;
    const R alpha = (R)ldg(cs.alpha + j);
    const double beta64 = ldg(cs.beta + j);
    const R beta = (R)beta64;
    const bool keep = (ldg(cs.flags + j) & kFlagHold) || !ldg(cs.active + j);
    // XM = 1: does this lane defer its x update (else it updates x now)?
    // XM = 2: the deferred coefficient alpha_k / beta_k (0: nothing deferred)
    const bool dfr = XM == 1 && !keep && beta64 >= kDeferBetaMin<S>;
    const bool xio = XM != 1 || (!keep && !dfr);
    const R cdef = XM == 2 ? (R)ldg(cs.xdef + j) : (R)0;
    if (XM == 1 && bk.b == 0 && tid < W) cs.xdef[j] = dfr ? ldg(cs.alpha + j) / beta64 : 0.0;
    double acc[2] = {0.0, 0.0};
    int t0, t1;
    tile_range(bk, L.ntiles, t0, t1);
    // element e = ((site * nc + a) << logW) + j: lane j is tid & (W-1) for
    // every e = e0 + tid + k * kBlock since kBlock is a multiple of W
    const size_t e0 = (size_t)t0 * sites_per_tile * L.nc * W;
    const size_t e1 = min((size_t)t1 * sites_per_tile, (size_t)L.lat.N) * L.nc * W;
    R part = 0, partq = 0;
    int cnt = 0;
    size_t e = e0 + tid;
    // four elements per pass, all loads issued before the first use (more
    // loads in flight per wavefront); the same summation order as the
    // element-by-element tail below; no branch inside (a kept direction is
    // stored back unchanged: a loaded value is stored exactly)
    for (; e + 3 * kBlock < e1; e += 4 * kBlock) {
        R xr[4], xi[4], rr_[4], ri[4], pr[4], pi[4], qr[4], qi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            St<S>::ld(p, e + u * kBlock, pr[u], pi[u]);
            St<S>::ld(q, e + u * kBlock, qr[u], qi[u]);
            St<S>::ld(r, e + u * kBlock, rr_[u], ri[u]);
            if (xio) St<S>::ld(x, e + u * kBlock, xr[u], xi[u]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (XM == 2) {
                xr[u] = fmaR(cdef, pr[u] - rr_[u], xr[u]);
                xi[u] = fmaR(cdef, pi[u] - ri[u], xi[u]);
            }
            if (xio) St<S>::st(x, e + u * kBlock, fmaR(alpha, pr[u], xr[u]), fmaR(alpha, pi[u], xi[u]));
            rr_[u] = fmaR(-alpha, qr[u], rr_[u]);
            ri[u] = fmaR(-alpha, qi[u], ri[u]);
            St<S>::st(r, e + u * kBlock, rr_[u], ri[u]);
            // the next iteration uses the stored (rounded) residual
            St<S>::round(rr_[u], ri[u]);
            R npr = keep ? pr[u] : fmaR(beta, pr[u], rr_[u]), npi = keep ? pi[u] : fmaR(beta, pi[u], ri[u]);
            St<S>::st(p, e + u * kBlock, npr, npi);
            St<S>::round(npr, npi);
            part = fmaR(rr_[u], rr_[u], fmaR(ri[u], ri[u], part));
            partq = fmaR(qr[u], npr, fmaR(qi[u], npi, partq));
        }
        if ((cnt += 4) == 24) {
            acc[0] += (double)part;
            acc[1] += (double)partq;
            part = partq = 0;
            cnt = 0;
        }
    }
    for (; e < e1; e += kBlock) {
        R xr, xi, rr_, ri, pr, pi, qr, qi;
        St<S>::ld(p, e, pr, pi);
        St<S>::ld(q, e, qr, qi);
        St<S>::ld(r, e, rr_, ri);
        if (xio) St<S>::ld(x, e, xr, xi);
        if (XM == 2) {
            xr = fmaR(cdef, pr - rr_, xr);
            xi = fmaR(cdef, pi - ri, xi);
        }
        if (xio) St<S>::st(x, e, fmaR(alpha, pr, xr), fmaR(alpha, pi, xi));
        rr_ = fmaR(-alpha, qr, rr_);
        ri = fmaR(-alpha, qi, ri);
        St<S>::st(r, e, rr_, ri);
        St<S>::round(rr_, ri);
        R npr = keep ? pr : fmaR(beta, pr, rr_), npi = keep ? pi : fmaR(beta, pi, ri);
        St<S>::st(p, e, npr, npi);
        St<S>::round(npr, npi);
        part = fmaR(rr_, rr_, fmaR(ri, ri, part));
        partq = fmaR(qr, npr, fmaR(qi, npi, partq));
        if (++cnt == 24) {
            acc[0] += (double)part;
            acc[1] += (double)partq;
            part = partq = 0;
            cnt = 0;
        }
    }
    acc[0] += (double)part;
    acc[1] += (double)partq;
    // a kept direction keeps the Re q_prev^H p of the update that formed it
    // (the q loaded here is A of the kept direction itself): its total comes
    // back from cs.qp, once per lane
    if (keep) acc[1] = (bk.b == 0 && tid < W) ? ldg(cs.qp + j) : 0.0;
    block_partials_to<2>(bk, acc, W, logW, rd.part2, rd.nblk, sm);
}

template <typename S, int XM>
__global__ __launch_bounds__(kBlock) void k_update(Launch L, S *__restrict__ x, S *__restrict__ r,
                                                   S *__restrict__ p, const S *__restrict__ q, Red rd, CgState cs) {
    k_update_body<S, XM>(own_blk(), L, x, r, p, q, rd, cs);
}

// Mixed precision: x64 += xlo, xlo = 0 (the low-precision iterate folded
// into the FP64 solution before a reliable update).
template <typename S>
__device__ __forceinline__ void k_fold_body(const Blk &bk, Launch L, double2 *__restrict__ x64, S *__restrict__ xlo) {
    using R = typename St<S>::R;
    const int tid = threadIdx.x, W = L.W;
    const int sites_per_tile = kBlock >> L.logW;
    int t0, t1;
    tile_range(bk, L.ntiles, t0, t1);
    const size_t e0 = (size_t)t0 * sites_per_tile * L.nc * W;
    const size_t e1 = min((size_t)t1 * sites_per_tile, (size_t)L.lat.N) * L.nc * W;
    for (size_t e = e0 + tid; e < e1; e += kBlock) {
        R xr, xi;
        St<S>::ld(xlo, e, xr, xi);
        double2 v = x64[e];
        v.x += (double)xr;
        v.y += (double)xi;
        St<S>::st(xlo, e, 0, 0);
        x64[e] = v;
    }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_fold(Launch L, double2 *__restrict__ x64, S *__restrict__ xlo) {
    k_fold_body<S>(own_blk(), L, x64, xlo);
}

// FP64 true residual r_new = b - A x64 with the FP64 hop links, |r_new|^2 per
// lane into rd.part2.  ru (a reliable update): r_new replaces the residual in the
// storage precision; a lane flagged to restart takes r_new as its direction.
// The other directions: FP32 storage continues them as p + (r_new - r_old),
// the direction the last update would have formed from r_new (so that
// r = p - beta p_prev still holds exactly for the finishing kernel), and
// sums Re q^H p of it (q = A p_prev, still in qin) beside |r_new|^2; BF16
// storage keeps them (residual replacement; its finishing kernel takes the
// exact line search along p) and writes the lane's total cs.qp back.
// Otherwise (statistics) nothing is written but the norm.
template <typename S, int NC, bool LINKS, int MODE>
__device__ __forceinline__ void k_true_resid_body(const Blk &bk, Launch L, double diag, const double2 *__restrict__ b64,
                                                  const double2 *__restrict__ x64, const double2 *__restrict__ U,
                                                  const int *__restrict__ nbr, S *__restrict__ rout,
                                                  S *__restrict__ pio, const S *__restrict__ qin, int ru, Red rd,
                                                  CgState cs, ProbeGen g, int gen) {
    constexpr int kMaxSites = kBlock / 16;
    // STAGE: two tile buffers, each the tile's hop links then its neighbour
    // indices; the next tile is copied into one while the other is read
    constexpr bool STAGE = MODE == 1 && LINKS;
    constexpr int kBufB = kMaxSites * 8 * NC * NC * 16 + kMaxSites * 8 * 4;
    __shared__ __align__(16) char sbuf[STAGE ? 2 * kBufB : 16];
    __shared__ int snb[MODE == 1 && !STAGE ? kMaxSites * 8 : 1];
    // the reduction at the end reuses the tile buffers when there are any
    __shared__ double sm_own[STAGE ? 1 : 2 * kBlock];
    double *sm = STAGE ? (double *)sbuf : sm_own;
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1);
    const int sl = MODE == 2 ? __builtin_amdgcn_readfirstlane(tid >> logW) : tid >> logW;
    const int sites_per_tile = kBlock >> logW;
    double acc[2] = {0.0, 0.0};
    const SiteWalk wk = site_walk(L, bk);
    const unsigned long long seedmix = gen ? mix64(g.seed) : 0ull;
    const ProbeLane pl = gen ? probe_lane(g, NC, g.rhs0 + j) : ProbeLane{};
    const bool restart = ru && (cs.flags[j] & kFlagRestart);
    if (STAGE && wk.first * sites_per_tile < wk.items)
        dma_tile<double2, NC>(sbuf, wk, wk.first * sites_per_tile, sites_per_tile, U, nbr);
    int cur = 0;
    for (int t = wk.first; t * sites_per_tile < wk.items; t += wk.stride, cur ^= 1) {
        const double *tsu = (const double *)(sbuf + cur * kBufB);  // this tile's hop links
        const int *tnb = (const int *)(sbuf + cur * kBufB + sites_per_tile * 8 * NC * NC * 16);
        if (STAGE) {
            // this tile's copy is complete, and every wavefront is done with the other buffer
            dma_wait_barrier();
            const int next0 = (t + wk.stride) * sites_per_tile;
            if (next0 < wk.items) dma_tile<double2, NC>(sbuf + (cur ^ 1) * kBufB, wk, next0, sites_per_tile, U, nbr);
        } else if (MODE == 1) {
            stage_nbr(snb, wk, t * sites_per_tile, sites_per_tile, nbr);
        }
        if (t * sites_per_tile + sl >= wk.items) continue;
        const int site = walk_site(wk, t * sites_per_tile + sl);
        int y[9];
        y[0] = site;
#pragma unroll
        for (int dir = 0; dir < 8; ++dir)
            y[dir + 1] = STAGE ? tnb[sl * 8 + dir] : (MODE == 1 ? snb[sl * 8 + dir] : ldg(nbr + site * 8 + dir));
        // Two halves: the site and its forward neighbours, then the backward
        // ones, each half's loads in flight together before its arithmetic
        // (all nine at once hold 108 registers of FP64 values: two waves per
        // SIMD instead of four)
        double vr[5][NC], vi[5][NC], br[NC], bi[NC];
#pragma unroll
        for (int k = 0; k < 5; ++k) ld_site<double2, NC>(x64, y[k], logW, j, vr[k], vi[k]);
        if (gen) {
            // probes are regenerated instead of read back (exact values)
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                br[a] = bi[a] = 0.0;
                if (j < g.nvalid) probe_at(g, seedmix, L.lat, NC, pl, site, a, br[a], bi[a]);
            }
        } else {
            ld_site<double2, NC>(b64, site, logW, j, br, bi);
        }
        // r = b - diag x + sum of hops: accumulated with the sign flipped
        double ar[NC], ai[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            ar[a] = -fma(-diag, vr[0][a], br[a]);
            ai[a] = -fma(-diag, vi[0][a], bi[a]);
        }
#pragma unroll
        for (int dir = 0; dir < 8; ++dir) {
            if (dir == 4) {
                // the backward half: its loads wait until the forward values are spent
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 1; k < 5; ++k) ld_site<double2, NC>(x64, y[k + 4], logW, j, vr[k], vi[k]);
            }
            const int k = (dir & 3) + 1;
            if (!LINKS) {
#pragma unroll
                for (int a = 0; a < NC; ++a) {
                    ar[a] -= vr[k][a];
                    ai[a] -= vi[k][a];
                }
                continue;
            }
            double u[2 * NC * NC];
            if (STAGE) {
#pragma unroll
                for (int e = 0; e < 2 * NC * NC; ++e) u[e] = tsu[(sl * 8 + dir) * NC * NC * 2 + e];
            } else {
                ld_hop<double2, double, NC>(U, site, dir, u);
            }
            if (dir < 4)
                mul_sub<double, NC, false>(u, vr[k], vi[k], ar, ai);
            else
                mul_sub<double, NC, true>(u, vr[k], vi[k], ar, ai);
        }
        if (ru) {
            using R = typename St<S>::R;
            // (the neighbours' registers are free from here on)
            __builtin_amdgcn_sched_barrier(0);
            S *rrow = rout + ((size_t)(site * NC) << logW);
            S *prow = pio + ((size_t)(site * NC) << logW);
            const S *qrow = qin + ((size_t)(site * NC) << logW);
#pragma unroll
            for (int a = 0; a < NC; ++a) {
                const size_t i = ((size_t)a << logW) + j;
                R nr = (R)(-ar[a]), ni = (R)(-ai[a]);
                if (cs.rq_direct) {
                    St<S>::st(rrow, i, nr, ni);
                    if (restart) St<S>::st(prow, i, nr, ni);
                } else {
                    R ro_r, ro_i, po_r, po_i, qr, qi;
                    St<S>::ld(rrow, i, ro_r, ro_i);
                    St<S>::ld(prow, i, po_r, po_i);
                    St<S>::ld(qrow, i, qr, qi);
                    St<S>::st(rrow, i, nr, ni);
                    St<S>::round(nr, ni);
                    R npr = restart ? nr : po_r + (nr - ro_r), npi = restart ? ni : po_i + (ni - ro_i);
                    St<S>::st(prow, i, npr, npi);
                    St<S>::round(npr, npi);
                    acc[1] += (double)(qr * npr + qi * npi);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < NC; ++a) acc[0] += ar[a] * ar[a] + ai[a] * ai[a];
    }
    if (ru && cs.rq_direct) acc[1] = (bk.b == 0 && tid < W) ? cs.qp[j] : 0.0;
    if (STAGE) __syncthreads();  // every wavefront is done with the tile buffers
    block_partials_to<2>(bk, acc, W, logW, rd.part2, rd.nblk, sm);
}


// The true residual from q64 = A x64 (the FP64 stencil, run just before on
// x64 with the FP64 hop links): r = b - q64 in FP64 element by element, with
// |r|^2 summed; with ru the inner-precision residual and direction are
// replaced as in k_true_resid_body (the FP32 continuation p += r_new - r,
// or p = r_new for a restarting lane) and Re q^H p of the new p summed.
// b is read, or regenerated from the probes (gen).
template <typename S, int NC>
__device__ __forceinline__ void k_resid_q_body(const Blk &bk, Launch L, const double2 *__restrict__ b64,
                                               const double2 *__restrict__ q64, S *__restrict__ rout,
                                               S *__restrict__ pio, const S *__restrict__ qin, int ru, Red rd,
                                               CgState cs, ProbeGen g, int gen) {
    using R = typename St<S>::R;
    __shared__ double sm[2 * kBlock];
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1);
    const int sites_per_tile = kBlock >> logW;
    const unsigned long long seedmix = gen ? mix64(g.seed) : 0ull;
    const ProbeLane pl = gen ? probe_lane(g, NC, g.rhs0 + j) : ProbeLane{};
    const bool restart = ru && (ldg(cs.flags + j) & kFlagRestart);
    double acc[2] = {0.0, 0.0};
    int t0, t1;
    tile_range(bk, L.ntiles, t0, t1);
    // element e = ((site * NC + a) << logW) + j: lane j is tid % W for every
    // e = e0 + tid + k kBlock (kBlock is a multiple of W)
    const size_t e0 = (size_t)t0 * sites_per_tile * NC * W;
    const size_t e1 = min((size_t)t1 * sites_per_tile, (size_t)L.lat.N) * NC * W;
    for (size_t e = e0 + tid; e < e1; e += kBlock) {
        double qr, qi, br, bi;
        St<double2>::ld(q64, e, qr, qi);
        if (gen) {
            const int row = (int)(e >> logW), site = row / NC, a = row - site * NC;
            br = bi = 0.0;
            if (j < g.nvalid) probe_at(g, seedmix, L.lat, NC, pl, site, a, br, bi);
        } else {
            St<double2>::ld(b64, e, br, bi);
        }
        const double nr64 = br - qr, ni64 = bi - qi;
        acc[0] += nr64 * nr64 + ni64 * ni64;
        if (ru) {
            R nr = (R)nr64, ni = (R)ni64;
            if (cs.rq_direct) {
                St<S>::st(rout, e, nr, ni);
                if (restart) St<S>::st(pio, e, nr, ni);
            } else {
                R ro_r, ro_i, po_r, po_i, sqr, sqi;
                St<S>::ld(rout, e, ro_r, ro_i);
                St<S>::ld(pio, e, po_r, po_i);
                St<S>::ld(qin, e, sqr, sqi);
                St<S>::st(rout, e, nr, ni);
                St<S>::round(nr, ni);
                R npr = restart ? nr : po_r + (nr - ro_r), npi = restart ? ni : po_i + (ni - ro_i);
                St<S>::st(pio, e, npr, npi);
                St<S>::round(npr, npi);
                acc[1] += (double)(sqr * npr + sqi * npi);
            }
        }
    }
    if (ru && cs.rq_direct) acc[1] = (bk.b == 0 && tid < W) ? ldg(cs.qp + j) : 0.0;
    block_partials_to<2>(bk, acc, W, logW, rd.part2, rd.nblk, sm);
}

template <typename S, int NC>
__global__ __launch_bounds__(kBlock) void k_resid_q(Launch L, const double2 *__restrict__ b64,
                                                    const double2 *__restrict__ q64, S *__restrict__ rout,
                                                    S *__restrict__ pio, const S *__restrict__ qin, int ru, Red rd,
                                                    CgState cs, ProbeGen g, int gen) {
    k_resid_q_body<S, NC>(own_blk(), L, b64, q64, rout, pio, qin, ru, rd, cs, g, gen);
}

// t_j = sum_x sum_b conj(v_j(x,b)) x_j(x + p e0, b), probes regenerated.
__device__ __forceinline__ void k_displaced_dot_body(const Blk &bk, Launch L, ProbeGen g, int p,
                                                         const double2 *__restrict__ x64, Red rd, CgState cs) {
    __shared__ double sm[2 * kBlock];
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1), sl = tid >> logW;
    const int sites_per_tile = kBlock >> logW, nc = L.nc;
    const unsigned long long seedmix = mix64(g.seed);
    double acc[2] = {0.0, 0.0};
    int t0, t1;
    tile_range(bk, L.ntiles, t0, t1);
    if (j < g.nvalid) {
        ProbeLane pl = probe_lane(g, nc, g.rhs0 + j);
        if (g.cmap) pl.c = g.cmap[pl.c];  // the parent class's probe: same noise, coarse colour
        for (int t = t0; t < t1; ++t) {
            const int site = t * sites_per_tile + sl;
            if (site >= L.lat.N || g.colors[site] != pl.c) continue;
            const int y = shift0(L.lat, site, p);
            for (int b = 0; b < nc; ++b) {
                double zr, zi;
                probe_at(g, seedmix, L.lat, nc, pl, site, b, zr, zi);
                if (zr == 0.0 && zi == 0.0) continue;
                const double2 xv = x64[((size_t)(y * nc + b) << logW) + j];
                acc[0] += zr * xv.x + zi * xv.y;  // conj(z) * x
                acc[1] += zr * xv.y - zi * xv.x;
            }
        }
    }
    block_partials<2>(bk, acc, W, logW, rd, sm);
}

// Map of a nested colouring's fine colours to coarse ones (three passes:
// clear, scatter, check; every colour is range-checked before it indexes).
__global__ void k_level_map_clear(int *cmap, int nfine, int *bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nfine) cmap[i] = -1;
    if (i == 0) *bad = 0;
}

__global__ void k_level_map_scatter(int N, const int *fine, int nfine, const int *coarse, int ncoarse, int *cmap,
                                    int *bad) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    const int c = fine[x], cc = coarse[x];
    if (c < 0 || c >= nfine || cc < 0 || cc >= ncoarse) {
        *bad = 1;
        return;
    }
    cmap[c] = cc;  // equal values from every site of a nested colouring
}

__global__ void k_level_map_check(int N, const int *fine, int nfine, const int *coarse, const int *cmap, int *bad) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    const int c = fine[x];
    if (c >= 0 && c < nfine && cmap[c] != coarse[x]) *bad = 1;
}

__global__ __launch_bounds__(kBlock) void k_displaced_dot(Launch L, ProbeGen g, int p,
                                                         const double2 *__restrict__ x64, Red rd, CgState cs) {
    k_displaced_dot_body(own_blk(), L, g, p, x64, rd, cs);
}

// t_j = a_j^H b_j (FP64 vectors)
__device__ __forceinline__ void k_dot_body(const Blk &bk, Launch L, const double2 *__restrict__ a64,
                                               const double2 *__restrict__ b64, Red rd, CgState cs) {
    __shared__ double sm[2 * kBlock];
    const int tid = threadIdx.x, W = L.W;
    const int sites_per_tile = kBlock >> L.logW;
    double acc[2] = {0.0, 0.0};
    int t0, t1;
    tile_range(bk, L.ntiles, t0, t1);
    const size_t e0 = (size_t)t0 * sites_per_tile * L.nc * W;
    const size_t e1 = min((size_t)t1 * sites_per_tile, (size_t)L.lat.N) * L.nc * W;
    for (size_t e = e0 + tid; e < e1; e += kBlock) {
        const double2 u = a64[e], v = b64[e];
        acc[0] += u.x * v.x + u.y * v.y;
        acc[1] += u.x * v.y - u.y * v.x;
    }
    block_partials<2>(bk, acc, W, L.logW, rd, sm);
}

__global__ __launch_bounds__(kBlock) void k_dot(Launch L, const double2 *__restrict__ a64,
                                               const double2 *__restrict__ b64, Red rd, CgState cs) {
    k_dot_body(own_blk(), L, a64, b64, rd, cs);
}

// Adjoint force of one block of right-hand sides, one thread per output
// entry (site, mu, a, b):
//   dU[mu][x][a][b]    (+)= scale * sum_j conj(l_j(x)_a) x_j(x+mu)_b
//   dUbar[mu][x][a][b] (+)= scale * sum_j x_j(x)_a conj(l_j(x+mu)_b)
__global__ __launch_bounds__(kBlock) void k_force(Launch L, const double2 *__restrict__ x64,
                                                 const double2 *__restrict__ l64, const int *__restrict__ nbr,
                                                 double scale, int first, double2 *__restrict__ dU,
                                                 double2 *__restrict__ dUbar) {
    const int nc = L.nc, W = L.W, logW = L.logW;
    const long long n = (long long)L.lat.N * 4 * nc * nc;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int b = (int)(e % nc);
    const int a = (int)((e / nc) % nc);
    const int mu = (int)((e / (nc * nc)) % 4);
    const int site = (int)(e / (4 * nc * nc));
    const int y = nbr[site * 8 + mu];
    double ur = 0, ui = 0, vr = 0, vi = 0;
    const double2 *la = l64 + ((size_t)(site * nc + a) << logW);
    const double2 *xb = x64 + ((size_t)(y * nc + b) << logW);
    const double2 *xa = x64 + ((size_t)(site * nc + a) << logW);
    const double2 *lb = l64 + ((size_t)(y * nc + b) << logW);
    for (int j = 0; j < W; ++j) {
        const double2 l1 = la[j], x1 = xb[j], x2 = xa[j], l2 = lb[j];
        ur += l1.x * x1.x + l1.y * x1.y;  // conj(l) x
        ui += l1.x * x1.y - l1.y * x1.x;
        vr += x2.x * l2.x + x2.y * l2.y;  // x conj(l)
        vi += x2.y * l2.x - x2.x * l2.y;
    }
    const size_t o = ((size_t)mu * L.lat.N + site) * nc * nc + a * nc + b;
    double2 du = make_double2(scale * ur, scale * ui), db = make_double2(scale * vr, scale * vi);
    if (!first) {
        if (dU) {
            const double2 t = dU[o];
            du.x += t.x;
            du.y += t.y;
        }
        if (dUbar) {
            const double2 t = dUbar[o];
            db.x += t.x;
            db.y += t.y;
        }
    }
    if (dU) dU[o] = du;
    if (dUbar) dUbar[o] = db;
}

// internal FP64 -> ABI [rhs][site][nc] for lanes < nvalid
__global__ void k_to_abi(Launch L, const double2 *__restrict__ x64, double2 *__restrict__ xabi, long long rhs0,
                         long long nvalid) {
    const long long n = (long long)L.lat.N * L.nc * L.W;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int j = (int)(e & (L.W - 1));
    const long long sa = e >> L.logW;  // site * nc + a
    if (j >= nvalid) return;
    xabi[(size_t)(rhs0 + j) * L.lat.N * L.nc + sa] = x64[e];
}

template <typename S>
__global__ void k_abi_to_internal(Launch L, const double2 *__restrict__ vabi, long long rhs0, long long nvalid,
                                  S *__restrict__ out) {
    const long long n = (long long)L.lat.N * L.nc * L.W;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int j = (int)(e & (L.W - 1));
    const long long sa = e >> L.logW;
    double re = 0, im = 0;
    if (j < nvalid) {
        const double2 v = vabi[(size_t)(rhs0 + j) * L.lat.N * L.nc + sa];
        re = v.x;
        im = v.y;
    }
    St<S>::st(out, e, (typename St<S>::R)re, (typename St<S>::R)im);
}

template <typename S>
__global__ void k_internal_to_abi(Launch L, const S *__restrict__ in, double2 *__restrict__ yabi, long long rhs0,
                                  long long nvalid) {
    const long long n = (long long)L.lat.N * L.nc * L.W;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int j = (int)(e & (L.W - 1));
    if (j >= nvalid) return;
    typename St<S>::R re, im;
    St<S>::ld(in, e, re, im);
    yabi[(size_t)(rhs0 + j) * L.lat.N * L.nc + (e >> L.logW)] = make_double2((double)re, (double)im);
}

// probes in the ABI layout [rhs][site][nc]
__global__ void k_probes_abi(Lat lat, int nc, ProbeGen g, long long nrhs, double2 *__restrict__ out) {
    const long long n = nrhs * lat.N * nc;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int b = (int)(e % nc);
    const int site = (int)((e / nc) % lat.N);
    const long long jj = e / ((long long)nc * lat.N);
    double re, im;
    probe_value(g, mix64(g.seed), lat, nc, g.rhs0 + jj, site, b, re, im);
    out[e] = make_double2(re, im);
}

// ============================================================ multi-instance launches
//
// One launch covers every slot (job) of a batch: workgroup w belongs to slot
// slot_of[w] and runs the same body as a standalone launch on that slot's
// lattice, with the slot's own buffers.  Slots whose flags do not include
// the kernel's phase return at once.  The descriptors live in device memory
// and are rewritten by the host between launches, so a captured graph of
// these launches stays valid while finished slots are refilled.

__device__ __forceinline__ const SlotDesc *slot_of_block(const BatchLaunch &B, Blk &bk, int phase) {
    const int s = B.slot_of[blockIdx.x];
    const SlotDesc *d = B.sd + s;
    if (!(d->flags & phase)) return nullptr;
    // an iterating slot whose lanes all stopped at a reliable update waits,
    // idle, for the host to retire it at its next check
    if (phase == kSlotIter && d->cs.live && ldg(d->cs.live) == 0) return nullptr;
    bk.b = (int)blockIdx.x - d->blk0;
    bk.nb = d->L.nblk;
    return d;
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_b_init(BatchLaunch B, int mixed) {
    Blk bk;
    const SlotDesc *d = slot_of_block(B, bk, kSlotInit);
    if (!d) return;
    k_init_body<S, 0>(bk, d->L, d->g, nullptr, 0, 0, (double2 *)d->b64, (S *)d->r, (S *)d->p,
                      (S *)d->xlo, (double2 *)d->x64, mixed, d->rd, d->cs);
}

template <typename S, typename LS, int NC, bool LINKS, int MODE>
__global__ __launch_bounds__(kBlock) void k_b_stencil(BatchLaunch B) {
    Blk bk;
    const SlotDesc *d = slot_of_block(B, bk, kSlotIter);
    if (!d) return;
    k_stencil_body<S, LS, NC, LINKS, MODE>(bk, d->L, (typename St<S>::R)d->diag, (const S *)d->p,
                                           (const S *)d->r, (S *)d->q, (const LS *)d->U,
                                           d->nbr, 1, d->rd);
}

template <typename S, int XM>
__global__ __launch_bounds__(kBlock) void k_b_update(BatchLaunch B) {
    Blk bk;
    const SlotDesc *d = slot_of_block(B, bk, kSlotIter);
    if (!d) return;
    // FP64: the iterate is x64 itself (xlo aliases it)
    k_update_body<S, XM>(bk, d->L, (S *)d->xlo, (S *)d->r, (S *)d->p, (const S *)d->q,
                         d->rd, d->cs);
}

template <typename S>
__global__ __launch_bounds__(kBlock) void k_b_fold(BatchLaunch B, int phase) {
    Blk bk;
    const SlotDesc *d = slot_of_block(B, bk, phase);
    if (!d) return;
    k_fold_body<S>(bk, d->L, (double2 *)d->x64, (S *)d->xlo);
}

template <typename S, int NC, bool LINKS, int MODE>
__global__ __launch_bounds__(kBlock) void k_b_true_resid(BatchLaunch B, int phase, int ru) {
    Blk bk;
    const SlotDesc *d = slot_of_block(B, bk, phase);
    if (!d) return;
    k_true_resid_body<S, NC, LINKS, MODE>(bk, d->L, d->diag, (const double2 *)d->b64,
                                          (const double2 *)d->x64, (const double2 *)d->U64, d->nbr,
                                          (S *)d->r, (S *)d->p, (const S *)d->q, ru, d->rd,
                                          d->cs, d->g, d->gen_b);
}

__global__ __launch_bounds__(kBlock) void k_b_dot(BatchLaunch B) {
    Blk bk;
    const SlotDesc *d = slot_of_block(B, bk, kSlotFinal);
    if (!d) return;
    k_displaced_dot_body(bk, d->L, d->g, d->disp, (const double2 *)d->x64, d->rd, d->cs);
}

// one workgroup per (slot, lane)
template <int NV, int EPI>
__global__ __launch_bounds__(kBlock) void k_b_finish(BatchLaunch B, int phase) {
    const int s = blockIdx.x / B.W, lane = blockIdx.x % B.W;
    const SlotDesc *d = B.sd + s;
    if (!(d->flags & phase) || lane >= d->L.W) return;
    k_finish_body<NV, EPI>(lane, d->rd, d->cs);
}

// After the workgroups were shared anew among the slots, the |r|^2 and
// Re q^H p partials of an iterating slot (written by its last update with its
// old number of workgroups) are replaced by the lane's totals, cs.rr and
// cs.qp (which the check before the new sharing took from them): partial 0
// holds them, the others 0.
__global__ __launch_bounds__(kBlock) void k_b_reseed(BatchLaunch B) {
    const int s = blockIdx.x / B.W, lane = blockIdx.x % B.W;
    const SlotDesc *d = B.sd + s;
    if (!(d->flags & kSlotIter) || lane >= d->L.W) return;
    const double rr = d->cs.rr[lane], qp = d->cs.qp[lane];
    double *dst = d->rd.part2 + (size_t)lane * d->rd.nblk * 2;
    for (int b = threadIdx.x; b < d->rd.nblk; b += kBlock) {
        dst[2 * b] = b == 0 ? rr : 0.0;
        dst[2 * b + 1] = b == 0 ? qp : 0.0;
    }
}

// One wavefront per (slot, lane): wavefront g = blockIdx.x * 4 + wave takes
// slot g / W, lane g % W (a slot's few dozen partials per lane need no
// more; with a workgroup per lane the launch was mostly idle threads).
__global__ __launch_bounds__(kBlock) void k_b_finish_cg(BatchLaunch B) {
    const int g = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6);
    const int s = g / B.W, lane = g % B.W;
    if (s >= B.nslots) return;
    const SlotDesc *d = B.sd + s;
    if (!(d->flags & kSlotIter) || lane >= d->L.W || (d->cs.live && ldg(d->cs.live) == 0)) return;
    k_finish_cg_wave_body(lane, d->rd, d->cs);
}

__global__ void k_b_ctrl(BatchLaunch B) {
    const SlotDesc *d = B.sd + blockIdx.x;
    k_ctrl_body(d->cs, d->L.W);
}

// ============================================================ deflation
//
// Dense pieces of the deflated estimator (Sec. Deflation) on blocks of FP64
// vectors in the internal layout, read as row-major matrices [n rows =
// N * nc][width] (width = the block's lanes).

// t_j = sum_x sum_b conj(u_j(x,b)) w_j(x + p e0, b)
__global__ __launch_bounds__(kBlock) void k_dot_shift(Launch L, const double2 *__restrict__ u,
                                                      const double2 *__restrict__ w, int p, Red rd) {
    __shared__ double sm[2 * kBlock];
    const int tid = threadIdx.x, logW = L.logW, W = L.W;
    const int j = tid & (W - 1), sl = tid >> logW;
    const int sites_per_tile = kBlock >> logW, nc = L.nc;
    double acc[2] = {0.0, 0.0};
    int t0, t1;
    const Blk bk = own_blk();
    tile_range(bk, L.ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const int site = t * sites_per_tile + sl;
        if (site >= L.lat.N) continue;
        const int y = shift0(L.lat, site, p);
        for (int b = 0; b < nc; ++b) {
            const double2 a = u[((size_t)(site * nc + b) << logW) + j];
            const double2 c = w[((size_t)(y * nc + b) << logW) + j];
            acc[0] += a.x * c.x + a.y * c.y;
            acc[1] += a.x * c.y - a.y * c.x;
        }
    }
    block_partials<2>(bk, acc, W, logW, rd, sm);
}

// per-lane |u_j - theta_j w_j|^2 (Ritz residuals: u = A v, w = v)
__global__ __launch_bounds__(kBlock) void k_resid_norm(Launch L, const double2 *__restrict__ u,
                                                       const double2 *__restrict__ w,
                                                       const double *__restrict__ theta, Red rd) {
    __shared__ double sm[kBlock];
    const int tid = threadIdx.x, W = L.W;
    const int sites_per_tile = kBlock >> L.logW;
    const double th = theta[tid & (W - 1)];
    double acc[1] = {0.0};
    int t0, t1;
    const Blk bk = own_blk();
    tile_range(bk, L.ntiles, t0, t1);
    const size_t e0 = (size_t)t0 * sites_per_tile * L.nc * W;
    const size_t e1 = min((size_t)t1 * sites_per_tile, (size_t)L.lat.N) * L.nc * W;
    for (size_t e = e0 + tid; e < e1; e += kBlock) {
        const double2 a = u[e], c = w[e];
        const double dr = a.x - th * c.x, di = a.y - th * c.y;
        acc[0] += dr * dr + di * di;
    }
    block_partials<1>(bk, acc, W, L.logW, rd, sm);
}

// out = a q + b v (real a, b; out may alias v)
__global__ void k_axpby(long long n, double a, const double2 *__restrict__ q, double b, const double2 *v,
                        double2 *out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double2 x = q[e], y = v[e];
    out[e] = make_double2(a * x.x + b * y.x, a * x.y + b * y.y);
}

// v[e] = (+-1 +- i) from a SplitMix64 hash of (seed, e): start vectors of
// the subspace iteration
__global__ void k_rand_fill(long long n, unsigned long long seed, double2 *__restrict__ v) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const unsigned long long h = mix64(mix64(seed) ^ (unsigned long long)e);
    v[e] = make_double2((h >> 63) ? -1.0 : 1.0, ((h >> 62) & 1) ? -1.0 : 1.0);
}

// out lane j = v lane j * s[j] (s[j] = 0 clears the lane)
__global__ void k_scale_lanes(long long n, int W, const double *__restrict__ s, const double2 *__restrict__ v,
                              double2 *__restrict__ out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double f = s[e % W];
    const double2 x = v[e];
    out[e] = make_double2(f * x.x, f * x.y);
}

// Partial products H = X^H Y over one range of rows per workgroup (blockIdx.x)
// for one 64 x 64 output tile (blockIdx.y): part[blockIdx.x][blockIdx.y][64 * 64].
// Rows are staged through LDS 8 at a time; thread t owns the entries
// (t / 64 + 4 k, t % 64), k < 16, of the tile.
constexpr int kGramTile = 64;
__global__ __launch_bounds__(kBlock) void k_gram(long long n, int WX, int WY, const double2 *__restrict__ X,
                                                 const double2 *__restrict__ Y, double2 *__restrict__ part) {
    __shared__ double2 sx[8][kGramTile], sy[8][kGramTile];
    const int tilesY = (WY + kGramTile - 1) / kGramTile;
    const int i0 = (blockIdx.y / tilesY) * kGramTile, j0 = (blockIdx.y % tilesY) * kGramTile;
    const int t = threadIdx.x, jl = t & (kGramTile - 1), il = t / kGramTile;
    double ar[16], ai[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) ar[k] = ai[k] = 0.0;
    const long long r0 = n * blockIdx.x / gridDim.x, r1 = n * (blockIdx.x + 1) / gridDim.x;
    for (long long rb = r0; rb < r1; rb += 8) {
        __syncthreads();
        for (int e = t; e < 8 * kGramTile; e += kBlock) {
            const int rr = e / kGramTile, c = e % kGramTile;
            const long long r = rb + rr;
            sx[rr][c] = (r < r1 && i0 + c < WX) ? X[r * WX + i0 + c] : make_double2(0.0, 0.0);
            sy[rr][c] = (r < r1 && j0 + c < WY) ? Y[r * WY + j0 + c] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
            const double2 y = sy[rr][jl];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double2 x = sx[rr][il + 4 * k];
                ar[k] = fma(x.x, y.x, fma(x.y, y.y, ar[k]));   // conj(x) y
                ai[k] = fma(x.x, y.y, fma(-x.y, y.x, ai[k]));
            }
        }
    }
    double2 *o = part + ((size_t)blockIdx.x * gridDim.y + blockIdx.y) * kGramTile * kGramTile;
#pragma unroll
    for (int k = 0; k < 16; ++k) o[k * kBlock + t] = make_double2(ar[k], ai[k]);
}

// H[i][j] = scale * sum over the row ranges (in order) of the partials
__global__ void k_gram_reduce(int nrb, int WX, int WY, const double2 *__restrict__ part, double scale,
                              double2 *__restrict__ H) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= WX * WY) return;
    const int i = e / WY, j = e % WY;
    const int tilesY = (WY + kGramTile - 1) / kGramTile;
    const int tiles = ((WX + kGramTile - 1) / kGramTile) * tilesY;
    const int tile = (i / kGramTile) * tilesY + j / kGramTile;
    const int off = (i % kGramTile) * kGramTile + j % kGramTile;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < nrb; ++b) {
        const double2 v = part[((size_t)b * tiles + tile) * kGramTile * kGramTile + off];
        sr += v.x;
        si += v.y;
    }
    H[e] = make_double2(scale * sr, scale * si);
}

// out[r][j] (+)= sum_i X[r][i] C[i][j], j < WY, i < WX (out must not alias X)
__global__ void k_rot(long long n, int WX, int WY, const double2 *__restrict__ X, const double2 *__restrict__ C,
                      double2 *__restrict__ out, int accumulate) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * WY) return;
    const long long r = e / WY;
    const int j = (int)(e - r * WY);
    double sr = 0.0, si = 0.0;
    if (accumulate) {
        sr = out[e].x;
        si = out[e].y;
    }
    const double2 *xr = X + r * WX;
    for (int i = 0; i < WX; ++i) {
        const double2 x = xr[i], c = C[(size_t)i * WY + j];
        sr = fma(x.x, c.x, fma(-x.y, c.y, sr));
        si = fma(x.x, c.y, fma(x.y, c.x, si));
    }
    out[e] = make_double2(sr, si);
}

// per-site bound sum over the eight hops of |U|_F (FP64 hop links)
__global__ void k_hop_bound(Lat lat, int nc, const double2 *__restrict__ U8, double *__restrict__ out) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= lat.N) return;
    double s = 0.0;
    for (int d = 0; d < 8; ++d) {
        double f = 0.0;
        for (int e = 0; e < nc * nc; ++e) {
            const double2 u = U8[((size_t)site * 8 + d) * nc * nc + e];
            f += u.x * u.x + u.y * u.y;
        }
        s += sqrt(f);
    }
    out[site] = s;
}

// ============================================================ launchers

static int blocks_for(long long n) { return (int)((n + kBlock - 1) / kBlock); }

int grid_blocks(int ntiles) {
    // four workgroups per CU, a multiple of 8 (one contiguous share per
    // XCD); never more than there are tiles.  All of them are resident at
    // once, so they walk their slabs in step (16^4 sites, FP32, W = 32: a
    // CG iteration took 3% less time than with 2048, 14% less than with 512)
    const int cap = 1024;
    if (ntiles <= 8) return ntiles;
    int n = ntiles < cap ? ntiles : cap;
    return n - n % 8;
}

void prepare_links(const Lat &lat, int nc, const void *abi, int *nbr, double *u64, int prec, void *u8,
                   double *u8x, hipStream_t s) {
    const long long n = 8LL * lat.N * (abi ? nc * nc : 1);
    const double2 *in = (const double2 *)abi;
    if (prec == kF64)
        k_prepare<double2><<<blocks_for(n), kBlock, 0, s>>>(lat, nc, in, nbr, (double2 *)u64, (double2 *)u8,
                                                            (double2 *)u8x);
    else if (prec == kF32)
        k_prepare<float2><<<blocks_for(n), kBlock, 0, s>>>(lat, nc, in, nbr, (double2 *)u64, (float2 *)u8,
                                                           (double2 *)u8x);
    else
        k_prepare<bf16x2><<<blocks_for(n), kBlock, 0, s>>>(lat, nc, in, nbr, (double2 *)u64, (bf16x2 *)u8,
                                                           (double2 *)u8x);
}

#define DP_DISPATCH_PREC(prec, S, ...)          \
    do {                                        \
        if ((prec) == kF64) {                   \
            using S = double2;                  \
            __VA_ARGS__;                        \
        } else if ((prec) == kF32) {            \
            using S = float2;                   \
            __VA_ARGS__;                        \
        } else {                                \
            using S = bf16x2;                   \
            __VA_ARGS__;                        \
        }                                       \
    } while (0)

void launch_init_probe(const Launch &L, int prec, const ProbeGen &g, double *b64, void *r, void *p, void *xlo,
                       double *x64, int mixed, const Red &rd, const CgState &cs) {
    DP_DISPATCH_PREC(prec, S,
                     k_init<S, 0><<<L.nblk, kBlock, 0, L.stream>>>(L, g, nullptr, 0, 0, (double2 *)b64, (S *)r,
                                                                   (S *)p, (S *)xlo, (double2 *)x64, mixed, rd,
                                                                   cs));
    k_finish<2, kEpiInit><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

void launch_init_abi(const Launch &L, int prec, const double *babi, long long rhs0, long long nvalid, double *b64,
                     void *r, void *p, void *xlo, double *x64, int mixed, const Red &rd, const CgState &cs) {
    ProbeGen g{};
    DP_DISPATCH_PREC(prec, S,
                     k_init<S, 1><<<L.nblk, kBlock, 0, L.stream>>>(L, g, (const double2 *)babi, rhs0, nvalid,
                                                                   (double2 *)b64, (S *)r, (S *)p, (S *)xlo,
                                                                   (double2 *)x64, mixed, rd, cs));
    k_finish<2, kEpiInit><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

// Stencil modes a launch shape admits.  The grouped modes need the slab walk
// (a grid of a multiple of 8 workgroups over x0-slabs): pairs an even
// number of slices per slab, quads two slices and an even D3, lines a
// multiple of four slices; the LDS tiles take W >= 16 (pairs, mode 1) or
// W >= 32 (quads, lines); mode 2 a wavefront per site (W >= 64); mode 5
// one right-hand side (not BF16).
bool stencil_mode_valid(const Launch &L, int prec, int mode) {
    const bool slabs = L.nblk >= 8 && L.nblk % 8 == 0 && L.lat.D[0] % 8 == 0;
    const int n0 = L.lat.D[0] / 8;
    switch (mode) {
        case 0: return true;
        case 1: return L.W >= 16;
        case 2: return L.W >= 64;
        case 3: return slabs && n0 % 2 == 0 && L.W >= 16;
        case 4: return slabs && n0 == 2 && L.lat.D[3] % 2 == 0 && L.W >= 32;
        case 5: return L.W == 1 && prec != kBF16;
        case 6: return slabs && n0 % 4 == 0 && L.W >= 32;
        default: return false;
    }
}

// The choice without timing: the grouped modes where they apply (not for
// BF16, whose packed-dot body has none), else by width.
int stencil_mode_rule(const Launch &L, int prec) {
    const bool bf = prec == kBF16;
    if (L.W == 1 && !bf) return 5;
    if (L.W >= 64) return 2;
    if (!bf && stencil_mode_valid(L, prec, 4)) return 4;
    if (!bf && stencil_mode_valid(L, prec, 6)) return 6;
    if (!bf && stencil_mode_valid(L, prec, 3)) return 3;
    return L.W >= 16 ? 1 : 0;
}

template <typename S, typename LS, int NC, bool LINKS>
static void stencil_nc(const Launch &L, const StencilArgs &a) {
    using R = typename St<S>::R;
    dim3 grid(L.nblk), blk(kBlock);
    const S *pin = (const S *)a.pin, *rin = (const S *)a.rin;
    S *q = (S *)a.q;
    const LS *U = (const LS *)a.U;
#define DP_ST(M)                                                                                        \
    if (a.ev0)                                                                                          \
        hipExtLaunchKernelGGL(k_stencil<S, LS, NC, LINKS, M>, grid, blk, 0, L.stream, a.ev0, a.ev1, 0, L, \
                              (R)a.diag, pin, rin, q, U, a.nbr, a.cg, a.rd);                            \
    else                                                                                                \
        k_stencil<S, LS, NC, LINKS, M><<<grid, blk, 0, L.stream>>>(L, (R)a.diag, pin, rin, q, U, a.nbr, a.cg, a.rd)
    constexpr int prec = std::is_same<S, double2>::value ? kF64 : (std::is_same<S, float2>::value ? kF32 : kBF16);
    const int mode = L.smode >= 0 && stencil_mode_valid(L, prec, L.smode) ? L.smode : stencil_mode_rule(L, prec);
    switch (mode) {
        case 5:
            if constexpr (prec != kBF16) {
                DP_ST(5);
                break;
            }
            [[fallthrough]];
        case 0: DP_ST(0); break;
        case 1: DP_ST(1); break;
        case 2: DP_ST(2); break;
        case 3: DP_ST(3); break;
        case 4: DP_ST(4); break;
        default: DP_ST(6); break;
    }
#undef DP_ST
}

template <typename S, typename LS>
static void stencil_t(const Launch &L, const StencilArgs &a) {
    if (L.nc == 3) {
        if (a.links)
            stencil_nc<S, LS, 3, true>(L, a);
        else
            stencil_nc<S, LS, 3, false>(L, a);
    } else {
        if (a.links)
            stencil_nc<S, LS, 1, true>(L, a);
        else
            stencil_nc<S, LS, 1, false>(L, a);
    }
}

void launch_stencil(const Launch &L, int prec, const StencilArgs &a) {
    if (prec == kF64)
        stencil_t<double2, double2>(L, a);
    else if (prec == kF32)
        stencil_t<float2, float2>(L, a);
    else
        stencil_t<bf16x2, bf16x2>(L, a);
    if (a.cg) k_finish_cg<<<L.W, kBlock, 0, L.stream>>>(a.rd, a.cs);
}

void launch_update(const Launch &L, int prec, void *x, void *r, void *p, const void *q, const Red &rd,
                   const CgState &cs, int xmode) {
    if (prec == kF64 || !cs.xdef) xmode = 0;  // deferral: FP32 and BF16 storage
    DP_DISPATCH_PREC(prec, S, {
        if (xmode == 1)
            k_update<S, 1><<<L.nblk, kBlock, 0, L.stream>>>(L, (S *)x, (S *)r, (S *)p, (const S *)q, rd, cs);
        else if (xmode == 2)
            k_update<S, 2><<<L.nblk, kBlock, 0, L.stream>>>(L, (S *)x, (S *)r, (S *)p, (const S *)q, rd, cs);
        else
            k_update<S, 0><<<L.nblk, kBlock, 0, L.stream>>>(L, (S *)x, (S *)r, (S *)p, (const S *)q, rd, cs);
    });
}

void launch_fold(const Launch &L, int prec, double *x64, void *xlo) {
    DP_DISPATCH_PREC(prec, S, k_fold<S><<<L.nblk, kBlock, 0, L.stream>>>(L, (double2 *)x64, (S *)xlo));
}


void launch_resid_q(const Launch &L, int prec, const double *b64, const double *q64, void *r, void *p,
                    const void *q, int ru_mode, const Red &rd, const CgState &cs, const ProbeGen *gen) {
    const ProbeGen g = gen ? *gen : ProbeGen{};
    const int use_gen = gen ? 1 : 0;
    const double2 *b = (const double2 *)b64, *qq = (const double2 *)q64;
    DP_DISPATCH_PREC(prec, S, {
        if (L.nc == 3)
            k_resid_q<S, 3><<<L.nblk, kBlock, 0, L.stream>>>(L, b, qq, (S *)r, (S *)p, (const S *)q, ru_mode, rd, cs,
                                                             g, use_gen);
        else
            k_resid_q<S, 1><<<L.nblk, kBlock, 0, L.stream>>>(L, b, qq, (S *)r, (S *)p, (const S *)q, ru_mode, rd, cs,
                                                             g, use_gen);
    });
    if (ru_mode)
        k_finish<2, kEpiRU><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
    else
        k_finish<2, kEpiStats><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

void launch_level_map(int N, const int *fine, int nfine, const int *coarse, int ncoarse, int *cmap, int *bad,
                      hipStream_t s) {
    k_level_map_clear<<<blocks_for(nfine), kBlock, 0, s>>>(cmap, nfine, bad);
    k_level_map_scatter<<<blocks_for(N), kBlock, 0, s>>>(N, fine, nfine, coarse, ncoarse, cmap, bad);
    k_level_map_check<<<blocks_for(N), kBlock, 0, s>>>(N, fine, nfine, coarse, cmap, bad);
}

void launch_displaced_dot(const Launch &L, const ProbeGen &g, int p, const double *x64, const Red &rd,
                          const CgState &cs) {
    k_displaced_dot<<<L.nblk, kBlock, 0, L.stream>>>(L, g, p, (const double2 *)x64, rd, cs);
    k_finish<2, kEpiTj><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

void launch_dot(const Launch &L, const double *a64, const double *b64, const Red &rd, const CgState &cs) {
    k_dot<<<L.nblk, kBlock, 0, L.stream>>>(L, (const double2 *)a64, (const double2 *)b64, rd, cs);
    k_finish<2, kEpiTj><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

void launch_ctrl(const Red &rd, const CgState &cs, int W, hipStream_t s) {
    k_finish<2, kEpiCheck><<<W, kBlock, 0, s>>>(rd, cs);
    k_ctrl<<<1, 64, 0, s>>>(cs, W);
}

// The same force for W >= 8, W threads per (site, mu) pair: thread j loads
// lane j of the four rows the pair needs (coalesced, each once per pair) and
// forms its lane's 4 nc^2 doubles (padded to 8 * 5 = 40 for nc = 3); the
// lanes are summed by a reduce-scatter inside the wavefront (three halvings:
// a lane keeps one half of its values and adds its partner's copy of that
// half, so the shuffles move 20 + 10 + 5 values instead of 3 x 40), a
// butterfly on the remaining five, and through LDS across the wavefronts of
// a pair (W > 64); all in a fixed order.
template <int NC>
__global__ __launch_bounds__(kBlock) void k_force_lanes(Launch L, const double2 *__restrict__ x64,
                                                        const double2 *__restrict__ l64, const int *__restrict__ nbr,
                                                        double scale, int first, double *__restrict__ dU,
                                                        double *__restrict__ dUbar) {
    constexpr int NV = 4 * NC * NC;         // dU re, dU im, dUbar re, dUbar im per (a, b)
    constexpr int NP = (NV + 7) / 8 * 8;    // padded so that three halvings divide it
    __shared__ double red[kBlock / 8][NP];  // one row per pair (W < 64) or per wavefront (W >= 64)
    const int W = L.W, logW = L.logW, tid = threadIdx.x;
    const int j = tid & (W - 1), pl = tid >> logW;
    const long long pair = (long long)blockIdx.x * (kBlock >> logW) + pl;
    const bool live = pair < (long long)L.lat.N * 4;
    const int site = live ? (int)(pair >> 2) : 0, mu = (int)(pair & 3);
    double v[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) v[k] = 0.0;
    if (live) {
        const int y = nbr[site * 8 + mu];
        double2 la[NC], xa[NC], xb[NC], lb[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            la[c] = l64[((size_t)(site * NC + c) << logW) + j];
            xa[c] = x64[((size_t)(site * NC + c) << logW) + j];
            xb[c] = x64[((size_t)(y * NC + c) << logW) + j];
            lb[c] = l64[((size_t)(y * NC + c) << logW) + j];
        }
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                const int k = 4 * (a * NC + b);
                v[k] = la[a].x * xb[b].x + la[a].y * xb[b].y;  // conj(l) x
                v[k + 1] = la[a].x * xb[b].y - la[a].y * xb[b].x;
                v[k + 2] = xa[a].x * lb[b].x + xa[a].y * lb[b].y;  // x conj(l)
                v[k + 3] = xa[a].y * lb[b].x - xa[a].x * lb[b].y;
            }
    }
    // reduce-scatter over the span = min(W, 64) lanes of a group (W >= 8:
    // three halvings fit), then a butterfly over the rest of the span
    const int span = W < 64 ? W : 64, lane = tid & 63;
    int base = 0;  // first value this lane holds after the halvings
#pragma unroll
    for (int step = 0; step < 3; ++step) {
        const int off = span >> (step + 1);
        const int half = NP >> (step + 1);
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            const double keep = upper ? v[k + half] : v[k];
            const double give = upper ? v[k] : v[k + half];
            v[k] = keep + __shfl_xor(give, off, 64);
        }
        base += upper ? half : 0;
    }
    constexpr int NR = NP / 8;  // values per lane after the halvings
    for (int off = span >> 4; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NR; ++k) v[k] += __shfl_xor(v[k], off, 64);
    // lanes with the low bits of the span clear hold the sums of their values
    const int row = W < 64 ? pl : (tid >> 6);
    if ((lane & ((span >> 3) - 1)) == 0)
#pragma unroll
        for (int k = 0; k < NR; ++k) red[row][base + k] = v[k];
    __syncthreads();
    if (!live) return;
    const int nw = W < 64 ? 1 : W >> 6, r0 = W < 64 ? pl : (pl * W) >> 6;
    for (int k = j; k < NV; k += W) {
        double t = red[r0][k];
        for (int w = 1; w < nw; ++w) t += red[r0 + w][k];
        const int ab = k >> 2, comp = k & 3;
        const size_t o = 2 * (((size_t)mu * L.lat.N + site) * NC * NC + ab) + (comp & 1);
        double *out = comp < 2 ? dU : dUbar;
        if (!out) continue;
        t *= scale;
        out[o] = first ? t : out[o] + t;
    }
}

void launch_force(const Launch &L, const double *x64, const double *l64, const int *nbr, double scale, int first,
                  double *dU, double *dUbar) {
    if (L.W >= 8) {
        // W threads per (site, mu) pair
        const long long nthreads = (long long)L.lat.N * 4 * L.W;
        if (L.nc == 3)
            k_force_lanes<3><<<blocks_for(nthreads), kBlock, 0, L.stream>>>(L, (const double2 *)x64,
                                                                           (const double2 *)l64, nbr, scale, first,
                                                                           dU, dUbar);
        else
            k_force_lanes<1><<<blocks_for(nthreads), kBlock, 0, L.stream>>>(L, (const double2 *)x64,
                                                                           (const double2 *)l64, nbr, scale, first,
                                                                           dU, dUbar);
        return;
    }
    const long long n = (long long)L.lat.N * 4 * L.nc * L.nc;
    k_force<<<blocks_for(n), kBlock, 0, L.stream>>>(L, (const double2 *)x64, (const double2 *)l64, nbr, scale,
                                                    first, (double2 *)dU, (double2 *)dUbar);
}

void launch_to_abi(const Launch &L, const double *x64, double *xabi, long long rhs0, long long nvalid) {
    const long long n = (long long)L.lat.N * L.nc * L.W;
    k_to_abi<<<blocks_for(n), kBlock, 0, L.stream>>>(L, (const double2 *)x64, (double2 *)xabi, rhs0, nvalid);
}

void launch_abi_to_internal(const Launch &L, int prec, const double *vabi, long long rhs0, long long nvalid,
                            void *out) {
    const long long n = (long long)L.lat.N * L.nc * L.W;
    DP_DISPATCH_PREC(prec, S,
                     k_abi_to_internal<S><<<blocks_for(n), kBlock, 0, L.stream>>>(L, (const double2 *)vabi, rhs0,
                                                                                  nvalid, (S *)out));
}

void launch_internal_to_abi_prec(const Launch &L, int prec, const void *in, double *yabi, long long rhs0,
                                 long long nvalid) {
    const long long n = (long long)L.lat.N * L.nc * L.W;
    DP_DISPATCH_PREC(prec, S,
                     k_internal_to_abi<S><<<blocks_for(n), kBlock, 0, L.stream>>>(L, (const S *)in, (double2 *)yabi,
                                                                                  rhs0, nvalid));
}

void launch_make_probes_abi(const Lat &lat, int nc, const ProbeGen &g, long long nrhs, double *out, hipStream_t s) {
    const long long n = nrhs * lat.N * nc;
    k_probes_abi<<<blocks_for(n), kBlock, 0, s>>>(lat, nc, g, nrhs, (double2 *)out);
}

// ------------------------------------------------------------ multi-instance launchers

void launch_b_init(const BatchLaunch &B, int mixed) {
    DP_DISPATCH_PREC(B.prec, S, k_b_init<S><<<B.nblocks, kBlock, 0, B.stream>>>(B, mixed));
    k_b_finish<2, kEpiInit><<<B.nslots * B.W, kBlock, 0, B.stream>>>(B, kSlotInit);
}

template <typename S, typename LS, int NC, bool LINKS, int M>
static void b_stencil_m(const BatchLaunch &B, hipEvent_t ev0, hipEvent_t ev1) {
    if (ev0)
        hipExtLaunchKernelGGL(k_b_stencil<S, LS, NC, LINKS, M>, dim3(B.nblocks), dim3(kBlock), 0, B.stream, ev0, ev1,
                              0, B);
    else
        k_b_stencil<S, LS, NC, LINKS, M><<<B.nblocks, kBlock, 0, B.stream>>>(B);
}

template <typename S, typename LS, int NC, bool LINKS>
static void b_stencil_t(const BatchLaunch &B, hipEvent_t ev0, hipEvent_t ev1) {
    if (B.mode == 2)
        b_stencil_m<S, LS, NC, LINKS, 2>(B, ev0, ev1);
    else if (B.mode == 1)
        b_stencil_m<S, LS, NC, LINKS, 1>(B, ev0, ev1);
    else
        b_stencil_m<S, LS, NC, LINKS, 0>(B, ev0, ev1);
}

template <typename S>
static void b_stencil(const BatchLaunch &B, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    if (B.nc == 3)
        B.links ? b_stencil_t<S, S, 3, true>(B, ev0, ev1) : b_stencil_t<S, S, 3, false>(B, ev0, ev1);
    else
        B.links ? b_stencil_t<S, S, 1, true>(B, ev0, ev1) : b_stencil_t<S, S, 1, false>(B, ev0, ev1);
}

void launch_b_stencil(const BatchLaunch &B, hipEvent_t ev0, hipEvent_t ev1) {
    DP_DISPATCH_PREC(B.prec, S, b_stencil<S>(B, ev0, ev1));
}

void launch_b_update(const BatchLaunch &B, int xmode) {
    k_b_finish_cg<<<(B.nslots * B.W + kBlock / 64 - 1) / (kBlock / 64), kBlock, 0, B.stream>>>(B);
    if (B.prec == kF64) xmode = 0;  // the slots' state of mixed precision has xdef
    DP_DISPATCH_PREC(B.prec, S, {
        if (xmode == 1)
            k_b_update<S, 1><<<B.nblocks, kBlock, 0, B.stream>>>(B);
        else if (xmode == 2)
            k_b_update<S, 2><<<B.nblocks, kBlock, 0, B.stream>>>(B);
        else
            k_b_update<S, 0><<<B.nblocks, kBlock, 0, B.stream>>>(B);
    });
}

void launch_b_reseed(const BatchLaunch &B) { k_b_reseed<<<B.nslots * B.W, kBlock, 0, B.stream>>>(B); }

void launch_b_iteration(const BatchLaunch &B, int xmode) {
    launch_b_stencil(B);
    launch_b_update(B, xmode);
}

template <typename S, int NC, bool LINKS>
static void b_tr_t(const BatchLaunch &B, int phase, int ru) {
    if (B.mode == 2)
        k_b_true_resid<S, NC, LINKS, 2><<<B.nblocks, kBlock, 0, B.stream>>>(B, phase, ru);
    else if (B.mode == 1)
        k_b_true_resid<S, NC, LINKS, 1><<<B.nblocks, kBlock, 0, B.stream>>>(B, phase, ru);
    else
        k_b_true_resid<S, NC, LINKS, 0><<<B.nblocks, kBlock, 0, B.stream>>>(B, phase, ru);
}

// Reliable update (final_stats = 0: slots flagged kSlotRU; mixed precision:
// fold, then the true residual replaces r and continues p) or the final
// statistics (final_stats = 1: slots flagged kSlotFinal; FP64, whose iterate
// is already the solution: the true residual's norm only).
void launch_b_ru(const BatchLaunch &B, int final_stats) {
    const int phase = final_stats ? kSlotFinal : kSlotRU;
    const int ru = final_stats ? 0 : 1;
    DP_DISPATCH_PREC(B.prec, S, {
        if (B.prec != kF64) k_b_fold<S><<<B.nblocks, kBlock, 0, B.stream>>>(B, phase);
        if (B.nc == 3)
            B.links ? b_tr_t<S, 3, true>(B, phase, ru) : b_tr_t<S, 3, false>(B, phase, ru);
        else
            B.links ? b_tr_t<S, 1, true>(B, phase, ru) : b_tr_t<S, 1, false>(B, phase, ru);
    });
    if (final_stats)
        k_b_finish<2, kEpiStats><<<B.nslots * B.W, kBlock, 0, B.stream>>>(B, phase);
    else
        k_b_finish<2, kEpiRU><<<B.nslots * B.W, kBlock, 0, B.stream>>>(B, phase);
}

void launch_b_dot(const BatchLaunch &B) {
    k_b_dot<<<B.nblocks, kBlock, 0, B.stream>>>(B);
    k_b_finish<2, kEpiTj><<<B.nslots * B.W, kBlock, 0, B.stream>>>(B, kSlotFinal);
}

void launch_b_ctrl(const BatchLaunch &B) {
    k_b_finish<2, kEpiCheck><<<B.nslots * B.W, kBlock, 0, B.stream>>>(B, kSlotIter);
    k_b_ctrl<<<B.nslots, 64, 0, B.stream>>>(B);
}

void launch_b_count(const BatchLaunch &B) { k_b_ctrl<<<B.nslots, 64, 0, B.stream>>>(B); }

// Copies the CG state block of every slot flagged kSlotFinal (stride bytes,
// a multiple of 16) from st_all to dst, the device alias of a pinned host
// buffer with the same layout.
__global__ void k_b_state_out(BatchLaunch B, const char *__restrict__ st_all, char *__restrict__ dst, size_t stride) {
    const SlotDesc *d = B.sd + blockIdx.x;
    if (!(d->flags & kSlotFinal)) return;
    const uint4 *src = (const uint4 *)(st_all + stride * blockIdx.x);
    uint4 *out = (uint4 *)(dst + stride * blockIdx.x);
    for (size_t i = threadIdx.x; i < stride / 16; i += blockDim.x) out[i] = ldg(src + i);
}

// dst[0 .. bytes) = src[0 .. bytes): bytes a multiple of 4; src may be the
// device alias of pinned host memory
__global__ void k_copy_in(void *__restrict__ dst, const void *__restrict__ src, size_t bytes) {
    const size_t n16 = bytes / 16;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, st = (size_t)gridDim.x * blockDim.x;
    for (size_t i = i0; i < n16; i += st) stg((uint4 *)dst + i, ldg((const uint4 *)src + i));
    for (size_t i = n16 * 4 + i0; i < bytes / 4; i += st) stg((uint32_t *)dst + i, ldg((const uint32_t *)src + i));
}

void launch_copy_in(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (!bytes) return;
    const int blocks = (int)std::min<size_t>(64, (bytes / 16 + kBlock - 1) / kBlock + 1);
    k_copy_in<<<blocks, kBlock, 0, s>>>(dst, src, bytes);
}

void launch_b_state_out(const BatchLaunch &B, const char *st_all, char *dst, size_t stride) {
    k_b_state_out<<<B.nslots, kBlock, 0, B.stream>>>(B, st_all, dst, stride);
}


void launch_init_b64(const Launch &L, int prec, double *b64, void *r, void *p, void *xlo, double *x64, int mixed,
                     const Red &rd, const CgState &cs) {
    ProbeGen g{};
    DP_DISPATCH_PREC(prec, S,
                     k_init<S, 2><<<L.nblk, kBlock, 0, L.stream>>>(L, g, nullptr, 0, 0, (double2 *)b64, (S *)r,
                                                                   (S *)p, (S *)xlo, (double2 *)x64, mixed, rd,
                                                                   cs));
    k_finish<2, kEpiInit><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

void launch_dot_shift(const Launch &L, const double *u, const double *w, int p, const Red &rd, const CgState &cs) {
    k_dot_shift<<<L.nblk, kBlock, 0, L.stream>>>(L, (const double2 *)u, (const double2 *)w, p, rd);
    k_finish<2, kEpiTj><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

void launch_resid_norm(const Launch &L, const double *u, const double *w, const double *theta, const Red &rd,
                       const CgState &cs) {
    k_resid_norm<<<L.nblk, kBlock, 0, L.stream>>>(L, (const double2 *)u, (const double2 *)w, theta, rd);
    k_finish<1, kEpiStatsP1><<<L.W, kBlock, 0, L.stream>>>(rd, cs);
}

void launch_axpby(long long n, double a, const double *q, double b, const double *v, double *out, hipStream_t s) {
    k_axpby<<<blocks_for(n), kBlock, 0, s>>>(n, a, (const double2 *)q, b, (const double2 *)v, (double2 *)out);
}

void launch_rand_fill(long long n, unsigned long long seed, double *v, hipStream_t s) {
    k_rand_fill<<<blocks_for(n), kBlock, 0, s>>>(n, seed, (double2 *)v);
}

void launch_scale_lanes(long long n, int W, const double *sc, const double *v, double *out, hipStream_t s) {
    k_scale_lanes<<<blocks_for(n), kBlock, 0, s>>>(n, W, sc, (const double2 *)v, (double2 *)out);
}

int gram_row_blocks(long long n) { return (int)std::max<long long>(1, std::min<long long>(256, n / 512)); }

void launch_gram(long long n, int WX, int WY, const double *X, const double *Y, double *part, double scale, double *H,
                 hipStream_t s) {
    const int nrb = gram_row_blocks(n);
    const int tiles = ((WX + kGramTile - 1) / kGramTile) * ((WY + kGramTile - 1) / kGramTile);
    k_gram<<<dim3(nrb, tiles), kBlock, 0, s>>>(n, WX, WY, (const double2 *)X, (const double2 *)Y, (double2 *)part);
    k_gram_reduce<<<blocks_for((long long)WX * WY), kBlock, 0, s>>>(nrb, WX, WY, (const double2 *)part, scale,
                                                                   (double2 *)H);
}

void launch_rot(long long n, int WX, int WY, const double *X, const double *C, double *out, int accumulate,
                hipStream_t s) {
    k_rot<<<blocks_for(n * WY), kBlock, 0, s>>>(n, WX, WY, (const double2 *)X, (const double2 *)C, (double2 *)out,
                                               accumulate);
}

void launch_hop_bound(const Lat &lat, int nc, const double *U8, double *out, hipStream_t s) {
    k_hop_bound<<<blocks_for(lat.N), kBlock, 0, s>>>(lat, nc, (const double2 *)U8, out);
}

}  // namespace dp
