// Internal declarations of the dp library (not part of the ABI).
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dp.h"

namespace dp {

// ---------------------------------------------------------------- colouring
std::vector<std::array<int32_t, 4>> displaced_stencil(int32_t p, int32_t k);
std::vector<std::array<int32_t, 4>> displaced_stencil(const int32_t *ps, int32_t np, int32_t k);
dp_status build_coloring(const int32_t dims[4], int32_t p, const int32_t *ks, int32_t nlevels,
                         int32_t order, int32_t *colors, int32_t *ncolors, int32_t *order_used,
                         std::string &err);
dp_status build_coloring_multi(const int32_t dims[4], const int32_t *ps, int32_t np, const int32_t *ks,
                               int32_t nlevels, int32_t order, int32_t *colors, int32_t *ncolors,
                               int32_t *order_used, std::string &err);
void tile_shape(const int32_t dims[4], int32_t p, int32_t k, int32_t tile[4]);
dp_status build_coloring_tiled(const int32_t dims[4], int32_t p, int32_t k, int32_t order, int32_t *colors,
                               int32_t *ncolors, int32_t *order_used, int32_t tile[4], std::string &err);
dp_status clearance(const int32_t dims[4], const int32_t *colors, int32_t p, int32_t kmax, double *pct,
                    std::string &err);

// ---------------------------------------------------------------- device side
constexpr int kBlock = 256;      // threads per workgroup of every lattice kernel
constexpr int kMaxW = 256;       // largest right-hand-side block width
// doubles of one block's per-lane state: rr, qp, rr_ref, bb, alpha, beta,
// true_rr, tj (two per lane), xdef, and 8 more; its ints follow
constexpr size_t kStateDoubles = 10 * kMaxW + 8;

// Per-workgroup partial sums of the reductions.  part1 [W][nblk][NV] (NV <=
// 4): the stencil's p^H q, r^H q, |q|^2, r^H p of a CG iteration (r^H q and
// r^H p with BF16 storage only), and the other dot products; part2 [W][nblk][2]: |r|^2 and
// Re q^H p of the residual and direction that the last vector update,
// initialisation or reliable update wrote (q = A p of the direction before;
// the next finishing kernel of the CG iteration adds them up).
struct Red {
    double *part1;
    double *part2;
    int nblk;
};

// Per-right-hand-side CG state of one block of W right-hand sides (device).
struct CgState {
    double *rr, *qp, *rr_ref, *bb, *alpha, *beta, *true_rr;  // qp: Re q^H p total of part2
    double *xdef;        // alpha / beta of an x update deferred by one iteration (null: none)
    double *tj;          // [W][2] contraction results / dot products
    int *active, *iters, *flags;
    int *ctrl;           // [0] active, [1] candidates, [2] need reliable update, [3] breakdowns
    double *ctrld;       // [0] max over active lanes of |r|^2 / (tol^2 |b|^2)
    double tol2, delta2;
    int exact;           // 1: FP64 inner solve (no reliable updates)
    int hold;            // 1: lanes due a reliable update wait for it (BF16 storage)
    int rq_direct;       // 1 exactly for BF16 storage, whose stencil sums r^H q and
                         //    r^H p itself; 0: the finishing kernel forms r^H q from
                         //    p^H q and Re q^H p
    int *live;           // multi-instance slots: the slot's active lanes (device),
                         //    written by the control kernel, set by the initialisation;
                         //    iteration kernels skip a slot with none.  Null otherwise.
};

// kFlagRestart (mixed precision): p^H A p <= 0 in low precision; the next
// reliable update restarts the search direction from the true residual.
// kFlagHold (BF16 storage): the lane is due a reliable update (its residual
// fell by the factor delta, or it must restart); it does not move (alpha = 0,
// p kept, iteration count unchanged) until the update is done, so it never
// iterates past what the low precision resolves.  (FP32 lanes go on: a few
// iterations beyond delta cost them nothing.)
enum { kFlagBreakdown = 1, kFlagConverged = 2, kFlagRestart = 4, kFlagHold = 8 };

// Geometry of a lattice on the device.
struct Lat {
    int D[4];
    int N;
};

// How probing vectors are enumerated (device copy of dp_probe_spec fields).
struct ProbeGen {
    const int *colors;
    unsigned long long seed;
    int ncolors, sample0, noise, dilute;
    long long rhs0;      // enumeration index of lane 0
    long long nvalid;    // lanes [0, nvalid) carry probes
    int shift;           // 0: v_j; p: (P^T v_j)(y) = v_j(y - p e0)
    const int *cmap;     // displaced dot only: non-null, lane j (colour c_j) is contracted with
                         // the probe of colour cmap[c_j] of the colouring `colors` (its parent
                         // class on a coarser nested level); null, with its own probe
};

enum Prec { kF64 = 0, kF32 = 1, kBF16 = 2 };

// Launch helpers (kernels.hip).  All vectors in the internal layout
// [site][nc][W] complex of the given precision; W a power of two.
struct Launch {
    Lat lat;
    int nc, W, logW;
    int nblk, ntiles;   // grid size and number of site tiles
    hipStream_t stream;
    int smode = -1;     // stencil mode (kernels.hip); -1: the built-in choice for the shape
};

// One job of a multi-instance launch: a block of W right-hand sides of one
// lattice instance, with its own buffers and CG state.  All slots of a
// launch share the precision, nc, W and whether links are present.
struct SlotDesc {
    Launch L;            // geometry; L.nblk workgroups starting at blk0
    int blk0;
    int flags;           // kSlot* phases this slot takes part in
    double diag;         // m2 + 8
    const void *U;       // inner-precision hop links [N][8][nc][nc]
    const void *U64;     // FP64 hop links [N][8][nc][nc] (the true residual)
    const int *nbr;
    void *r, *p, *q, *xlo;
    double *x64, *b64;
    Red rd;
    CgState cs;
    ProbeGen g;          // probes of the slot's right-hand sides
    int gen_b;           // 1: b is those probes (the true residual regenerates it)
    int disp;            // displacement of the contraction
};
enum { kSlotIter = 1, kSlotInit = 2, kSlotRU = 4, kSlotFinal = 8 };

// A multi-instance block of nv right-hand sides at width W runs at W / 2
// when it fills at most half of W and the launch's stencil mode takes both
// widths (the LDS-tile mode: 32 and 16 lanes; the wavefront-per-site mode:
// 128 and more): an instance's last block then pays for less padding.
inline bool batch_narrow_last(int W, long long nv) { return (W == 32 || W >= 128) && 2 * nv <= W; }

// Multi-instance launches: slot_of[workgroup] = slot; W lanes per slot.
struct BatchLaunch {
    const SlotDesc *sd;  // device array [nslots]
    const int *slot_of;  // device array [total workgroups]
    int nslots, nblocks, W, nc, prec, links, mode;
    hipStream_t stream;
};
void launch_b_init(const BatchLaunch &B, int mixed);
// xmode: as launch_update's (the slots of mixed precision have cs.xdef)
void launch_b_iteration(const BatchLaunch &B, int xmode = 0);
// the stencil with its three dot products (ev0/ev1: its own start and stop)
void launch_b_stencil(const BatchLaunch &B, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_b_update(const BatchLaunch &B, int xmode = 0);  // the finishing kernel, then the vector update
// iterating slots: |r|^2 partials rebuilt from cs.rr (after a new sharing of the workgroups)
void launch_b_reseed(const BatchLaunch &B);
void launch_b_ru(const BatchLaunch &B, int final_stats);
void launch_b_dot(const BatchLaunch &B);
void launch_b_ctrl(const BatchLaunch &B);
// the control words and the slots' active-lane counts only (after a reliable
// update, which has set the lanes' state itself)
void launch_b_count(const BatchLaunch &B);
// the state blocks of the finished slots to the device alias of their pinned mirror
void launch_b_state_out(const BatchLaunch &B, const char *st_all, char *dst, size_t stride);
// a device-side copy of `bytes` (a multiple of 4; both ends 16-byte aligned)
// whose source may be the device alias of pinned host memory
void launch_copy_in(void *dst, const void *src, size_t bytes, hipStream_t s);

int grid_blocks(int ntiles);
// One launch: the neighbour table nbr[N][8] (x + mu, then x - mu) and, from
// the ABI links (complex128 [4][N][nc][nc]; null for the free field), the
// FP64 links [N][4][nc][nc] (u64), and the hop links [N][8][nc][nc], entry
// (x, mu) = U_mu(x), entry (x, 4 + mu) = U_mu(x - mu) (not conjugated), so a
// site's eight hops are one contiguous record, in storage precision prec (u8)
// and in FP64 (u8x).  Null outputs are skipped.
void prepare_links(const Lat &lat, int nc, const void *abi, int *nbr, double *u64, int prec, void *u8,
                   double *u8x, hipStream_t s);

void launch_init_probe(const Launch &L, int prec, const ProbeGen &g, double *b64, void *r, void *p,
                       void *xlo, double *x64, int mixed, const Red &rd, const CgState &cs);
void launch_init_abi(const Launch &L, int prec, const double *babi, long long rhs0, long long nvalid,
                     double *b64, void *r, void *p, void *xlo, double *x64, int mixed, const Red &rd,
                     const CgState &cs);
// Arguments of the stencil launch: q = A pin; with cg (a CG iteration) also
// p^H q and |q|^2 per lane (BF16 storage: r^H q and r^H p too, rin = r), then
// the finishing kernel that forms alpha, the new |r|^2 and beta.
struct StencilArgs {
    bool links = false;
    double diag = 0;
    const void *pin = nullptr;
    const void *rin = nullptr;
    void *q = nullptr;
    const void *U = nullptr;     // hop links [N][8][nc][nc] (gather_links)
    const int *nbr = nullptr;
    int cg = 0;
    Red rd{};
    CgState cs{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // if set: the stencil kernel's own start and stop times
};
void launch_stencil(const Launch &L, int prec, const StencilArgs &a);
// stencil modes 0..6 a launch shape admits, and the choice without timing
bool stencil_mode_valid(const Launch &L, int prec, int mode);
int stencil_mode_rule(const Launch &L, int prec);
// The vector update of a CG iteration: x += alpha p, r -= alpha q,
// p = r + beta p, and |r|^2 per lane into rd.part2.  xmode (FP32 or BF16
// storage with cs.xdef set, else taken as 0): 1 defers this iteration's x
// update to the next update, which must be launched with xmode 2; 0 the
// plain update.
void launch_update(const Launch &L, int prec, void *x, void *r, void *p, const void *q, const Red &rd,
                   const CgState &cs, int xmode = 0);
// x64 += xlo, xlo = 0 (mixed precision)
void launch_fold(const Launch &L, int prec, double *x64, void *xlo);
// The FP64 true residual r = b - q64, with q64 = A x64 computed by the FP64
// stencil beforehand, element by element (gen set: b is regenerated from
// those probes instead of read from b64).  ru_mode 1 (reliable update): r
// becomes it, p is continued from it (FP32) or kept (BF16; restarted as r
// for lanes flagged to restart), then the reliable-update epilogue; ru_mode
// 0: only its norm, for the statistics.  q: A p_prev, read by the FP32
// continuation.
void launch_resid_q(const Launch &L, int prec, const double *b64, const double *q64, void *r, void *p,
                    const void *q, int ru_mode, const Red &rd, const CgState &cs, const ProbeGen *gen);
// cmap[c] = the coarse colour of the sites of fine colour c (-1 for a colour
// no site has); *bad set to 1 when a colour is out of range or two sites of
// one fine colour have different coarse colours (not nested).
void launch_level_map(int N, const int *fine, int nfine, const int *coarse, int ncoarse, int *cmap, int *bad,
                      hipStream_t s);
void launch_displaced_dot(const Launch &L, const ProbeGen &g, int p, const double *x64, const Red &rd,
                          const CgState &cs);
void launch_dot(const Launch &L, const double *a64, const double *b64, const Red &rd,
                const CgState &cs);
void launch_force(const Launch &L, const double *x64, const double *l64, const int *nbr, double scale,
                  int first, double *dU, double *dUbar);
// |r|^2 of every lane from rd.part2 (and, FP64, its convergence), then the
// control word
void launch_ctrl(const Red &rd, const CgState &cs, int W, hipStream_t s);

// Deflation (dense pieces over FP64 blocks [n rows][width], internal layout)
// r = p = b read from b64 in place, xlo = 0, |b|^2 (the init of probes that
// were modified in b64)
void launch_init_b64(const Launch &L, int prec, double *b64, void *r, void *p, void *xlo, double *x64, int mixed,
                     const Red &rd, const CgState &cs);
// cs.tj[j] = sum_x sum_b conj(u_j(x,b)) w_j(x + p e0, b)
void launch_dot_shift(const Launch &L, const double *u, const double *w, int p, const Red &rd, const CgState &cs);
// cs.true_rr[j] = |u_j - theta_j w_j|^2 (theta: device double[W])
void launch_resid_norm(const Launch &L, const double *u, const double *w, const double *theta, const Red &rd,
                       const CgState &cs);
void launch_axpby(long long n, double a, const double *q, double b, const double *v, double *out, hipStream_t s);
void launch_rand_fill(long long n, unsigned long long seed, double *v, hipStream_t s);
void launch_scale_lanes(long long n, int W, const double *sc, const double *v, double *out, hipStream_t s);
// H [WX][WY] = scale * X^H Y over n rows; part: workspace of gram_row_blocks(n)
// * ceil(WX / 64) * ceil(WY / 64) * 64 * 64 complex numbers
int gram_row_blocks(long long n);
void launch_gram(long long n, int WX, int WY, const double *X, const double *Y, double *part, double scale, double *H,
                 hipStream_t s);
// out [n][WY] (+)= X [n][WX] C [WX][WY]
void launch_rot(long long n, int WX, int WY, const double *X, const double *C, double *out, int accumulate,
                hipStream_t s);
void launch_hop_bound(const Lat &lat, int nc, const double *U8, double *out, hipStream_t s);
void launch_to_abi(const Launch &L, const double *x64, double *xabi, long long rhs0, long long nvalid);
void launch_abi_to_internal(const Launch &L, int prec, const double *vabi, long long rhs0,
                            long long nvalid, void *out);
void launch_internal_to_abi_prec(const Launch &L, int prec, const void *in, double *yabi,
                                 long long rhs0, long long nvalid);
void launch_make_probes_abi(const Lat &lat, int nc, const ProbeGen &g, long long nrhs, double *out,
                            hipStream_t s);

}  // namespace dp
