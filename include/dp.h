/*
 * dp.h -- C ABI of the MI355X (gfx950) library for displacement-based probing
 * of Tr(P A^{-1}) (Switzer, Stathopoulos, Romero, Laeuchli, Orginos,
 * "Probing for the trace estimation of a permuted matrix inverse
 * corresponding to a lattice displacement", arXiv:2106.01275).
 *
 * The problem (Sec. 3): A is a nearest-neighbour operator on a 4-D torus,
 * P the permutation that shifts sites by p along dimension 0, and the wanted
 * quantity is Tr(P A^{-1}) = sum_x A^{-1}[x + p e0, x].  It is estimated with
 * Hutchinson's estimator (Sec. 2, eq. (1)) on probing vectors built from a
 * greedy colouring of the displaced distance-k neighbourhoods (Sec. 3,
 * eqs. (5)-(6); Sec. 2.1-2.2, eqs. (3)-(4)); every probe costs one linear
 * solve A x = z, followed by the displaced contraction z^H P x.
 *
 * Conventions shared by every call
 *   - Lattice extents dims[4]; site index idx = ((x0*D1 + x1)*D2 + x2)*D3 + x3
 *     (dimension 0, the displacement dimension, varies slowest).
 *   - (P v)(x) = v(x + p e0).
 *   - Vectors at the ABI are complex128 (re, im interleaved), layout
 *     [rhs][site][colour], colour = 0..nc-1, nc in {1, 3}.
 *   - Links are complex128 [4][N][nc][nc]; U_mu(x)[a][b] connects x to x+mu.
 *   - The operator (free field for nc = 1 and links == NULL, otherwise
 *     gauge covariant):
 *       (A v)(x) = (m2 + 8) v(x) - sum_mu [U_mu(x) v(x+mu) + U_mu(x-mu)^H v(x-mu)].
 *   - The caller owns every buffer passed in; the library never frees one.
 *     "device" buffers live on the context's HIP device; "host" buffers in
 *     host memory.
 *   - Device work is ordered on the stream argument.  Calls that return host
 *     results synchronise that stream before returning.
 *   - No exception crosses the ABI.  Every call returns a dp_status;
 *     dp_last_error() gives a message for the last failure.
 *   - A context is used by one host thread at a time.
 */
#ifndef DP_H
#define DP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dp_status;
enum {
    DP_OK = 0,
    DP_EINVAL = 1,        /* bad argument: dims <= 0, nc not 1 or 3, p < 0, ... */
    DP_ENOMEM = 2,        /* device or host allocation failed */
    DP_EHIP = 3,          /* a HIP runtime call failed */
    DP_ENOCONV = 4,       /* max_iter reached; outputs are written, stats say which */
    DP_EBREAKDOWN = 5,    /* CG breakdown: p^H A p <= 0 or not finite */
    DP_EUNSUPPORTED = 6   /* valid request the library does not support */
};

/* visitation order of the greedy colouring (Sec. 3.1) */
enum { DP_ORDER_NATURAL = 0, DP_ORDER_REDBLACK = 1, DP_ORDER_BEST = 2 };

/* noise of the probing vectors (Sec. 2): real Rademacher, complex
 * Z2 x Z2 stored unnormalised as (+-1) + i(+-1) (quadratic results carry a
 * factor 1/2), and Z4 = {1, i, -1, -i} */
enum { DP_NOISE_REAL_Z2 = 0, DP_NOISE_Z2_COMPLEX = 1, DP_NOISE_Z4 = 2 };

/* storage precision of the inner solver's vectors and links */
enum { DP_PREC_F64 = 0, DP_PREC_F32 = 1, DP_PREC_BF16 = 2 };

typedef struct dp_ctx dp_ctx;

/* Creates a context bound to HIP device hip_device.  The context owns all
 * scratch memory (workspaces, reduction buffers, tuning results). */
dp_status dp_create(dp_ctx **ctx, int32_t hip_device);
void dp_destroy(dp_ctx *ctx);
/* Message of the last failure of a call on ctx (ctx == NULL: of the last
 * context-free call in this thread).  Never NULL. */
const char *dp_last_error(const dp_ctx *ctx);

/*
 * Greedy displaced distance-k colouring (Sec. 3.1; DisColoring and
 * CreateStencil): each site, in the visitation order, gets the smallest
 * colour not used by an already coloured site of
 *     N(x, p, k) = {y != x : |y - (x + p e0)|_1 <= k or |y - (x - p e0)|_1 <= k}
 * (distances on the torus).  Colours are 0-based and dense.
 *   dims      host int32[4], each >= 1.
 *   p         displacement along dimension 0, >= 0.
 *   ks        host int32[nlevels], distances, strictly increasing, >= 0.
 *   nlevels   1: a flat distance-ks[0] colouring.  > 1: nested levels
 *             (hierarchical probing, Sec. 2.3): level l refines every colour
 *             class of level l-1 by a distance-ks[l] colouring of that class;
 *             the children of parent colour c are numbered after those of
 *             colours 0..c-1.
 *   order     DP_ORDER_*; BEST takes the order with fewer colours at the last
 *             level, ties to NATURAL (Sec. 4.1).
 *   colors    host int32[nlevels][N], written.
 *   ncolors   host int32[nlevels], written.
 *   order_used host int32, written with the order taken (may be NULL).
 * Host only; deterministic. */
dp_status dp_build_coloring(const int32_t dims[4], int32_t p, const int32_t *ks,
                            int32_t nlevels, int32_t order, int32_t *colors,
                            int32_t *ncolors, int32_t *order_used);

/*
 * Colouring for several displacements at once (Sec. 3.4): the greedy
 * colouring of N(x, [p_1..p_n], k) = N(x, p_1, k) u ... u N(x, p_n, k).
 *   disp   host int32[ndisp], each >= 0, ndisp >= 1 (ndisp = 1 is
 *          dp_build_coloring).  The other arguments are those of
 *          dp_build_coloring (nested levels included).
 * Host only; deterministic. */
dp_status dp_build_coloring_multi(const int32_t dims[4], const int32_t *disp, int32_t ndisp,
                                  const int32_t *ks, int32_t nlevels, int32_t order, int32_t *colors,
                                  int32_t *ncolors, int32_t *order_used);

/*
 * Tile of the displaced distance-k colouring (Sec. 3.5): along dimension 0
 * (the displacement) at least 2(p+k)+1 sites, along the others at least
 * 2k+1, each rounded up to a power of two and capped at the lattice extent
 * (an extent the power of two does not divide takes its smallest divisor
 * that is at least the minimum).
 *   tile   host int32[4], written. */
dp_status dp_tile_shape(const int32_t dims[4], int32_t p, int32_t k, int32_t tile[4]);

/*
 * Tiled colouring (Sec. 3.5): the greedy (p, k) colouring of the tile torus
 * (dp_tile_shape), repeated over the lattice; valid on the lattice because
 * every tile side holds a whole neighbourhood or equals the lattice extent.
 * With the environment variable DP_COLOR_CACHE naming a directory, tile
 * colourings are read from and written to files there (one per tile, p, k
 * and order), the colouring database of Sec. 3.5.
 *   colors  host int32[N], ncolors host int32, order_used host int32 (may
 *           be NULL), tile host int32[4] (may be NULL): written. */
dp_status dp_build_coloring_tiled(const int32_t dims[4], int32_t p, int32_t k, int32_t order,
                                  int32_t *colors, int32_t *ncolors, int32_t *order_used,
                                  int32_t tile[4]);

/*
 * Clearance of a colouring for displacement p (Sec. 4.3, Table Clearance):
 * for k = 0..kmax, the percentage of the sites at torus L1 distance exactly k
 * from x + p e0 or from x - p e0 (x excluded) that share the colour of x,
 * averaged over all sites x; 0 means distance k is cleared (for a (p0, k0)
 * colouring every k <= k0 - |p0 - p|, Thm. Clearance).
 *   colors  host int32[N]; pct host double[kmax+1], written.
 * Host only; cost N times the number of offsets within reach. */
dp_status dp_clearance(const int32_t dims[4], const int32_t *colors, int32_t p, int32_t kmax,
                       double *pct);

/* Which probing vectors to use (Sec. 2.1-2.2, eqs. (3)-(4)). */
typedef struct {
    int32_t dims[4];
    int32_t nc;                 /* colours per site: 1 or 3 */
    const int32_t *colors_dev;  /* device int32[N], one colouring level */
    int32_t ncolors;            /* number of colours m in colors_dev */
    uint64_t seed;              /* noise seed */
    int32_t sample0;            /* first noise sample s */
    int32_t nsamples;           /* number of noise samples */
    int32_t noise;              /* DP_NOISE_* */
    int32_t dilute;             /* 1: one probe per colour component (n_dil = nc) */
} dp_probe_spec;

/*
 * Writes probing vectors j in [rhs0, rhs0 + nrhs) of the enumeration
 *     j = ((s - sample0) * ncolors + c) * n_dil + a,   n_dil = dilute ? nc : 1:
 *     v_j(x, b) = z0(s, x, b) * [colour(x) == c] * (dilute ? [b == a] : 1),
 * with z0 from the counter-based SplitMix64 hash
 *     h = mix(mix(seed) ^ ((s*N + idx)*nc + b))
 * (REAL_Z2: -1 if bit 63 else +1; Z2_COMPLEX: re from bit 63, im from bit 62;
 *  Z4: h >> 62 -> {1, i, -1, -i}).
 *   out  device complex128 [nrhs][N][nc], caller-owned.
 * Values are exact (+-1, +-i, +-1+-i). */
dp_status dp_make_probes(dp_ctx *ctx, const dp_probe_spec *ps, int64_t rhs0, int64_t nrhs,
                         void *out, hipStream_t stream);

/* One operator instance. */
typedef struct {
    int32_t dims[4];
    int32_t nc;          /* 1 or 3 */
    double m2;           /* mass term */
    const void *links;   /* device complex128 [4][N][nc][nc]; NULL means U = 1 */
} dp_operator;

typedef struct {
    double tol;             /* stop when |b - A x| / |b| <= tol (FP64 true residual
                               for mixed precision; recursive residual for F64) */
    int32_t max_iter;       /* iteration limit per right-hand side (0: 100000) */
    int32_t inner;          /* DP_PREC_*: storage of the inner CG vectors and links;
                               F32 and BF16 accumulate in FP32 and are refined by
                               FP64 reliable updates */
    int32_t rhs_block;      /* right-hand sides solved together (W): 0 = autotune
                               (one instance: a few timed CG iterations per width,
                               cached, DP_TUNE_CACHE names a file; the least time
                               for all right-hand sides, padding of the last block
                               included; several: the least traffic per useful
                               lane-site, padding of each instance's last block
                               included), else a power of two <= 256 whose block
                               vectors (N * nc * W elements of the inner precision)
                               stay under 4 GiB (DP_EINVAL otherwise) */
    double reliable_delta;  /* mixed precision: replace the residual by the FP64
                               true residual once it dropped by this factor; a lane
                               that reaches it waits for that update before it moves
                               on (0: 0.002 for BF16, 1e-3 for F32).  BF16 storage
                               resolves about 3 digits: smaller values cost extra
                               iterations, larger ones extra FP64 updates */
    int32_t use_graph;      /* 1: replay the iteration loop from a captured hipGraph */
    int32_t profile;        /* 1: time stencil kernel launches with HIP events (single
                               instance: every 8th when a launch moves less than 256 MB of
                               algorithmic traffic, else all; many instances: all) */
} dp_solve_opts;

typedef struct {
    int64_t nrhs;            /* right-hand sides solved */
    int64_t rhs_iters;       /* sum over right-hand sides of CG iterations to convergence */
    int32_t max_iters;       /* largest iteration count of one right-hand side */
    int32_t nconverged;      /* right-hand sides that met tol */
    int32_t nbreakdown;      /* right-hand sides that broke down */
    int32_t reliable_updates;/* FP64 reliable updates performed (all blocks) */
    double max_true_resid;   /* max over right-hand sides of |b - A x| / |b| (FP64) */
    int32_t rhs_block;       /* W used */
    int32_t stencil_launches;/* profile = 1: stencil kernel launches timed (see profile) */
    double stencil_ms;       /* profile = 1: summed duration of those launches */
    double stencil_bytes;    /* profile = 1: their algorithmic bytes, per lattice site of a
                                launch 2*W*V + 4*L (read p and write q for the W right-hand
                                sides, read each of the 4 links once), V = bytes of one site
                                vector, L = bytes of one link matrix (0 without links).
                                A multi-instance launch (solve_batch / trace_estimate with
                                ninst > 1) covers every instance: its totals are reported
                                in the stats of instance 0 only */
    double seconds;          /* wall time of the call */
    double stencil_bytes_all;/* profile = 1: algorithmic bytes of all the stencil launches,
                                timed or not (same accounting as stencil_bytes) */
} dp_solve_stats;

/*
 * Solves A_i x = b for every right-hand side of every instance with CG
 * (Hestenes-Stiefel, x0 = 0).  These solves, one per probing vector, are
 * what the paper names the bulk of the cost of the estimator (Sec. 2.1):
 * every probe of eqs. (3)-(4) costs one of them.
 *   ninst  number of instances (>= 1).
 *   ops    host dp_operator[ninst].
 *   b      host array [ninst] of device complex128 [nrhs[i]][N_i][nc_i].
 *   x      host array [ninst] of device complex128 [nrhs[i]][N_i][nc_i], written.
 *   nrhs   host int64[ninst].
 *   st     host dp_solve_stats[ninst], written (may be NULL).
 * Returns DP_ENOCONV / DP_EBREAKDOWN (outputs still written) when some
 * right-hand side failed. */
dp_status dp_solve_batch(dp_ctx *ctx, int32_t ninst, const dp_operator *ops,
                         const void *const *b, void *const *x, const int64_t *nrhs,
                         const dp_solve_opts *o, dp_solve_stats *st, hipStream_t stream);

typedef struct {
    double tr[2];            /* the estimate T = (1/s) sum_s T_s (complex) */
    double stderr_;          /* sqrt(var_s(T_s) / s), unbiased variance; NaN if s < 2 */
    double *per_sample;      /* host double[nsamples][2] (T_s), written if non-NULL */
    double *per_rhs;         /* host double[nrhs][2] (t_j, unnormalised), written if non-NULL */
    dp_solve_stats solve;    /* statistics of the solves */
} dp_trace_result;

/*
 * Probed estimate of Tr(P A^{-1}) (eqs. (1), (3), (4); Sec. 3):
 *     t_j = sum_x sum_b conj(v_j(x,b)) x_j(x + p e0, b),  x_j = A^{-1} v_j,
 *     T_s = norm * sum_{j in sample s} t_j  (norm = 1/2 for Z2_COMPLEX, else 1),
 *     T = mean over samples.
 * Probes are generated on the device from the spec; solutions are contracted
 * as soon as their block converges and are never all held at once.
 *   ninst, ops, p, ps, out: arrays [ninst] (host); instance i uses ops[i],
 *   displacement p[i] >= 0 and probes ps[i] (ps[i].dims/nc must equal ops[i]'s).
 *   out[i].per_sample / per_rhs are optional caller-owned host buffers. */
dp_status dp_trace_estimate(dp_ctx *ctx, int32_t ninst, const dp_operator *ops,
                            const int32_t *p, const dp_probe_spec *ps, const dp_solve_opts *o,
                            dp_trace_result *out, hipStream_t stream);

/*
 * One probe set, many displacements (Sec. 4.3): the probes of ps (built from
 * a colouring for one (p0, k0)) are solved once and every solution is
 * contracted with each displacement disp[n] (any sign),
 *     t_j(n) = sum_x sum_b conj(v_j(x,b)) x_j(x + disp[n] e0, b),
 * giving the estimate of Tr(P_n A^{-1}) for all n at the cost of one set of
 * solves.  By Thm. Clearance the (p0, k0) colouring still removes every
 * neighbour up to distance max(0, k0 - |p0 - n|) for displacement n.
 *   disp   host int32[ndisp], ndisp >= 1.
 *   out    host dp_trace_result[ndisp], written (out[n] for disp[n]; each
 *          carries the same solve statistics).
 * Single instance; the other conventions are those of dp_trace_estimate. */
dp_status dp_trace_multi(dp_ctx *ctx, const dp_operator *op, const int32_t *disp, int32_t ndisp,
                         const dp_probe_spec *ps, const dp_solve_opts *o, dp_trace_result *out,
                         hipStream_t stream);

/*
 * Every level of a nested (hierarchical) colouring from the solves of the
 * finest one (Sec. 2.3): with one noise vector z0 for all levels the probe of
 * a class is the sum of the probes of its sub-classes, so by linearity
 *     T_l = sum_j v_{parent_l(j)}^H P x_j,   x_j = A^{-1} v_j,
 * the sum over the finest probes v_j of each solution contracted with the
 * probe of its parent class on level l.  Equal, up to the solver tolerance,
 * to dp_trace_estimate on level l's colouring with the same seed and
 * samples, for the price of one set of solves.
 *   ps              the finest level (its colouring and noise).
 *   coarse_colors   host array of ncoarse device int32[N] colourings, each
 *                   nested with the fine one (every fine class inside one
 *                   coarse class), coarse_ncolors their colour counts.
 *   out             host dp_trace_result[ncoarse + 1], written: out[0] the
 *                   finest level (as dp_trace_estimate), out[1 + l] level l;
 *                   per_rhs of a coarse level holds the per-solution terms
 *                   v_{parent_l(j)}^H P x_j.
 * DP_EINVAL when a coarse colouring is not nested in the fine one or a colour
 * is outside [0, ncolors) (checked on the device before any solve).
 * Single instance; the other conventions are those of dp_trace_estimate. */
dp_status dp_trace_levels(dp_ctx *ctx, const dp_operator *op, int32_t p, const dp_probe_spec *ps,
                          int32_t ncoarse, const int32_t *const *coarse_colors, const int32_t *coarse_ncolors,
                          const dp_solve_opts *o, dp_trace_result *out, hipStream_t stream);

/*
 * Adjoint gradient of the probed estimate T (same probes as dp_trace_estimate).
 * The paper has no gradient: this call is an addition to its method, derived
 * from dT = -lambda^H dA x for each probe (A Hermitian), and its results are
 * checked against central finite differences of T and, for the free field,
 * against the derivative of the Fourier closed form of Tr(P A^{-1}).
 * With x_j = A^{-1} v_j and lambda_j = A^{-1} P^T v_j ((P^T v)(y) = v(y - p e0)),
 * recomputed here (no Krylov history is kept):
 *     dT/dm2              = -(norm/s) sum_j lambda_j^H x_j
 *     dT/dU_mu(x)[a][b]    =  (norm/s) sum_j conj(lambda_j(x)_a) x_j(x+mu)_b
 *     dT/dconj(U)_mu(x)[a][b] = (norm/s) sum_j x_j(x)_a conj(lambda_j(x+mu)_b)
 * (Wirtinger derivatives with U and conj(U) independent).
 *   dT_dm2    host double[2], written.
 *   dT_dU, dT_dUbar  device complex128 [4][N][nc][nc], caller-owned, overwritten
 *             (either may be NULL). */
dp_status dp_trace_grad(dp_ctx *ctx, const dp_operator *op, int32_t p, const dp_probe_spec *ps,
                        const dp_solve_opts *o, dp_trace_result *out, double dT_dm2[2],
                        void *dT_dU, void *dT_dUbar, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * single-instance solve of dp_solve_batch (same kernels, same results) with
 * every workspace buffer in one static device array of
 * DP_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on holds
 * until the process ends.  The call allocates nothing: no hipMalloc, no
 * hipFree, no pool, graph or event.
 *   op     host dp_operator (one instance).
 *   b      device complex128 [nrhs][N][nc], caller-owned, read.
 *   x      device complex128 [nrhs][N][nc], caller-owned, written.
 *   o      as dp_solve_batch, except that use_graph and profile must be 0
 *          (DP_EINVAL otherwise) and rhs_block = 0 takes the widest power of
 *          two <= 32 (and <= the next power of two of nrhs) whose workspace
 *          fits, without timing; an explicit rhs_block must fit.
 *   st     host dp_solve_stats, written (may be NULL).
 * DP_EINVAL, with the bytes needed in the message, when the workspace of the
 * lattice at that width exceeds the array.  The workspace is, per site,
 * 32 (neighbours) + [links] 8 nc^2 s (+ 8 nc^2 16 mixed) + W nc (32 + 3 s
 * (+ 16 + s mixed)) bytes, s = 16 / 8 / 4 for F64 / F32 / BF16, plus 48 W
 * per workgroup and 23 KB of per-lane state: e.g. an 8^4 x 3 lattice with
 * links at F32, W = 32 takes about 40 MB.  Every call on one GPU uses that GPU's single
 * array (each call writes every part of it it reads, so no earlier contents
 * matter): calls that overlap on one GPU, from two host threads or two
 * contexts, race and must not be made. */
#define DP_NOALLOC_SCRATCH_BYTES (64ull << 20)
dp_status dp_solve_noalloc(dp_ctx *ctx, const dp_operator *op, const void *b, void *x, int64_t nrhs,
                           const dp_solve_opts *o, dp_solve_stats *st, hipStream_t stream);

/*
 * y = A v for nrhs vectors with the stencil kernel of the given storage
 * precision (DP_PREC_*): inputs are rounded to that precision, the result is
 * returned in complex128.  v, y: device complex128 [nrhs][N][nc].
 * The operator of the problem statement, exposed for verification. */
dp_status dp_apply(dp_ctx *ctx, const dp_operator *op, int32_t prec, const void *v, void *y,
                   int64_t nrhs, hipStream_t stream);

/*
 * Deflation (Sec. Deflation): with V the Ritz vectors of the nvec smallest
 * eigenvalues of the Hermitian A (orthonormal, V^H A V = Theta) and the
 * oblique projector Q = A V (V^H A V)^{-1} V^H, the trace splits exactly as
 *     Tr(P A^{-1}) = Tr(P A^{-1} Q) + Tr(P A^{-1} (I - Q)),
 * where A^{-1} Q = V Theta^{-1} V^H, so the first term is the sum over the
 * vectors of theta_i^{-1} sum_x sum_b conj(v_i(x,b)) v_i(x + p e0, b), and
 * the probes estimate only the second: t_j = z_j^H P A^{-1} (I - Q) z_j.
 * The identity holds for any V; how much variance the split removes (and how
 * many CG iterations the deflated right-hand sides save) depends on how well
 * V spans the low modes.
 *
 * The vectors come from a Chebyshev-filtered subspace iteration with
 * Rayleigh-Ritz (FP64, on the device) over a subspace of
 * W = next power of two of nvec + max(4, nvec / 4) vectors (W <= 128): each
 * outer iteration applies a degree-`degree` Chebyshev polynomial of A that
 * damps [theta_max, bound] (bound: a Gershgorin-type bound of the spectrum
 * from the links), then orthonormalises and rotates to Ritz vectors.  It
 * stops when the relative Ritz residual |A v_i - theta_i v_i| / theta_i of
 * every kept vector is <= tol, or after max_outer iterations.
 */
typedef struct dp_deflation dp_deflation;

typedef struct {
    int32_t degree;     /* Chebyshev degree per outer iteration (0: 16) */
    int32_t max_outer;  /* outer iterations (0: 60) */
    double tol;         /* relative Ritz residual of the kept vectors (0: 1e-10) */
    uint64_t seed;      /* start vectors */
} dp_eig_opts;

/*
 *   op     the operator (the same one must be passed to dp_trace_deflated).
 *   nvec   kept vectors, 1 <= nvec <= 103 (so that W <= 128).
 *   o      may be NULL (defaults).
 *   out    written: a deflation object owning its device memory (free it
 *          with dp_deflation_destroy; it stays valid after the context is
 *          destroyed only as long as the device is alive).
 * Returns DP_ENOCONV (the object is still written) when max_outer was
 * reached before tol. */
dp_status dp_deflation_create(dp_ctx *ctx, const dp_operator *op, int32_t nvec, const dp_eig_opts *o,
                              dp_deflation **out, hipStream_t stream);

/*   evals, resid  host double[nvec] (may be NULL): Ritz values (ascending)
 *                 and relative Ritz residuals; outer, subspace (may be NULL):
 *                 outer iterations run and the subspace size W. */
dp_status dp_deflation_info(const dp_deflation *d, double *evals, double *resid, int32_t *outer,
                            int32_t *subspace);

/*   out    device complex128 [nvec][N][nc], caller-owned, written (the Ritz
 *          vectors in the ABI layout).
 * DP_EINVAL when d lives on another device than ctx. */
dp_status dp_deflation_vectors(dp_ctx *ctx, const dp_deflation *d, void *out, hipStream_t stream);

/*
 * Deflated probed estimate of Tr(P A^{-1}): right-hand sides
 * b_j = (I - Q) z_j = z_j - A V Theta^{-1} V^H z_j (formed on the device,
 * FP64), solved and contracted as in dp_trace_estimate;
 *     T_s = tr_defl + norm * sum_{j in sample s} t_j,   T = mean over samples.
 *   tr_defl  host double[2] (may be NULL): Tr(P A^{-1} Q), written.
 * out.per_sample holds the T_s (each an unbiased estimate of the whole
 * trace), out.per_rhs the t_j. Single instance, p >= 0.  DP_EINVAL when d
 * was built for an operator of other dims, nc, m2 or link presence (its
 * link values are not compared: passing other links gives a wrong split),
 * or lives on another device than ctx. */
dp_status dp_trace_deflated(dp_ctx *ctx, const dp_operator *op, const dp_deflation *d, int32_t p,
                            const dp_probe_spec *ps, const dp_solve_opts *o, dp_trace_result *out,
                            double tr_defl[2], hipStream_t stream);

void dp_deflation_destroy(dp_deflation *d);

#ifdef __cplusplus
}
#endif

#endif /* DP_H */
