/*
 * Oracle for displacement-based probing of Tr(P A^{-1})
 * (Switzer, Stathopoulos, Romero, Laeuchli, Orginos, arXiv:2106.01275).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, FP64 CPU
 * implementation of what the GPU library computes.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (one reading of the paper, applied everywhere):
 *   - 4-D torus, dims D[0..3]; site index idx = ((x0*D1 + x1)*D2 + x2)*D3 + x3,
 *     dimension 0 is the displacement dimension and varies slowest
 *     (Sec. 3, the permutation built from Index2Coord/Coord2Index).
 *     A lattice with d < 4 active dimensions uses D = 1 and zero stencil
 *     offsets in the inactive ones.
 *   - (P v)(x) = v(x + p e0), so Tr(P A^{-1}) = sum_x A^{-1}[x+p e0, x]
 *     (Sec. 3, the MATLAB permutation).
 *   - Vectors are complex, element (site, colour b) at idx*nc + b.
 *   - Links U[mu][idx][a][b] (complex), U_mu(x) connects x to x + mu.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* Lattice geometry                                                    */
/* ------------------------------------------------------------------ */

static int64_t volume(const int32_t *D) {
    return (int64_t)D[0] * D[1] * D[2] * D[3];
}

static void to_coords(int64_t idx, const int32_t *D, int32_t *x) {
    for (int d = 3; d >= 0; --d) {
        x[d] = (int32_t)(idx % D[d]);
        idx /= D[d];
    }
}

static int32_t wrap(int64_t v, int32_t n) {
    int64_t r = v % n;
    return (int32_t)(r < 0 ? r + n : r);
}

static int64_t to_index(const int32_t *x, const int32_t *D) {
    int64_t idx = 0;
    for (int d = 0; d < 4; ++d) idx = idx * D[d] + wrap(x[d], D[d]);
    return idx;
}

/* site reached from idx by the offset o (componentwise, modulo D) */
static int64_t shifted(int64_t idx, const int32_t *o, const int32_t *D) {
    int32_t x[4], y[4];
    to_coords(idx, D, x);
    for (int d = 0; d < 4; ++d) y[d] = x[d] + o[d];
    return to_index(y, D);
}

/* ------------------------------------------------------------------ */
/* Stencil: the displaced distance-k neighbourhood N(0, p, k)          */
/* Sec. 3, eq. (5)-(6): the union of two L1 balls of radius k centred  */
/* at +p e0 and -p e0, with the centre itself excluded.  (Our reading  */
/* of the missing CreateStencil algorithm, Sec. 3.1.)                  */
/* ------------------------------------------------------------------ */

static int l1_from(const int32_t *o, int32_t c0) {
    int s = abs(o[0] - c0);
    for (int d = 1; d < 4; ++d) s += abs(o[d]);
    return s;
}

/* Writes up to cap offsets (4 ints each) into out and returns the total
 * number of offsets.  d = number of active dimensions (1..4). */
int or_stencil(int32_t p, int32_t k, int32_t d, int32_t *out, int64_t cap) {
    int64_t n = 0;
    int32_t R0 = p + k;
    int32_t R[4] = {R0, d > 1 ? k : 0, d > 2 ? k : 0, d > 3 ? k : 0};
    int32_t o[4];
    for (o[0] = -R[0]; o[0] <= R[0]; ++o[0])
        for (o[1] = -R[1]; o[1] <= R[1]; ++o[1])
            for (o[2] = -R[2]; o[2] <= R[2]; ++o[2])
                for (o[3] = -R[3]; o[3] <= R[3]; ++o[3]) {
                    if (o[0] == 0 && o[1] == 0 && o[2] == 0 && o[3] == 0) continue;
                    if (l1_from(o, p) <= k || l1_from(o, -p) <= k) {
                        if (out && n < cap) memcpy(out + 4 * n, o, sizeof o);
                        ++n;
                    }
                }
    return (int)n;
}

/* ------------------------------------------------------------------ */
/* Visitation orders (Sec. 3.1): natural = increasing index;           */
/* red-black = sites with even coordinate sum, then odd, each in index */
/* order (our reading; the paper does not define its red-black order). */
/* ------------------------------------------------------------------ */

void or_order(const int32_t *D, int32_t order, int64_t *out) {
    int64_t N = volume(D), n = 0;
    if (order == 0) {
        for (int64_t i = 0; i < N; ++i) out[i] = i;
        return;
    }
    for (int parity = 0; parity < 2; ++parity)
        for (int64_t i = 0; i < N; ++i) {
            int32_t x[4];
            to_coords(i, D, x);
            if (((x[0] + x[1] + x[2] + x[3]) & 1) == parity) out[n++] = i;
        }
}

/* ------------------------------------------------------------------ */
/* Greedy displaced colouring (Sec. 3.1; our reading of the missing    */
/* DisColoring algorithm).  Visit sites in the given order; a site gets */
/* the smallest colour not carried by an already coloured site of its  */
/* neighbourhood N(x,p,k).  Colours are 0-based.  With a parent        */
/* colouring given, only neighbours sharing the parent colour count     */
/* (used for the nested levels, see or_color_nested).                  */
/* ------------------------------------------------------------------ */

/* greedy first fit over the neighbourhood given by the S offsets st[S][4] */
static int greedy_offsets(const int32_t *D, const int32_t *st, int S, int32_t order,
                          const int32_t *parent, int32_t *col) {
    int64_t N = volume(D);
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    or_order(D, order, ord);
    /* at most |stencil| neighbours, so at most S+1 colours (Sec. 3.1) */
    unsigned char *used = (unsigned char *)calloc((size_t)S + 2, 1);
    for (int64_t i = 0; i < N; ++i) col[i] = -1;
    int ncol = 0;
    for (int64_t t = 0; t < N; ++t) {
        int64_t x = ord[t];
        memset(used, 0, (size_t)S + 2);
        for (int s = 0; s < S; ++s) {
            int64_t y = shifted(x, st + 4 * s, D);
            if (y == x || col[y] < 0) continue;
            if (parent && parent[y] != parent[x]) continue;
            used[col[y]] = 1;
        }
        int c = 0;
        while (used[c]) ++c;
        col[x] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(used);
    free(ord);
    return ncol;
}

static int greedy(const int32_t *D, int32_t d, int32_t p, int32_t k, int32_t order,
                  const int32_t *parent, int32_t *col) {
    int S = or_stencil(p, k, d, NULL, 0);
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(S > 0 ? S : 1));
    or_stencil(p, k, d, st, S);
    int ncol = greedy_offsets(D, st, S, order, parent, col);
    free(st);
    return ncol;
}

int or_color(const int32_t *D, int32_t d, int32_t p, int32_t k, int32_t order,
             int32_t *colors) {
    return greedy(D, d, p, k, order, NULL, colors);
}

/* Multiple displacements (Sec. 3.4): the neighbourhood is the union
 * N(x,p_1,k) u ... u N(x,p_n,k); the offsets of the n stencils are simply
 * concatenated (an offset listed twice marks the same colour twice). */
int or_color_multi(const int32_t *D, int32_t d, const int32_t *ps, int32_t np, int32_t k,
                   int32_t order, int32_t *colors) {
    int S = 0;
    for (int i = 0; i < np; ++i) S += or_stencil(ps[i], k, d, NULL, 0);
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(S > 0 ? S : 1));
    int at = 0;
    for (int i = 0; i < np; ++i) {
        int Si = or_stencil(ps[i], k, d, NULL, 0);
        or_stencil(ps[i], k, d, st + 4 * at, Si);
        at += Si;
    }
    int ncol = greedy_offsets(D, st, S, order, NULL, colors);
    free(st);
    return ncol;
}

/* Nested (hierarchical) displaced colouring for distances ks[0] < ks[1] < ...
 * Hierarchical probing (Sec. 2.3) needs: same colour at a level implies
 * same colour at every coarser level.  The paper gives no displaced
 * hierarchical algorithm; our reading: level l splits each level-(l-1)
 * colour class by a greedy distance-ks[l] colouring restricted to that
 * class (sub-colour s(x)), and numbers the children of parent colour c
 * consecutively after those of colours 0..c-1.
 * colors is [nlev][N]; ncolors is [nlev]. */
int or_color_nested(const int32_t *D, int32_t d, int32_t p, const int32_t *ks,
                    int32_t nlev, int32_t order, int32_t *colors, int32_t *ncolors) {
    int64_t N = volume(D);
    ncolors[0] = greedy(D, d, p, ks[0], order, NULL, colors);
    for (int l = 1; l < nlev; ++l) {
        const int32_t *par = colors + (size_t)(l - 1) * N;
        int32_t *cur = colors + (size_t)l * N;
        int32_t *sub = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
        greedy(D, d, p, ks[l], order, par, sub);
        int32_t np = ncolors[l - 1];
        int32_t *cnt = (int32_t *)calloc((size_t)np, sizeof(int32_t));
        int32_t *off = (int32_t *)calloc((size_t)np + 1, sizeof(int32_t));
        for (int64_t i = 0; i < N; ++i)
            if (sub[i] + 1 > cnt[par[i]]) cnt[par[i]] = sub[i] + 1;
        for (int c = 0; c < np; ++c) off[c + 1] = off[c] + cnt[c];
        for (int64_t i = 0; i < N; ++i) cur[i] = off[par[i]] + sub[i];
        ncolors[l] = off[np];
        free(cnt);
        free(off);
        free(sub);
    }
    return ncolors[nlev - 1];
}

/* ------------------------------------------------------------------ */
/* Noise.  The paper specifies no generator; both sides implement the  */
/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014) as a   */
/* counter-based hash:  h = mix(mix(seed) ^ ((s*N + idx)*nc + b)).     */
/* kind 0 = real Rademacher {+1,-1} (Sec. 2, eq. (1));                  */
/* kind 1 = complex Z2 x Z2, stored unnormalised as (+-1) + i(+-1);     */
/* kind 2 = Z4 {1, i, -1, -i} (Sec. 2).                                  */
/* ------------------------------------------------------------------ */

uint64_t or_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static cplx noise_value(uint64_t seed, int64_t s, int64_t N, int64_t idx, int32_t nc,
                        int32_t b, int32_t kind) {
    uint64_t ctr = ((uint64_t)s * (uint64_t)N + (uint64_t)idx) * (uint64_t)nc + (uint64_t)b;
    uint64_t h = or_mix64(or_mix64(seed) ^ ctr);
    int top = (int)(h >> 63), next = (int)((h >> 62) & 1);
    if (kind == 0) return top ? -1.0 : 1.0;
    if (kind == 1) return (top ? -1.0 : 1.0) + (next ? -1.0 : 1.0) * I;
    switch ((int)(h >> 62)) {
        case 0: return 1.0;
        case 1: return I;
        case 2: return -1.0;
        default: return -I;
    }
}

/* quadratic forms in unnormalised complex Z2 noise carry |z|^2 = 2 */
static double noise_norm(int32_t kind) { return kind == 1 ? 0.5 : 1.0; }

/* Unbiased probing vector (Sec. 2.2, eq. (4)): z0 masked to the sites of
 * colour c (eq. (3)); with dilution only colour component a is kept
 * (Sec. 4.2 dilutes every internal degree of freedom). */
void or_probe(const int32_t *D, int32_t nc, const int32_t *colors, uint64_t seed,
              int64_t s, int32_t c, int32_t a, int32_t dilute, int32_t kind, double *out) {
    int64_t N = volume(D);
    cplx *v = (cplx *)out;
    for (int64_t x = 0; x < N; ++x)
        for (int32_t b = 0; b < nc; ++b) {
            cplx z = 0.0;
            if (colors[x] == c && (!dilute || b == a)) z = noise_value(seed, s, N, x, nc, b, kind);
            v[x * nc + b] = z;
        }
}

/* ------------------------------------------------------------------ */
/* Operator: (A v)(x) = (m2 + 8) v(x)                                   */
/*                      - sum_mu [ U_mu(x) v(x+mu) + U_mu(x-mu)^H v(x-mu) ] */
/* links == NULL means U = 1 (free field).                              */
/* ------------------------------------------------------------------ */

static void apply_serial(const int32_t *D, int32_t nc, double m2, const double *links,
                         const cplx *in, cplx *out);

void or_apply(const int32_t *D, int32_t nc, double m2, const double *links, const double *in,
              double *out) {
    apply_serial(D, nc, m2, links, (const cplx *)in, (cplx *)out);
}

/* ------------------------------------------------------------------ */
/* Conjugate gradients (Hestenes-Stiefel), x0 = 0, stop when the        */
/* recursive residual satisfies |r|/|b| <= tol.  Returns the iteration  */
/* count, -1 on breakdown (p^H A p <= 0 or not finite), -2 when maxit   */
/* is exhausted.  relres receives the true residual |b - A x| / |b|.    */
/* ------------------------------------------------------------------ */

static double dotr(const cplx *a, const cplx *b, int64_t n) { /* Re(a^H b) */
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
    return s;
}

int or_cg(const int32_t *D, int32_t nc, double m2, const double *links, const double *b_,
          double *x_, double tol, int32_t maxit, double *relres) {
    int64_t n = volume(D) * nc;
    const cplx *b = (const cplx *)b_;
    cplx *x = (cplx *)x_;
    cplx *r = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *q = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; p[i] = b[i]; }
    double bb = dotr(b, b, n), rr = bb;
    int it = 0, status = 0;
    if (bb > 0.0) {
        for (;;) {
            if (it >= maxit) { status = -2; break; }
            apply_serial(D, nc, m2, links, p, q);
            double pq = dotr(p, q, n);
            if (!(pq > 0.0) || !isfinite(pq)) { status = -1; break; }
            double alpha = rr / pq;
            for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            double rr_new = dotr(r, r, n);
            ++it;
            if (sqrt(rr_new / bb) <= tol) break;
            double beta = rr_new / rr;
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            rr = rr_new;
        }
    }
    if (relres) {
        apply_serial(D, nc, m2, links, x, q);
        double e = 0.0;
        for (int64_t i = 0; i < n; ++i) { cplx d = b[i] - q[i]; e += creal(conj(d) * d); }
        *relres = bb > 0.0 ? sqrt(e / bb) : 0.0;
    }
    free(r); free(p); free(q);
    return status ? status : it;
}

/* the operator, single-threaded (callers parallelise over right-hand sides) */
static void apply_serial(const int32_t *D, int32_t nc, double m2, const double *links_,
                         const cplx *in, cplx *out) {
    int64_t N = volume(D);
    const cplx *U = (const cplx *)links_;
    for (int64_t x = 0; x < N; ++x) {
        int32_t e[4] = {0, 0, 0, 0};
        int64_t xp[4], xm[4];
        for (int mu = 0; mu < 4; ++mu) {
            e[mu] = 1;  xp[mu] = shifted(x, e, D);
            e[mu] = -1; xm[mu] = shifted(x, e, D);
            e[mu] = 0;
        }
        for (int a = 0; a < nc; ++a) {
            cplx acc = (m2 + 8.0) * in[x * nc + a];
            for (int mu = 0; mu < 4; ++mu)
                for (int b = 0; b < nc; ++b) {
                    cplx uf = U ? U[((size_t)mu * N + x) * nc * nc + a * nc + b] : (a == b);
                    cplx ub = U ? conj(U[((size_t)mu * N + xm[mu]) * nc * nc + b * nc + a]) : (a == b);
                    acc -= uf * in[xp[mu] * nc + b] + ub * in[xm[mu] * nc + b];
                }
            out[x * nc + a] = acc;
        }
    }
}

/* Many independent solves, one right-hand side per thread. b and x are
 * [nrhs][N][nc] complex; iters/relres are [nrhs]. */
void or_cg_many(const int32_t *D, int32_t nc, double m2, const double *links, int64_t nrhs,
                const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                double *relres) {
    int64_t n2 = volume(D) * nc * 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < nrhs; ++j)
        iters[j] = or_cg(D, nc, m2, links, b + j * n2, x + j * n2, tol, maxit,
                         relres ? relres + j : NULL);
}

/* ------------------------------------------------------------------ */
/* Probed trace estimate of Tr(P A^{-1}) (Sec. 2.1-2.2, eq. (1), (3),  */
/* (4); Sec. 3 for P).  Right-hand side j of the batch is              */
/*   j = ((s - s0) * ncolors + c) * ndil + a,   ndil = dilute ? nc : 1.  */
/* For each: t_j = z_j^H P x_j with x_j = A^{-1} z_j, i.e.              */
/*   t_j = sum_x sum_b conj(z_j(x,b)) x_j(x + p e0, b).                   */
/* T_s = norm * sum over the probes of sample s;  T = mean_s T_s;       */
/* stderr = sqrt(var_s(T_s) / ns) with the unbiased sample variance.    */
/* out: [0..1] T, [2] stderr; per_sample: [ns] complex; tj: [nrhs]      */
/* complex (may be NULL); iters: [nrhs] (may be NULL).                  */
/* ------------------------------------------------------------------ */

static cplx displaced_dot(const int32_t *D, int32_t nc, int32_t p, const cplx *z,
                          const cplx *x) {
    int64_t N = volume(D);
    int32_t e[4] = {p, 0, 0, 0};
    cplx t = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t ip = shifted(i, e, D);
        for (int b = 0; b < nc; ++b) t += conj(z[i * nc + b]) * x[ip * nc + b];
    }
    return t;
}

int or_trace(const int32_t *D, int32_t nc, double m2, const double *links, int32_t p,
             const int32_t *colors, int32_t ncolors, uint64_t seed, int64_t s0, int64_t ns,
             int32_t kind, int32_t dilute, double tol, int32_t maxit, double *out,
             double *per_sample, double *tj_out, int32_t *iters_out) {
    int64_t N = volume(D), n = N * nc;
    int32_t ndil = dilute ? nc : 1;
    int64_t nrhs = ns * ncolors * ndil;
    cplx *tj = (cplx *)malloc(sizeof(cplx) * (size_t)nrhs);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t j = 0; j < nrhs; ++j) {
        int64_t s = s0 + j / ((int64_t)ncolors * ndil);
        int32_t c = (int32_t)((j / ndil) % ncolors), a = (int32_t)(j % ndil);
        cplx *z = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *x = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        or_probe(D, nc, colors, seed, s, c, a, dilute, kind, (double *)z);
        int it = or_cg(D, nc, m2, links, (const double *)z, (double *)x, tol, maxit, NULL);
        if (it < 0) bad = 1;
        if (iters_out) iters_out[j] = it;
        tj[j] = displaced_dot(D, nc, p, z, x);
        free(z);
        free(x);
    }
    double norm = noise_norm(kind);
    cplx T = 0.0;
    cplx *Ts = (cplx *)calloc((size_t)ns, sizeof(cplx));
    for (int64_t j = 0; j < nrhs; ++j) Ts[j / ((int64_t)ncolors * ndil)] += norm * tj[j];
    for (int64_t s = 0; s < ns; ++s) T += Ts[s];
    T /= (double)ns;
    double var = 0.0;
    for (int64_t s = 0; s < ns; ++s) {
        cplx d = Ts[s] - T;
        var += creal(conj(d) * d);
    }
    out[0] = creal(T);
    out[1] = cimag(T);
    out[2] = ns > 1 ? sqrt(var / (double)(ns - 1) / (double)ns) : NAN;
    if (per_sample) memcpy(per_sample, Ts, sizeof(cplx) * (size_t)ns);
    if (tj_out) memcpy(tj_out, tj, sizeof(cplx) * (size_t)nrhs);
    free(Ts);
    free(tj);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Adjoint gradient of the probed estimate T (same inputs as or_trace). */
/* With x_j = A^{-1} z_j and lambda_j = A^{-1} P^T z_j  (A Hermitian,   */
/* (P^T v)(y) = v(y - p e0)), dt_j = -lambda_j^H dA x_j, giving          */
/*   dT/dm2            = -norm/ns sum_j lambda_j^H x_j                    */
/*   dT/dU_mu(x)[a][b]  =  norm/ns sum_j conj(lambda_j(x)_a) x_j(x+mu)_b  */
/*   dT/dUbar_mu(x)[a][b] = norm/ns sum_j x_j(x)_a conj(lambda_j(x+mu)_b) */
/* (Wirtinger derivatives, U and conj(U) independent).  dU and dUbar are */
/* [4][N][nc][nc] complex and may be NULL.                               */
/* ------------------------------------------------------------------ */

int or_trace_grad(const int32_t *D, int32_t nc, double m2, const double *links, int32_t p,
                  const int32_t *colors, int32_t ncolors, uint64_t seed, int64_t s0,
                  int64_t ns, int32_t kind, int32_t dilute, double tol, int32_t maxit,
                  double *out, double *dT_dm2, double *dU_, double *dUbar_) {
    int64_t N = volume(D), n = N * nc;
    int32_t ndil = dilute ? nc : 1;
    int64_t nrhs = ns * ncolors * ndil;
    double norm = noise_norm(kind) / (double)ns;
    cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)(n * nrhs));
    cplx *L = (cplx *)malloc(sizeof(cplx) * (size_t)(n * nrhs));
    cplx *tj = (cplx *)malloc(sizeof(cplx) * (size_t)nrhs);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t j = 0; j < nrhs; ++j) {
        int64_t s = s0 + j / ((int64_t)ncolors * ndil);
        int32_t c = (int32_t)((j / ndil) % ncolors), a = (int32_t)(j % ndil);
        cplx *z = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *zb = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        or_probe(D, nc, colors, seed, s, c, a, dilute, kind, (double *)z);
        int32_t e[4] = {-p, 0, 0, 0};
        for (int64_t y = 0; y < N; ++y) {
            int64_t ym = shifted(y, e, D);
            for (int b = 0; b < nc; ++b) zb[y * nc + b] = z[ym * nc + b];
        }
        int i1 = or_cg(D, nc, m2, links, (const double *)z, (double *)(X + j * n), tol, maxit, NULL);
        int i2 = or_cg(D, nc, m2, links, (const double *)zb, (double *)(L + j * n), tol, maxit, NULL);
        if (i1 < 0 || i2 < 0) bad = 1;
        tj[j] = displaced_dot(D, nc, p, z, X + j * n);
        free(z);
        free(zb);
    }
    cplx T = 0.0, g = 0.0;
    for (int64_t j = 0; j < nrhs; ++j) {
        T += tj[j];
        for (int64_t i = 0; i < n; ++i) g += conj(L[j * n + i]) * X[j * n + i];
    }
    T *= norm;
    g *= -norm;
    out[0] = creal(T);
    out[1] = cimag(T);
    out[2] = NAN;
    dT_dm2[0] = creal(g);
    dT_dm2[1] = cimag(g);
    cplx *dU = (cplx *)dU_, *dUbar = (cplx *)dUbar_;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        for (int mu = 0; mu < 4; ++mu) {
            int32_t e[4] = {0, 0, 0, 0};
            e[mu] = 1;
            int64_t xp = shifted(x, e, D);
            for (int a = 0; a < nc; ++a)
                for (int b = 0; b < nc; ++b) {
                    cplx su = 0.0, sb = 0.0;
                    for (int64_t j = 0; j < nrhs; ++j) {
                        const cplx *xj = X + j * n, *lj = L + j * n;
                        su += conj(lj[x * nc + a]) * xj[xp * nc + b];
                        sb += xj[x * nc + a] * conj(lj[xp * nc + b]);
                    }
                    size_t o = ((size_t)mu * N + x) * nc * nc + a * nc + b;
                    if (dU) dU[o] = norm * su;
                    if (dUbar) dUbar[o] = norm * sb;
                }
        }
    }
    free(X);
    free(L);
    free(tj);
    return bad ? -1 : 0;
}
