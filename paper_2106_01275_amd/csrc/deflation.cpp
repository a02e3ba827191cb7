// Deflation of the trace estimator (Sec. Deflation): the low eigenvectors of
// the Hermitian operator A from a Chebyshev-filtered subspace iteration with
// Rayleigh-Ritz (FP64 on the device; the small dense eigenproblems on the
// host), and the projection of the probes, b = z - A V Theta^{-1} V^H z.
//
// One outer iteration on the block V of W vectors (internal layout, W lanes):
//   Y  = p(A) V, p the degree-m Chebyshev polynomial of the first kind
//        mapped to damp [a, b] and scaled to 1 at the lower spectral bound
//        (three-term recurrence, one stencil and one axpby per degree);
//   G  = Y^H Y,  M = Y^H (A Y)  (Gram kernels, FP64);
//   host: G = Q D Q^H, S = Q D^{-1/2}, S^H M S = X Theta X^H (Jacobi),
//         C = S X (Ritz coefficients, ascending Theta);
//   V  = Y C,  A V = (A Y) C,  a = a little above max Theta.
// The Ritz residuals |A v_i - theta_i v_i| of the kept vectors decide
// convergence.  The filter polynomial and the Rayleigh-Ritz step follow the
// standard Chebyshev-filtered subspace iteration; the interval bound b comes
// from the links (each row of the hop part has norm at most the sum over
// its eight hops of |U|_F).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "context.h"

namespace dp {

namespace {

using cplx = std::complex<double>;

// Eigen-decomposition of the Hermitian n x n matrix A (row-major, destroyed)
// by cyclic Jacobi rotations: on return w holds the eigenvalues ascending and
// the columns of Vec (row-major) the eigenvectors.
void herm_eig(int n, std::vector<cplx> &A, std::vector<double> &w, std::vector<cplx> &Vec) {
    std::vector<cplx> VT((size_t)n * n, cplx(0, 0));  // eigenvectors as rows
    for (int i = 0; i < n; ++i) VT[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> cplx & { return A[(size_t)i * n + j]; };
    for (int i = 0; i < n; ++i) a(i, i) = a(i, i).real();
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, diag = 0;
        for (int i = 0; i < n; ++i) {
            diag += std::norm(a(i, i));
            for (int j = i + 1; j < n; ++j) off += std::norm(a(i, j));
        }
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double g = std::abs(a(p, q));
                if (g == 0.0) continue;
                const cplx e = a(p, q) / g;  // phase of the off-diagonal entry
                const double app = a(p, p).real(), aqq = a(q, q).real();
                const double tau = (aqq - app) / (2.0 * g);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // U = D R on the (p, q) plane: U_pp = c, U_pq = s, U_qp = -s conj(e), U_qq = c conj(e)
                const cplx upp = c, upq = s, uqp = -s * std::conj(e), uqq = c * std::conj(e);
                // A <- U^H A U: outside the (p, q) block only columns p, q
                // change (rows p, q are their conjugates); inside, the
                // rotation leaves app - t g, aqq + t g and a zero
                for (int k = 0; k < n; ++k) {
                    if (k == p || k == q) continue;
                    const cplx akp = a(k, p), akq = a(k, q);
                    const cplx np = akp * upp + akq * uqp, nq = akp * upq + akq * uqq;
                    a(k, p) = np;
                    a(k, q) = nq;
                    a(p, k) = std::conj(np);
                    a(q, k) = std::conj(nq);
                }
                a(p, p) = app - t * g;
                a(q, q) = aqq + t * g;
                a(p, q) = a(q, p) = 0.0;
                cplx *vp = &VT[(size_t)p * n], *vq = &VT[(size_t)q * n];
                for (int k = 0; k < n; ++k) {  // eigenvectors <- eigenvectors U
                    const cplx vkp = vp[k], vkq = vq[k];
                    vp[k] = vkp * upp + vkq * uqp;
                    vq[k] = vkp * upq + vkq * uqq;
                }
            }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x).real() < a(y, y).real(); });
    Vec.assign((size_t)n * n, cplx(0, 0));
    w.resize(n);
    for (int c = 0; c < n; ++c) {
        w[c] = a(idx[c], idx[c]).real();
        for (int r = 0; r < n; ++r) Vec[(size_t)r * n + c] = VT[(size_t)idx[c] * n + r];
    }
}

// Device buffers of one eigensolve, returned to the context's pool.
struct Bufs {
    dp_ctx *ctx;
    hipStream_t s;
    std::vector<std::pair<void *, size_t>> held;
    Bufs(dp_ctx *c, hipStream_t st) : ctx(c), s(st) {}
    ~Bufs() {
        (void)hipStreamSynchronize(s);
        for (auto &b : held) ctx->pool_put(b.first, b.second);
    }
    dp_status get(size_t bytes, double **out) {
        void *p = nullptr;
        size_t got = 0;
        DP_TRY(ctx->pool_get(bytes, &p, &got));
        held.emplace_back(p, got);
        *out = (double *)p;
        return DP_OK;
    }
};

Launch block_launch(const Lat &lat, int nc, int W, hipStream_t s) {
    Launch L;
    int logW = 0;
    while ((1 << logW) < W) ++logW;
    L.lat = lat;
    L.nc = nc;
    L.W = W;
    L.logW = logW;
    L.ntiles = (lat.N + (kBlock >> logW) - 1) / (kBlock >> logW);
    L.nblk = grid_blocks(L.ntiles);
    L.stream = s;
    return L;
}

size_t gram_part_bytes(long long n, int WX, int WY) {
    const size_t tiles = (size_t)((WX + 63) / 64) * ((WY + 63) / 64);
    return (size_t)gram_row_blocks(n) * tiles * 64 * 64 * 16;
}

}  // namespace

dp_status deflation_build(dp_ctx *ctx, const dp_operator &opd, int nvec, const dp_eig_opts &eo, dp_deflation &D,
                          hipStream_t s) {
    OpPrep op;
    DP_TRY(prepare_operator(ctx, opd, kF64, op, s));
    int W = 1;
    while (W < nvec + std::max(4, nvec / 4)) W *= 2;
    if (nvec < 1 || W > 128) {
        ctx->err = "deflation: nvec must be in [1, 103]";
        return DP_EINVAL;
    }
    if ((long long)W > (long long)op.lat.N * op.nc) {
        ctx->err = "deflation: the subspace is larger than the operator";
        return DP_EINVAL;
    }
    const int degree = eo.degree > 0 ? eo.degree : 16;
    const int max_outer = eo.max_outer > 0 ? eo.max_outer : 60;
    const double tol = eo.tol > 0 ? eo.tol : 1e-10;
    D.nvec = nvec;
    D.W = W;
    D.lat = op.lat;
    D.nc = op.nc;
    D.m2 = op.m2;
    D.links = op.links;
    const long long n = (long long)op.lat.N * op.nc;  // rows
    const long long ne = n * W;                       // complex entries of a block
    const size_t vb = (size_t)ne * 16;
    const Launch L = block_launch(op.lat, op.nc, W, s);
    DP_HIP(hipMalloc(&D.V, vb));
    DP_HIP(hipMalloc(&D.Z, vb));
    DP_HIP(hipMalloc(&D.scratch, (size_t)(4 * W + (size_t)L.nblk * W * 2) * sizeof(double)));
    Bufs B(ctx, s);
    double *Y, *Q, *AV, *part, *H, *th_dev;
    DP_TRY(B.get(vb, &Y));
    DP_TRY(B.get(vb, &Q));
    DP_TRY(B.get(vb, &AV));
    DP_TRY(B.get(gram_part_bytes(n, W, W), &part));
    DP_TRY(B.get((size_t)W * W * 16, &H));
    DP_TRY(B.get((size_t)W * sizeof(double), &th_dev));
    CgState cs{};
    cs.tj = D.scratch;
    cs.true_rr = D.scratch + 2 * W;
    cs.alpha = D.scratch + 3 * W;
    Red rd{};
    rd.part1 = D.scratch + 4 * W;
    rd.part2 = nullptr;  // (no CG here)
    rd.nblk = L.nblk;

    // spectral bounds: A = (m2 + 8) - H with |H| <= max over sites of the
    // sum of the hop norms
    double hb = 8.0;
    if (op.links) {
        double *bnd = nullptr;
        DP_TRY(B.get((size_t)op.lat.N * sizeof(double), &bnd));
        launch_hop_bound(op.lat, op.nc, (const double *)op.U8, bnd, s);
        std::vector<double> hbnd(op.lat.N);
        DP_HIP(hipMemcpyAsync(hbnd.data(), bnd, hbnd.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        DP_HIP(hipStreamSynchronize(s));
        hb = *std::max_element(hbnd.begin(), hbnd.end());
    }
    const double lo_bound = op.m2 + 8.0 - hb, hi_bound = op.m2 + 8.0 + hb;

    StencilArgs sa;
    sa.links = op.links;
    sa.U = op.U8;
    sa.nbr = op.nbr;
    sa.cg = 0;
    auto apply_shift = [&](const double *in, double *out, double shift) {
        sa.diag = op.m2 + 8.0 - shift;
        sa.pin = in;
        sa.q = out;
        launch_stencil(L, kF64, sa);
    };
    std::vector<cplx> G((size_t)W * W), M((size_t)W * W);
    std::vector<double> theta(W), resid(W);
    // Rayleigh-Ritz on the block X with AX = A X: D.V = X C, AV = AX C
    auto rayleigh_ritz = [&](const double *X, const double *AX) -> dp_status {
        launch_gram(n, W, W, X, X, part, 1.0, H, s);
        DP_HIP(hipMemcpyAsync(G.data(), H, (size_t)W * W * 16, hipMemcpyDeviceToHost, s));
        launch_gram(n, W, W, X, AX, part, 1.0, H, s);
        DP_HIP(hipMemcpyAsync(M.data(), H, (size_t)W * W * 16, hipMemcpyDeviceToHost, s));
        DP_HIP(hipStreamSynchronize(s));
        std::vector<double> d;
        std::vector<cplx> Qg;
        herm_eig(W, G, d, Qg);
        const double dmax = std::max(d[W - 1], 1e-300);
        std::vector<cplx> S((size_t)W * W);  // S = Q D^{-1/2}
        for (int c = 0; c < W; ++c) {
            const double f = 1.0 / std::sqrt(std::max(d[c], 1e-15 * dmax));
            for (int r = 0; r < W; ++r) S[(size_t)r * W + c] = Qg[(size_t)r * W + c] * f;
        }
        std::vector<cplx> T((size_t)W * W, cplx(0, 0)), Bm((size_t)W * W, cplx(0, 0));
        for (int i = 0; i < W; ++i)  // T = M S
            for (int k = 0; k < W; ++k) {
                const cplx m = 0.5 * (M[(size_t)i * W + k] + std::conj(M[(size_t)k * W + i]));
                for (int j = 0; j < W; ++j) T[(size_t)i * W + j] += m * S[(size_t)k * W + j];
            }
        for (int i = 0; i < W; ++i)  // Bm = S^H T
            for (int k = 0; k < W; ++k) {
                const cplx sk = std::conj(S[(size_t)k * W + i]);
                for (int j = 0; j < W; ++j) Bm[(size_t)i * W + j] += sk * T[(size_t)k * W + j];
            }
        std::vector<cplx> Xr;
        herm_eig(W, Bm, theta, Xr);
        std::vector<cplx> C((size_t)W * W, cplx(0, 0));  // C = S Xr
        for (int i = 0; i < W; ++i)
            for (int k = 0; k < W; ++k) {
                const cplx sv = S[(size_t)i * W + k];
                for (int j = 0; j < W; ++j) C[(size_t)i * W + j] += sv * Xr[(size_t)k * W + j];
            }
        DP_HIP(hipMemcpyAsync(H, C.data(), (size_t)W * W * 16, hipMemcpyHostToDevice, s));
        launch_rot(n, W, W, X, H, D.V, 0, s);
        launch_rot(n, W, W, AX, H, AV, 0, s);
        // Ritz residuals
        DP_HIP(hipMemcpyAsync(th_dev, theta.data(), W * sizeof(double), hipMemcpyHostToDevice, s));
        launch_resid_norm(L, AV, D.V, th_dev, rd, cs);
        DP_HIP(hipMemcpyAsync(resid.data(), cs.true_rr, W * sizeof(double), hipMemcpyDeviceToHost, s));
        DP_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < W; ++i)
            resid[i] = std::sqrt(std::max(resid[i], 0.0)) / std::max(std::fabs(theta[i]), 1e-300);
        return DP_OK;
    };

    launch_rand_fill(ne, eo.seed, Y, s);
    apply_shift(Y, Q, 0.0);
    DP_HIP(hipGetLastError());
    DP_TRY(rayleigh_ritz(Y, Q));
    bool conv = false;
    int outer = 0;
    while (outer < max_outer) {
        double worst = 0;
        for (int i = 0; i < nvec; ++i) worst = std::max(worst, resid[i]);
        if (worst <= tol) {
            conv = true;
            break;
        }
        ++outer;
        // Y = p(A) V damping [a, hi_bound], scaled to 1 at lo_bound.  a sits
        // a little above the largest Ritz value: at a itself the filter is 1,
        // no gain over the damped interval, and a kept vector in a
        // degenerate cluster that reaches the top of the subspace would stall
        const double b = hi_bound;
        const double a = std::min(theta[W - 1] + 0.1 * (theta[W - 1] - theta[0]), 0.5 * (theta[W - 1] + b));
        const double e = 0.5 * (b - a), c = 0.5 * (b + a);
        if (!(e > 0)) break;
        double sigma = e / (lo_bound - c);
        const double tau = 2.0 / sigma;
        double *X0 = D.V, *X1 = Y;
        apply_shift(X0, Q, c);  // X1 = (sigma / e) (A - c) X0
        launch_axpby(ne, sigma / e, Q, 0.0, X0, X1, s);
        for (int k = 2; k <= degree; ++k) {
            const double sigma2 = 1.0 / (tau - sigma);
            apply_shift(X1, Q, c);  // X0 <- (2 sigma2 / e) (A - c) X1 - sigma sigma2 X0
            launch_axpby(ne, 2.0 * sigma2 / e, Q, -sigma * sigma2, X0, X0, s);
            std::swap(X0, X1);
            sigma = sigma2;
        }
        DP_HIP(hipGetLastError());
        // X1 holds the filtered block; move it out of D.V before the rotation
        double *F = X1;
        if (F == D.V) {
            DP_HIP(hipMemcpyAsync(Y, D.V, vb, hipMemcpyDeviceToDevice, s));
            F = Y;
        }
        apply_shift(F, Q, 0.0);
        DP_TRY(rayleigh_ritz(F, Q));
    }
    D.outer = outer;
    D.theta.assign(theta.begin(), theta.begin() + nvec);
    D.resid.assign(resid.begin(), resid.begin() + nvec);
    // Z = A V Theta^{-1} in the kept lanes
    std::vector<double> sc(W, 0.0);
    for (int i = 0; i < nvec; ++i) sc[i] = 1.0 / theta[i];
    DP_HIP(hipMemcpyAsync(th_dev, sc.data(), W * sizeof(double), hipMemcpyHostToDevice, s));
    launch_scale_lanes(ne, W, th_dev, AV, D.Z, s);
    DP_HIP(hipGetLastError());
    DP_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nvec; ++i)
        if (!(theta[i] > 0) || !std::isfinite(theta[i])) {
            ctx->err = "deflation: non-positive Ritz value (is A positive definite?)";
            return DP_EBREAKDOWN;
        }
    return conv ? DP_OK : DP_ENOCONV;
}

dp_status deflate_rhs(dp_ctx *ctx, const dp_deflation &d, const Launch &L, double *b64) {
    const long long n = (long long)d.lat.N * d.nc;
    void *part = nullptr, *H = nullptr;
    size_t gp = 0, gh = 0;
    DP_TRY(ctx->pool_get(gram_part_bytes(n, d.W, L.W), &part, &gp));
    DP_TRY(ctx->pool_get((size_t)d.W * L.W * 16, &H, &gh));
    // H = -V^H b, then b += Z H
    launch_gram(n, d.W, L.W, d.V, b64, (double *)part, -1.0, (double *)H, L.stream);
    launch_rot(n, d.W, L.W, d.Z, (const double *)H, b64, 1, L.stream);
    const hipError_t e = hipGetLastError();
    // back to the pool at once: whoever takes them next queues its work on
    // the library's stream, after these kernels
    ctx->pool_put(part, gp);
    ctx->pool_put(H, gh);
    if (e != hipSuccess) {
        ctx->err = std::string("deflate_rhs: ") + hipGetErrorString(e);
        return DP_EHIP;
    }
    return DP_OK;
}

dp_status deflation_trace_part(dp_ctx *ctx, const dp_deflation &d, int p, hipStream_t s, double out[2]) {
    const Launch L = block_launch(d.lat, d.nc, d.W, s);
    CgState cs{};
    cs.tj = d.scratch;
    cs.true_rr = d.scratch + 2 * d.W;
    cs.alpha = d.scratch + 3 * d.W;
    Red rd{};
    rd.part1 = d.scratch + 4 * d.W;
    rd.part2 = nullptr;  // (no CG here)
    rd.nblk = L.nblk;
    launch_dot_shift(L, d.V, d.V, p, rd, cs);
    std::vector<double> tj(2 * d.W);
    DP_HIP(hipMemcpyAsync(tj.data(), cs.tj, tj.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DP_HIP(hipStreamSynchronize(s));
    out[0] = out[1] = 0.0;
    for (int i = 0; i < d.nvec; ++i) {
        out[0] += tj[2 * i] / d.theta[i];
        out[1] += tj[2 * i + 1] / d.theta[i];
    }
    return DP_OK;
}

dp_status deflation_vectors(dp_ctx *ctx, const dp_deflation &d, double *out, hipStream_t s) {
    const Launch L = block_launch(d.lat, d.nc, d.W, s);
    launch_to_abi(L, d.V, out, 0, d.nvec);
    DP_HIP(hipGetLastError());
    return DP_OK;
}

}  // namespace dp
