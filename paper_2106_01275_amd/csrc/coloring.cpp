// Host-side greedy displaced distance-k colouring (Sec. 3.1 of
// arXiv:2106.01275, DisColoring / CreateStencil; nested levels per Sec. 2.3).
//
// Design: the stencil is the sorted union of the two L1 balls around +p e0
// and -p e0 (Sec. 3.1 removes the duplicates of the overlapping balls by
// sorting).  Offsets are grouped into runs that are contiguous along the
// fastest dimension, so the colours of a run of neighbours are one
// contiguous slice of the colour array for sites away from the x3 boundary.
// Colours in use are marked with a per-site stamp instead of clearing a bit
// array for every site.
#include <algorithm>
#include <array>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "dp_internal.h"

namespace dp {

std::vector<std::array<int32_t, 4>> displaced_stencil(int32_t p, int32_t k) {
    std::vector<std::array<int32_t, 4>> out;
    for (int32_t c0 : {p, -p}) {
        // L1 ball of radius k around (c0, 0, 0, 0)
        for (int32_t a = -k; a <= k; ++a)
            for (int32_t b = -(k - std::abs(a)); b <= k - std::abs(a); ++b)
                for (int32_t c = -(k - std::abs(a) - std::abs(b)); c <= k - std::abs(a) - std::abs(b); ++c) {
                    int32_t rest = k - std::abs(a) - std::abs(b) - std::abs(c);
                    for (int32_t d = -rest; d <= rest; ++d) {
                        std::array<int32_t, 4> o{c0 + a, b, c, d};
                        if (o[0] == 0 && o[1] == 0 && o[2] == 0 && o[3] == 0) continue;
                        out.push_back(o);
                    }
                }
        if (p == 0) break;
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
}

namespace {

struct Run {              // offsets (o0, o1, o2, lo..hi)
    int32_t o0, o1, o2, lo, hi;
};

struct Geometry {
    int32_t D[4];
    int64_t N;
    int32_t R[4];                     // largest |offset| per dimension
    std::vector<int64_t> wrap[3];     // wrap[d][v + R[d]] = ((v mod D) * stride_d)
    std::vector<int32_t> wrap3;       // wrap3[v + R[3]] = v mod D3
};

Geometry make_geometry(const int32_t *dims, const std::vector<Run> &runs) {
    Geometry g;
    for (int d = 0; d < 4; ++d) { g.D[d] = dims[d]; g.R[d] = 0; }
    g.N = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    for (const Run &r : runs) {
        g.R[0] = std::max(g.R[0], std::abs(r.o0));
        g.R[1] = std::max(g.R[1], std::abs(r.o1));
        g.R[2] = std::max(g.R[2], std::abs(r.o2));
        g.R[3] = std::max({g.R[3], std::abs(r.lo), std::abs(r.hi)});
    }
    int64_t stride[3] = {(int64_t)dims[1] * dims[2] * dims[3], (int64_t)dims[2] * dims[3], dims[3]};
    for (int d = 0; d < 3; ++d) {
        g.wrap[d].resize(2 * g.R[d] + dims[d]);
        for (int32_t v = -g.R[d]; v < dims[d] + g.R[d]; ++v) {
            int32_t w = ((v % dims[d]) + dims[d]) % dims[d];
            g.wrap[d][v + g.R[d]] = w * stride[d];
        }
    }
    g.wrap3.resize(2 * g.R[3] + dims[3]);
    for (int32_t v = -g.R[3]; v < dims[3] + g.R[3]; ++v)
        g.wrap3[v + g.R[3]] = ((v % dims[3]) + dims[3]) % dims[3];
    return g;
}

std::vector<Run> make_runs(const std::vector<std::array<int32_t, 4>> &st) {
    std::vector<Run> runs;  // st is sorted: equal (o0,o1,o2) are adjacent, o3 increasing
    for (size_t i = 0; i < st.size();) {
        size_t j = i;
        while (j + 1 < st.size() && st[j + 1][0] == st[i][0] && st[j + 1][1] == st[i][1] &&
               st[j + 1][2] == st[i][2] && st[j + 1][3] == st[j][3] + 1)
            ++j;
        runs.push_back({st[i][0], st[i][1], st[i][2], st[i][3], st[j][3]});
        i = j + 1;
    }
    return runs;
}

std::vector<int64_t> visit_order(const int32_t *D, int32_t order) {
    int64_t N = (int64_t)D[0] * D[1] * D[2] * D[3];
    std::vector<int64_t> ord;
    ord.reserve(N);
    if (order == DP_ORDER_NATURAL) {
        for (int64_t i = 0; i < N; ++i) ord.push_back(i);
        return ord;
    }
    for (int parity = 0; parity < 2; ++parity)
        for (int32_t a = 0; a < D[0]; ++a)
            for (int32_t b = 0; b < D[1]; ++b)
                for (int32_t c = 0; c < D[2]; ++c)
                    for (int32_t d = 0; d < D[3]; ++d)
                        if (((a + b + c + d) & 1) == parity)
                            ord.push_back((((int64_t)a * D[1] + b) * D[2] + c) * D[3] + d);
    return ord;
}

// First-fit colouring of the sites in `ord`; with `parent`, only neighbours
// with the same parent colour constrain a site.  Returns the colour count.
int32_t first_fit(const Geometry &g, const std::vector<Run> &runs, const std::vector<int64_t> &ord,
                  const int32_t *parent, int32_t *col, size_t max_colors) {
    std::fill(col, col + g.N, -1);
    std::vector<int64_t> stamp(max_colors + 2, -1);
    const int32_t D3 = g.D[3];
    int32_t ncol = 0;
    for (int64_t t = 0; t < (int64_t)ord.size(); ++t) {
        const int64_t x = ord[t];
        const int32_t x3 = (int32_t)(x % D3);
        int64_t rem = x / D3;
        const int32_t x2 = (int32_t)(rem % g.D[2]);
        rem /= g.D[2];
        const int32_t x1 = (int32_t)(rem % g.D[1]);
        const int32_t x0 = (int32_t)(rem / g.D[1]);
        const int32_t px = parent ? parent[x] : 0;
        for (const Run &r : runs) {
            const int64_t base = g.wrap[0][x0 + r.o0 + g.R[0]] + g.wrap[1][x1 + r.o1 + g.R[1]] +
                                 g.wrap[2][x2 + r.o2 + g.R[2]];
            if (x3 + r.lo >= 0 && x3 + r.hi < D3) {
                const int32_t *c = col + base + x3 + r.lo;
                const int32_t *pp = parent ? parent + base + x3 + r.lo : nullptr;
                for (int32_t i = 0; i <= r.hi - r.lo; ++i) {
                    int32_t cy = c[i];
                    if (cy >= 0 && (!pp || pp[i] == px) && base + x3 + r.lo + i != x) stamp[cy] = t;
                }
            } else {
                for (int32_t o3 = r.lo; o3 <= r.hi; ++o3) {
                    int64_t y = base + g.wrap3[x3 + o3 + g.R[3]];
                    int32_t cy = col[y];
                    if (cy >= 0 && y != x && (!parent || parent[y] == px)) stamp[cy] = t;
                }
            }
        }
        int32_t c = 0;
        while (stamp[c] == t) ++c;
        col[x] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

}  // namespace

dp_status build_coloring(const int32_t dims[4], int32_t p, const int32_t *ks, int32_t nlevels,
                         int32_t order, int32_t *colors, int32_t *ncolors, int32_t *order_used,
                         std::string &err) {
    for (int d = 0; d < 4; ++d)
        if (dims[d] < 1) { err = "build_coloring: dims must be >= 1"; return DP_EINVAL; }
    if (p < 0) { err = "build_coloring: p must be >= 0"; return DP_EINVAL; }
    if (nlevels < 1 || !ks || !colors || !ncolors) { err = "build_coloring: bad arguments"; return DP_EINVAL; }
    for (int l = 0; l < nlevels; ++l) {
        if (ks[l] < 0 || (l > 0 && ks[l] <= ks[l - 1])) {
            err = "build_coloring: ks must be >= 0 and strictly increasing";
            return DP_EINVAL;
        }
    }
    if (order != DP_ORDER_NATURAL && order != DP_ORDER_REDBLACK && order != DP_ORDER_BEST) {
        err = "build_coloring: unknown order";
        return DP_EINVAL;
    }
    const int64_t N = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    auto run_order = [&](int32_t ord_kind, int32_t *out, int32_t *nout) {
        std::vector<int64_t> ord = visit_order(dims, ord_kind);
        for (int l = 0; l < nlevels; ++l) {
            auto st = displaced_stencil(p, ks[l]);
            auto runs = make_runs(st);
            Geometry g = make_geometry(dims, runs);
            int32_t *cur = out + (size_t)l * N;
            if (l == 0) {
                nout[0] = first_fit(g, runs, ord, nullptr, cur, st.size());
                continue;
            }
            const int32_t *par = out + (size_t)(l - 1) * N;
            std::vector<int32_t> sub(N);
            first_fit(g, runs, ord, par, sub.data(), st.size());
            const int32_t np = nout[l - 1];
            std::vector<int32_t> cnt(np, 0), off(np + 1, 0);
            for (int64_t i = 0; i < N; ++i) cnt[par[i]] = std::max(cnt[par[i]], sub[i] + 1);
            for (int32_t c = 0; c < np; ++c) off[c + 1] = off[c] + cnt[c];
            for (int64_t i = 0; i < N; ++i) cur[i] = off[par[i]] + sub[i];
            nout[l] = off[np];
        }
    };
    if (order != DP_ORDER_BEST) {
        run_order(order, colors, ncolors);
        if (order_used) *order_used = order;
        return DP_OK;
    }
    run_order(DP_ORDER_NATURAL, colors, ncolors);
    std::vector<int32_t> alt((size_t)nlevels * N), nalt(nlevels);
    run_order(DP_ORDER_REDBLACK, alt.data(), nalt.data());
    if (nalt[nlevels - 1] < ncolors[nlevels - 1]) {
        std::copy(alt.begin(), alt.end(), colors);
        std::copy(nalt.begin(), nalt.end(), ncolors);
        if (order_used) *order_used = DP_ORDER_REDBLACK;
    } else if (order_used) {
        *order_used = DP_ORDER_NATURAL;
    }
    return DP_OK;
}

}  // namespace dp
