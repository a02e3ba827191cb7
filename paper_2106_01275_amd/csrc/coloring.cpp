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
#include <cstdio>
#include <cstdlib>
#include <string>
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

// N(0, [p_1..p_n], k) (Sec. 3.4): the union of the displaced neighbourhoods
// N(0, p_i, k), each the two L1 balls of radius k around +p_i e0 and -p_i e0
// without the centre (Sec. 3, eqs. (5)-(6)).
std::vector<std::array<int32_t, 4>> displaced_stencil(const int32_t *ps, int32_t np, int32_t k) {
    std::vector<std::array<int32_t, 4>> out;
    for (int32_t i = 0; i < np; ++i) {
        auto one = displaced_stencil(ps[i], k);
        out.insert(out.end(), one.begin(), one.end());
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
    return build_coloring_multi(dims, &p, 1, ks, nlevels, order, colors, ncolors, order_used, err);
}

dp_status build_coloring_multi(const int32_t dims[4], const int32_t *ps, int32_t np, const int32_t *ks,
                               int32_t nlevels, int32_t order, int32_t *colors, int32_t *ncolors,
                               int32_t *order_used, std::string &err) {
    for (int d = 0; d < 4; ++d)
        if (dims[d] < 1) { err = "build_coloring: dims must be >= 1"; return DP_EINVAL; }
    if (!ps || np < 1) { err = "build_coloring: no displacement"; return DP_EINVAL; }
    for (int32_t i = 0; i < np; ++i)
        if (ps[i] < 0) { err = "build_coloring: p must be >= 0"; return DP_EINVAL; }
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
            auto st = displaced_stencil(ps, np, ks[l]);
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

// Tile policy of Sec. 3.5 (displacement along dimension 0): each side at
// least 2k+1, 2(p+k)+1 along the displacement, rounded up to a power of two,
// capped at the lattice extent.  An extent that the power of two does not
// divide takes its smallest divisor that is at least the minimum (the paper's
// lattices are powers of two).
void tile_shape(const int32_t dims[4], int32_t p, int32_t k, int32_t tile[4]) {
    for (int d = 0; d < 4; ++d) {
        const int32_t need = d == 0 ? 2 * (p + k) + 1 : 2 * k + 1;
        int32_t t = 1;
        while (t < need) t *= 2;
        if (t >= dims[d]) {
            t = dims[d];
        } else if (dims[d] % t) {
            t = need;
            while (dims[d] % t) ++t;
        }
        tile[d] = t;
    }
}

namespace {

// Colouring database for tiles: one file per (tile, p, k, order) under the
// directory named by DP_COLOR_CACHE (unset: no cache).  Format: 8 int32
// (magic, version, T0..T3, p, k), order used, colour count, then the colours.
constexpr int32_t kCacheMagic = 0x44504331, kCacheVersion = 1;

std::string cache_path(const int32_t T[4], int32_t p, int32_t k, int32_t order) {
    const char *dir = std::getenv("DP_COLOR_CACHE");
    if (!dir || !*dir) return std::string();
    char name[160];
    std::snprintf(name, sizeof name, "/tile_%dx%dx%dx%d_p%d_k%d_o%d_v%d.bin", T[0], T[1], T[2], T[3], p, k, order,
                  kCacheVersion);
    return std::string(dir) + name;
}

bool cache_load(const std::string &path, const int32_t T[4], int32_t p, int32_t k, std::vector<int32_t> &col,
                int32_t &ncol, int32_t &used) {
    if (path.empty()) return false;
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    int32_t h[10];
    bool ok = std::fread(h, sizeof(int32_t), 10, f) == 10 && h[0] == kCacheMagic && h[1] == kCacheVersion &&
              h[2] == T[0] && h[3] == T[1] && h[4] == T[2] && h[5] == T[3] && h[6] == p && h[7] == k;
    if (ok) {
        used = h[8];
        ncol = h[9];
        ok = std::fread(col.data(), sizeof(int32_t), col.size(), f) == col.size();
    }
    std::fclose(f);
    for (size_t i = 0; ok && i < col.size(); ++i) ok = col[i] >= 0 && col[i] < ncol;
    return ok;
}

void cache_store(const std::string &path, const int32_t T[4], int32_t p, int32_t k, const std::vector<int32_t> &col,
                 int32_t ncol, int32_t used) {
    if (path.empty()) return;
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    const int32_t h[10] = {kCacheMagic, kCacheVersion, T[0], T[1], T[2], T[3], p, k, used, ncol};
    bool ok = std::fwrite(h, sizeof(int32_t), 10, f) == 10 &&
              std::fwrite(col.data(), sizeof(int32_t), col.size(), f) == col.size();
    ok = std::fclose(f) == 0 && ok;
    if (ok) std::rename(tmp.c_str(), path.c_str());
    else std::remove(tmp.c_str());
}

}  // namespace

dp_status build_coloring_tiled(const int32_t dims[4], int32_t p, int32_t k, int32_t order, int32_t *colors,
                               int32_t *ncolors, int32_t *order_used, int32_t tile[4], std::string &err) {
    for (int d = 0; d < 4; ++d)
        if (dims[d] < 1) { err = "build_coloring_tiled: dims must be >= 1"; return DP_EINVAL; }
    if (p < 0 || k < 0 || !colors || !ncolors) { err = "build_coloring_tiled: bad arguments"; return DP_EINVAL; }
    int32_t T[4];
    tile_shape(dims, p, k, T);
    const int64_t NT = (int64_t)T[0] * T[1] * T[2] * T[3];
    std::vector<int32_t> tc(NT);
    int32_t ntc = 0, used = order;
    const std::string path = cache_path(T, p, k, order);
    if (!cache_load(path, T, p, k, tc, ntc, used)) {
        dp_status st = build_coloring(T, p, &k, 1, order, tc.data(), &ntc, &used, err);
        if (st != DP_OK) return st;
        cache_store(path, T, p, k, tc, ntc, used);
    }
    // repeat the tile over the lattice (T divides every extent)
    int64_t i = 0;
    for (int32_t a = 0; a < dims[0]; ++a)
        for (int32_t b = 0; b < dims[1]; ++b)
            for (int32_t c = 0; c < dims[2]; ++c) {
                const int64_t row = (((int64_t)(a % T[0]) * T[1] + b % T[1]) * T[2] + c % T[2]) * T[3];
                for (int32_t d = 0; d < dims[3]; ++d) colors[i++] = tc[row + d % T[3]];
            }
    *ncolors = ntc;
    if (order_used) *order_used = used;
    if (tile)
        for (int d = 0; d < 4; ++d) tile[d] = T[d];
    return DP_OK;
}

// Table Clearance (Sec. 4.3): for k = 0..kmax, the percentage of the sites at
// torus L1 distance exactly k from x + p e0 or from x - p e0 (x itself
// excluded) that have the colour of x, averaged over all sites x.  By
// translation invariance the set of offsets is the same for every x.
dp_status clearance(const int32_t dims[4], const int32_t *colors, int32_t p, int32_t kmax, double *pct,
                    std::string &err) {
    for (int d = 0; d < 4; ++d)
        if (dims[d] < 1) { err = "clearance: dims must be >= 1"; return DP_EINVAL; }
    if (!colors || !pct || p < 0 || kmax < 0) { err = "clearance: bad arguments"; return DP_EINVAL; }
    auto tdist = [&](int32_t v, int d) {  // torus |v| along dimension d
        int32_t w = ((v % dims[d]) + dims[d]) % dims[d];
        return std::min(w, dims[d] - w);
    };
    // distinct offsets r (one per residue) with their distances to +p e0 and -p e0
    struct Off { int32_t r[4]; int32_t kp, km; };
    std::vector<Off> offs;
    int32_t lo[4], hi[4];
    for (int d = 0; d < 4; ++d) {
        const int32_t reach = (d == 0 ? p : 0) + kmax;
        lo[d] = -reach;
        hi[d] = reach;
        if (hi[d] - lo[d] + 1 > dims[d]) { lo[d] = 0; hi[d] = dims[d] - 1; }  // every residue once
    }
    for (int32_t a = lo[0]; a <= hi[0]; ++a)
        for (int32_t b = lo[1]; b <= hi[1]; ++b)
            for (int32_t c = lo[2]; c <= hi[2]; ++c)
                for (int32_t d = lo[3]; d <= hi[3]; ++d) {
                    if (tdist(a, 0) == 0 && tdist(b, 1) == 0 && tdist(c, 2) == 0 && tdist(d, 3) == 0) continue;
                    const int32_t rest = tdist(b, 1) + tdist(c, 2) + tdist(d, 3);
                    Off o{{a, b, c, d}, tdist(a - p, 0) + rest, tdist(a + p, 0) + rest};
                    if (std::min(o.kp, o.km) <= kmax) offs.push_back(o);
                }
    std::vector<double> same(kmax + 1, 0.0), total(kmax + 1, 0.0);
    const int64_t N = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    std::vector<int64_t> shift(offs.size());
    for (int32_t x0 = 0; x0 < dims[0]; ++x0)
        for (int32_t x1 = 0; x1 < dims[1]; ++x1)
            for (int32_t x2 = 0; x2 < dims[2]; ++x2)
                for (int32_t x3 = 0; x3 < dims[3]; ++x3) {
                    const int64_t x = (((int64_t)x0 * dims[1] + x1) * dims[2] + x2) * dims[3] + x3;
                    for (const Off &o : offs) {
                        const int32_t y0 = ((x0 + o.r[0]) % dims[0] + dims[0]) % dims[0];
                        const int32_t y1 = ((x1 + o.r[1]) % dims[1] + dims[1]) % dims[1];
                        const int32_t y2 = ((x2 + o.r[2]) % dims[2] + dims[2]) % dims[2];
                        const int32_t y3 = ((x3 + o.r[3]) % dims[3] + dims[3]) % dims[3];
                        const int64_t y = (((int64_t)y0 * dims[1] + y1) * dims[2] + y2) * dims[3] + y3;
                        const double s = colors[y] == colors[x] ? 1.0 : 0.0;
                        if (o.kp <= kmax) { same[o.kp] += s; total[o.kp] += 1.0; }
                        if (o.km <= kmax && o.km != o.kp) { same[o.km] += s; total[o.km] += 1.0; }
                    }
                }
    (void)N;
    for (int32_t k = 0; k <= kmax; ++k) pct[k] = total[k] > 0 ? 100.0 * same[k] / total[k] : 0.0;
    return DP_OK;
}

}  // namespace dp
