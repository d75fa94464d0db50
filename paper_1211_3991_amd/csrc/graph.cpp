// Host side of the graph path: Levy graph sampling (Sec. 2, Eq. Levyi),
// smallest-last-ordering colouring (App. B, "Graph coloring") and the
// colour-sorted CSR that the device kernels stream.  Runs once per sample
// before the dynamics, as in the paper.
#include <algorithm>
#include <cmath>
#include <new>
#include <numeric>
#include <set>
#include <unordered_set>
#include <utility>

#include "xy_internal.hpp"

namespace {
thread_local std::string g_last_error;
}

namespace xy {

xy_status set_error(xy_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

// Colouring and CSR.  Smallest-last ordering: repeatedly remove a site of
// minimum remaining degree (ties: smallest lattice index); colour sites in
// reverse removal order with the smallest colour unused by their already
// coloured neighbours.  Sites are then renumbered colour-major (by colour,
// then lattice index) so that each colour class is one contiguous range and
// every neighbour list, sorted by colour-major index, lists lower colours
// first.
xy_status finish_graph(xy_graph &g)
{
    const int n = g.n, m = g.m;
    std::vector<int32_t> deg(n, 0), start(n + 1, 0), adj(2 * (size_t)m);
    for (int e = 0; e < m; ++e) { deg[g.edges[2 * e]]++; deg[g.edges[2 * e + 1]]++; }
    for (int v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
    {
        std::vector<int32_t> pos(start.begin(), start.end() - 1);
        for (int e = 0; e < m; ++e) {
            const int a = g.edges[2 * e], b = g.edges[2 * e + 1];
            adj[pos[a]++] = b;
            adj[pos[b]++] = a;
        }
    }
    g.max_deg = n ? *std::max_element(deg.begin(), deg.end()) : 0;

    // removal order: an ordered set of (remaining degree, site)
    std::vector<int32_t> order;
    order.reserve(n);
    {
        std::vector<int32_t> rem(deg);
        std::vector<char> gone(n, 0);
        std::set<std::pair<int32_t, int32_t>> pool;
        for (int v = 0; v < n; ++v) pool.emplace(rem[v], v);
        while (!pool.empty()) {
            const int v = pool.begin()->second;
            pool.erase(pool.begin());
            gone[v] = 1;
            order.push_back(v);
            for (int a = start[v]; a < start[v + 1]; ++a) {
                const int w = adj[a];
                if (gone[w]) continue;
                pool.erase({rem[w], w});
                rem[w]--;
                pool.emplace(rem[w], w);
            }
        }
    }
    g.colour.assign(n, -1);
    int Q = 0;
    {
        std::vector<int32_t> seen(g.max_deg + 2, -1);
        for (int idx = n - 1; idx >= 0; --idx) {
            const int v = order[idx];
            for (int a = start[v]; a < start[v + 1]; ++a) {
                const int c = g.colour[adj[a]];
                if (c >= 0) seen[c] = v;
            }
            int c = 0;
            while (seen[c] == v) ++c;
            g.colour[v] = c;
            Q = std::max(Q, c + 1);
        }
    }
    if (n == 0) Q = 0;
    if (Q > kMaxColours)
        return set_error(XY_EUNSUP, "graph needs more than 31 colours");
    if (g.max_deg > 255)
        return set_error(XY_EUNSUP, "graph has a site of degree above 255");
    g.Q = Q;

    // colour-major renumbering (counting sort, stable in lattice index)
    g.colour_off.assign(Q + 1, 0);
    for (int v = 0; v < n; ++v) g.colour_off[g.colour[v] + 1]++;
    for (int c = 0; c < Q; ++c) g.colour_off[c + 1] += g.colour_off[c];
    g.perm.assign(n, 0);
    g.inv.assign(n, 0);
    {
        std::vector<int32_t> next(g.colour_off.begin(), g.colour_off.end() - 1);
        for (int v = 0; v < n; ++v) {
            const int k = next[g.colour[v]]++;
            g.perm[k] = v;
            g.inv[v] = k;
        }
    }
    g.row_ptr.assign(n + 1, 0);
    g.col.assign(2 * (size_t)m, 0);
    for (int k = 0; k < n; ++k) g.row_ptr[k + 1] = g.row_ptr[k] + deg[g.perm[k]];
    for (int k = 0; k < n; ++k) {
        const int v = g.perm[k];
        int32_t *row = g.col.data() + g.row_ptr[k];
        for (int a = start[v]; a < start[v + 1]; ++a) *row++ = g.inv[adj[a]];
        std::sort(g.col.data() + g.row_ptr[k], g.col.data() + g.row_ptr[k + 1]);
    }
    return XY_OK;
}

Sell build_sell(const xy_graph &g, int window)
{
    Sell S;
    const int n = g.n, Q = g.Q;
    S.order.resize(n);
    S.deg.resize(n);
    S.chunk_off.assign(Q + 1, 0);
    std::vector<int32_t> inv(n);
    // degree sort inside windows of `window` consecutive sites of a class: the
    // chunks get nearly uniform degree, and a small window still covers a
    // compact band of the lattice (neighbour gathers from global memory keep
    // their locality)
    if (window < 64) window = 64;
    for (int c = 0; c < Q; ++c) {
        const int c0 = g.colour_off[c], c1 = g.colour_off[c + 1];
        std::iota(S.order.begin() + c0, S.order.begin() + c1, c0);
        for (int w0 = c0; w0 < c1; w0 += window)
            std::stable_sort(S.order.begin() + w0, S.order.begin() + std::min(c1, w0 + window), [&](int a, int b) {
                return g.row_ptr[a + 1] - g.row_ptr[a] > g.row_ptr[b + 1] - g.row_ptr[b];
            });
        S.chunk_off[c + 1] = S.chunk_off[c] + (c1 - c0 + 63) / 64;
    }
    for (int k = 0; k < n; ++k) {
        inv[S.order[k]] = k;
        S.deg[k] = (uint8_t)(g.row_ptr[S.order[k] + 1] - g.row_ptr[S.order[k]]);
    }
    const int n_chunks = S.chunk_off[Q];
    S.chunk_ptr.assign(n_chunks + 1, 0);
    S.chunk_w.assign(n_chunks, 0);
    for (int c = 0; c < Q; ++c)
        for (int ch = S.chunk_off[c]; ch < S.chunk_off[c + 1]; ++ch) {
            const int first = g.colour_off[c] + (ch - S.chunk_off[c]) * 64;
            const int last = std::min(first + 64, g.colour_off[c + 1]);
            int w = 0, wmin = 255;
            for (int k = first; k < last; ++k) {
                w = std::max(w, (int)S.deg[k]);
                wmin = std::min(wmin, (int)S.deg[k]);
            }
            // at least kSellRows rows per chunk, so a kernel may read its
            // first kSellRows rows without a bound
            S.chunk_ptr[ch + 1] = S.chunk_ptr[ch] + 64 * std::max(w, kSellRows);
            S.chunk_w[ch] = wmin | (w << 8);
        }
    // a site's rows past its degree hold the site itself, so reading them is
    // valid and hits the site's own state (lanes past the class end hold 0);
    // 8 trailing padding rows let a kernel read 8 rows past any chunk
    S.col.assign((size_t)S.chunk_ptr[n_chunks] + 8 * 64, 0);
    std::vector<int32_t> row;
    for (int c = 0; c < Q; ++c)
        for (int ch = S.chunk_off[c]; ch < S.chunk_off[c + 1]; ++ch) {
            const int first = g.colour_off[c] + (ch - S.chunk_off[c]) * 64;
            const int last = std::min(first + 64, g.colour_off[c + 1]);
            for (int k = first; k < last; ++k) {
                const int cm = S.order[k];
                row.assign(g.col.begin() + g.row_ptr[cm], g.col.begin() + g.row_ptr[cm + 1]);
                for (int32_t &j : row) j = inv[j];
                std::sort(row.begin(), row.end());
                for (size_t a = 0; a < row.size(); ++a) S.col[S.chunk_ptr[ch] + a * 64 + (k - first)] = row[a];
                const int rows = (S.chunk_ptr[ch + 1] - S.chunk_ptr[ch]) / 64;
                for (int a = (int)row.size(); a < rows; ++a) S.col[S.chunk_ptr[ch] + a * 64 + (k - first)] = k;
            }
        }
    return S;
}

}  // namespace xy

using namespace xy;

extern "C" const char *xy_last_error(void) { return g_last_error.c_str(); }

namespace {

// Dilute Levy graph, periodic (the torus) or free (the open square).  The
// displacement set is listed in raster order (dy outer, dx inner) and drawn
// by inverting the sequential prefix sums of (dx^2 + dy^2)^(-rho/2).
xy_status levy_build(int L, int z, double rho, uint64_t seed, bool free_bc, const char *who, xy_graph **out)
{
    if (!out) return set_error(XY_EINVAL, std::string(who) + ": out is NULL");
    *out = nullptr;
    if (!free_bc && (L < 2 || (L & 1))) return set_error(XY_EINVAL, std::string(who) + ": L must be even and >= 2");
    if (free_bc && L < 2) return set_error(XY_EINVAL, std::string(who) + ": L must be >= 2");
    if (L > (free_bc ? 4096 : 46340)) return set_error(XY_EINVAL, std::string(who) + ": L too large");
    if (!(rho >= 0.0) || !std::isfinite(rho))
        return set_error(XY_EINVAL, std::string(who) + ": rho must be finite and >= 0");
    const int64_t N = (int64_t)L * L;
    if (z < 1 || (N * z) % 2 != 0 || z >= N - 1)
        return set_error(XY_EINVAL, std::string(who) + ": need z >= 1, N*z even and z < N-1");
    const int64_t M = N * z / 2;
    if (M > (int64_t)1 << 30) return set_error(XY_EINVAL, std::string(who) + ": too many links");

    xy_graph *g = new (std::nothrow) xy_graph;
    if (!g) return set_error(XY_ENOMEM, std::string(who) + ": out of memory");
    try {
        g->n = (int)N; g->m = (int)M; g->L = L;
        // side of the displacement square and its offset: periodic dx, dy in
        // {-L/2+1..L/2}, free in {-(L-1)..L-1}; entry f of the square is
        // (f % side - lo, f / side - lo), the centre (d = 0) left out
        const int64_t side = free_bc ? 2 * (int64_t)L - 1 : L, lo = free_bc ? L - 1 : L / 2 - 1;
        const int64_t centre = lo * side + lo, K = side * side - 1;
        auto disp = [&](int64_t k, int &dx, int &dy) {
            const int64_t f = k < centre ? k : k + 1;
            dx = (int)(f % side - lo);
            dy = (int)(f / side - lo);
        };
        std::vector<double> prefix((size_t)K);
        {
            double run = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                int dx, dy;
                disp(k, dx, dy);
                run = run + std::pow((double)((int64_t)dx * dx + (int64_t)dy * dy), -0.5 * rho);
                prefix[k] = run;
            }
        }
        const double total = prefix[K - 1];
        std::unordered_set<uint64_t> linked;
        linked.reserve((size_t)(2 * M));
        g->edges.reserve(2 * (size_t)M);
        const int64_t cap = 1000 * M + 1000000;
        int64_t t = 0, have = 0;
        const uint32_t s0 = (uint32_t)seed, s1 = (uint32_t)(seed >> 32);
        while (have < M) {
            if (t >= cap) {
                delete g;
                return set_error(XY_ECONVERGE, std::string(who) + ": attempt cap reached before N*z/2 links");
            }
            const U4 w = philox4x32_10({(uint32_t)t, (uint32_t)(t >> 32), free_bc ? 1u : 0u, tag(kGraph)}, s0, s1);
            ++t;
            const int32_t i = (int32_t)(((uint64_t)w.x * (uint64_t)N) >> 32);
            const double target = unit53(w.y, w.z) * total;
            int64_t k = std::upper_bound(prefix.begin(), prefix.end(), target) - prefix.begin();
            if (k == K) k = K - 1;
            int dx, dy;
            disp(k, dx, dy);
            const int xi = i % L, yi = i / L;
            int xj = xi + dx, yj = yi + dy;
            if (free_bc) {
                if (xj < 0 || xj >= L || yj < 0 || yj >= L) continue;     // outside the square
            } else {
                xj = (xj % L + L) % L;
                yj = (yj % L + L) % L;
            }
            const int32_t j = yj * L + xj;
            const uint64_t key = (uint64_t)std::min(i, j) * (uint64_t)N + (uint64_t)std::max(i, j);
            if (!linked.insert(key).second) continue;
            g->edges.push_back(i);
            g->edges.push_back(j);
            ++have;
        }
        g->attempts = t;
        g->cx.resize(N); g->cy.resize(N);
        for (int v = 0; v < N; ++v) { g->cx[v] = v % L; g->cy[v] = v / L; }
        const xy_status st = finish_graph(*g);
        if (st != XY_OK) { delete g; return st; }
    } catch (const std::bad_alloc &) {
        delete g;
        return set_error(XY_ENOMEM, std::string(who) + ": out of memory");
    }
    *out = g;
    return XY_OK;
}

}  // namespace

extern "C" xy_status xy_graph_levy(int L, int z, double rho, uint64_t seed, xy_graph **out)
{
    return levy_build(L, z, rho, seed, false, "xy_graph_levy", out);
}

extern "C" xy_status xy_graph_levy_free(int L, int z, double rho, uint64_t seed, xy_graph **out)
{
    return levy_build(L, z, rho, seed, true, "xy_graph_levy_free", out);
}

extern "C" xy_status xy_graph_from_edges(int n, int m, const int32_t *edges, const int32_t *coords,
                                         int L, xy_graph **out)
{
    if (!out) return set_error(XY_EINVAL, "xy_graph_from_edges: out is NULL");
    *out = nullptr;
    if (n < 1 || m < 0 || (m > 0 && !edges) || L < 1 || L > 65535)
        return set_error(XY_EINVAL, "xy_graph_from_edges: need n >= 1, m >= 0, edges, 1 <= L < 65536");
    xy_graph *g = new (std::nothrow) xy_graph;
    if (!g) return set_error(XY_ENOMEM, "xy_graph_from_edges: out of memory");
    try {
        g->n = n; g->m = m; g->L = L;
        std::unordered_set<uint64_t> seen;
        for (int e = 0; e < m; ++e) {
            const int a = edges[2 * e], b = edges[2 * e + 1];
            if (a < 0 || b < 0 || a >= n || b >= n || a == b) {
                delete g;
                return set_error(XY_EINVAL, "xy_graph_from_edges: index out of range or self link");
            }
            const uint64_t key = (uint64_t)std::min(a, b) * (uint64_t)n + (uint64_t)std::max(a, b);
            if (!seen.insert(key).second) {
                delete g;
                return set_error(XY_EINVAL, "xy_graph_from_edges: repeated link");
            }
        }
        g->edges.assign(edges, edges + 2 * (size_t)m);
        g->cx.resize(n); g->cy.resize(n);
        for (int v = 0; v < n; ++v) {
            g->cx[v] = coords ? coords[2 * v] : v % L;
            g->cy[v] = coords ? coords[2 * v + 1] : v / L;
            if (g->cx[v] < 0 || g->cy[v] < 0 || g->cx[v] >= L || g->cy[v] >= L) {
                delete g;
                return set_error(XY_EINVAL, "xy_graph_from_edges: coordinates must be in [0, L)");
            }
        }
        const xy_status st = finish_graph(*g);
        if (st != XY_OK) { delete g; return st; }
    } catch (const std::bad_alloc &) {
        delete g;
        return set_error(XY_ENOMEM, "xy_graph_from_edges: out of memory");
    }
    *out = g;
    return XY_OK;
}

extern "C" xy_status xy_graph_info(const xy_graph *g, int *n, int *m, int *n_colours, int *max_degree,
                                   int64_t *attempts)
{
    if (!g) return set_error(XY_EINVAL, "xy_graph_info: graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (n_colours) *n_colours = g->Q;
    if (max_degree) *max_degree = g->max_deg;
    if (attempts) *attempts = g->attempts;
    return XY_OK;
}

extern "C" xy_status xy_graph_export(const xy_graph *g, int32_t *edges, int32_t *colour, int32_t *perm,
                                     int32_t *colour_off, int32_t *row_ptr, int32_t *col)
{
    if (!g) return set_error(XY_EINVAL, "xy_graph_export: graph is NULL");
    if (edges) std::copy(g->edges.begin(), g->edges.end(), edges);
    if (colour) std::copy(g->colour.begin(), g->colour.end(), colour);
    if (perm) std::copy(g->perm.begin(), g->perm.end(), perm);
    if (colour_off) std::copy(g->colour_off.begin(), g->colour_off.end(), colour_off);
    if (row_ptr) std::copy(g->row_ptr.begin(), g->row_ptr.end(), row_ptr);
    if (col) std::copy(g->col.begin(), g->col.end(), col);
    return XY_OK;
}

extern "C" void xy_graph_free(xy_graph *g) { delete g; }
