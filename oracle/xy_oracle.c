/*
 * XY model on dilute Levy graphs -- sequential FP64 CPU ORACLE.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * reference for the GPU library.  It shares no code, header, table or constant
 * generator with the library under paper_1211_3991_amd/.  Only tests/,
 * __graft_entry__.smoke() and the cpu_baseline leg of bench.py may load it.
 *
 * Paper: Ibanez Berganza & Leuzzi, "Critical behavior of the XY model in
 * complex topologies" (arXiv:1211.3991).
 *   - Hamiltonian H = -sum_{i<j} J_ij S_i.S_j, J_ij in {0,1}        (Sec. 2, Eq. HXY)
 *   - dilute Levy graph, P(J_ij) ~ |r_i - r_j|^-rho, Nz/2 links, PBC (Sec. 2, Eq. Levyi;
 *                                                                    Sec. 1.1 "Levy lattice")
 *   - graph colouring by smallest-last ordering                      (App. B, "Graph coloring")
 *   - colour-parallel single-spin Metropolis, over-relaxation,
 *     parallel tempering every MCS                                   (App. B, "Improved
 *                                                                    equilibrium dynamics")
 *   - observables E, m, |m|^2, |m|^4, chi(k_min)                     (Sec. 3, Eqs. specificheat,
 *                                                                    chi, U4, xi_2)
 *
 * Readings where the paper is silent (the numbering matches the list of
 * readings kept with the design notes): unit-vector FP64 state, 1 Metropolis
 * + 5 OR sub-sweeps, uniform proposal by rejection in the unit disk, the
 * Philox counter layout, smallest-index tie break in SLO, even/odd PT pairing
 * by sweep parity, swap of temperature labels (not spins).
 *
 *   - random walks, histogram of self-return times                   (Sec. 2, spectral dimension;
 *                                                                    App. A)
 *
 * Parity status of each function is stated in its comment ("pinned by ...").
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -std=c99 -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Counter-based: out = bijection_key(counter).   */
/* Pinned by: rocRAND's host Philox4x32-10 generator (tests/test_oracle_rng) */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oxy_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int r;
    for (r = 0; r < 10; r++) {
        uint64_t p0, p1;
        uint32_t n0, n1, n2, n3;
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        n1 = (uint32_t)p1;
        n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Purposes of a draw (top byte of counter word 3). */
enum { P_GRAPH = 1, P_INIT = 2, P_MET = 3, P_MET_ACC = 4, P_OR = 5, P_PT = 6, P_RW = 7, P_RW_START = 8 };

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                 uint32_t c3, uint32_t w[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = c0; ctr[1] = c1; ctr[2] = c2; ctr[3] = c3;
    key[0] = (uint32_t)seed; key[1] = (uint32_t)(seed >> 32);
    oxy_philox(ctr, key, w);
}

/* 53-bit uniform in [0,1): high word gives 32 bits, low word its top 21. */
static double u53(uint32_t hi, uint32_t lo)
{
    uint64_t v = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
    return (double)v * (1.0 / 9007199254740992.0); /* 2^-53 */
}

/* ------------------------------------------------------------------------ */
/* Levy graph (Sec. 2, Eq. Levyi): N = L*L sites of a periodic square       */
/* lattice; a link i-j is drawn with probability proportional to r^-rho,   */
/* r the minimum-image Euclidean distance; links are drawn one at a time    */
/* and a drawn pair that is already linked is rejected, until Nz/2 links.   */
/* Pinned by: rho=0 degree law (Erdos-Renyi), rho->inf square lattice,     */
/* raw-draw length law vs direct enumeration, exact link count, symmetry.   */
/* ------------------------------------------------------------------------ */

/* Displacements d = (dx,dy), dx,dy in {-L/2+1..L/2}, d != 0, raster order
 * (dy outer, dx inner).  Each other site of the torus appears exactly once. */
static int disp_table(int L, double rho, int32_t *ddx, int32_t *ddy, double *cum)
{
    int K = 0, dx, dy;
    double acc = 0.0;
    for (dy = -L / 2 + 1; dy <= L / 2; dy++) {
        for (dx = -L / 2 + 1; dx <= L / 2; dx++) {
            double r2;
            if (dx == 0 && dy == 0) continue;
            r2 = (double)(dx * dx + dy * dy);
            acc = acc + pow(r2, -0.5 * rho);   /* (r^2)^(-rho/2) = r^-rho */
            ddx[K] = dx; ddy[K] = dy; cum[K] = acc;
            K++;
        }
    }
    return K;
}

/* index of the first cumulative weight strictly above t (K-1 if none) */
static int first_above(const double *cum, int K, double t)
{
    int lo = 0, hi = K - 1;
    if (!(cum[K - 1] > t)) return K - 1;
    while (lo < hi) {
        int mid = lo + (hi - lo) / 2;
        if (cum[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* One raw draw of attempt t: site i uniform, displacement by the weights. */
static void raw_draw(int L, uint64_t seed, uint64_t t, const int32_t *ddx,
                     const int32_t *ddy, const double *cum, int K,
                     int32_t *pi, int32_t *pj)
{
    uint32_t w[4];
    uint32_t N = (uint32_t)(L * L);
    int32_t i, xi, yi, xj, yj, k;
    draw(seed, (uint32_t)t, (uint32_t)(t >> 32), 0u, (uint32_t)P_GRAPH << 24, w);
    i = (int32_t)(((uint64_t)w[0] * (uint64_t)N) >> 32);
    k = first_above(cum, K, u53(w[1], w[2]) * cum[K - 1]);
    xi = i % L; yi = i / L;
    xj = ((xi + ddx[k]) % L + L) % L;
    yj = ((yi + ddy[k]) % L + L) % L;
    *pi = i; *pj = yj * L + xj;
}

/* Exposed for the raw-law test: the first n raw draws (no rejection). */
int oxy_levy_raw_draws(int L, double rho, uint64_t seed, int64_t n, int32_t *ij)
{
    int K = L * L - 1;
    int32_t *ddx = malloc(sizeof(int32_t) * K), *ddy = malloc(sizeof(int32_t) * K);
    double *cum = malloc(sizeof(double) * K);
    int64_t t;
    if (!ddx || !ddy || !cum) { free(ddx); free(ddy); free(cum); return -1; }
    disp_table(L, rho, ddx, ddy, cum);
    for (t = 0; t < n; t++) raw_draw(L, seed, (uint64_t)t, ddx, ddy, cum, K, &ij[2 * t], &ij[2 * t + 1]);
    free(ddx); free(ddy); free(cum);
    return 0;
}

/* Total weight sum_d r^-rho over the displacement set (for the A2 check). */
double oxy_levy_weight_total(int L, double rho)
{
    int K = L * L - 1;
    int32_t *ddx = malloc(sizeof(int32_t) * K), *ddy = malloc(sizeof(int32_t) * K);
    double *cum = malloc(sizeof(double) * K), tot;
    if (!ddx || !ddy || !cum) { free(ddx); free(ddy); free(cum); return -1.0; }
    disp_table(L, rho, ddx, ddy, cum);
    tot = cum[K - 1];
    free(ddx); free(ddy); free(cum);
    return tot;
}

typedef struct { int32_t *v; int n, cap; } ilist;

static int ilist_push(ilist *l, int32_t x)
{
    if (l->n == l->cap) {
        int nc = l->cap ? 2 * l->cap : 8;
        int32_t *nv = realloc(l->v, sizeof(int32_t) * nc);
        if (!nv) return -1;
        l->v = nv; l->cap = nc;
    }
    l->v[l->n++] = x;
    return 0;
}

static int ilist_has(const ilist *l, int32_t x)
{
    int a;
    for (a = 0; a < l->n; a++) if (l->v[a] == x) return 1;
    return 0;
}

/* Returns 0 on success, -1 on bad arguments / no memory, -2 if the attempt
 * cap was hit.  edges[2*e], edges[2*e+1] = (i, j) of the e-th accepted draw. */
int oxy_levy_graph(int L, int z, double rho, uint64_t seed, int32_t *edges,
                   int64_t *n_attempts)
{
    int64_t N, M, m = 0, t = 0, cap;
    int K, a, rc = 0;
    int32_t *ddx, *ddy;
    double *cum;
    ilist *adj;
    if (L < 2 || (L % 2) != 0 || z < 1 || !(rho >= 0.0)) return -1;
    N = (int64_t)L * L;
    if ((N * z) % 2 != 0 || z >= N - 1) return -1;
    M = N * z / 2;
    K = (int)(N - 1);
    ddx = malloc(sizeof(int32_t) * K); ddy = malloc(sizeof(int32_t) * K);
    cum = malloc(sizeof(double) * K);
    adj = calloc((size_t)N, sizeof(ilist));
    if (!ddx || !ddy || !cum || !adj) { rc = -1; goto out; }
    disp_table(L, rho, ddx, ddy, cum);
    cap = 1000 * M + 1000000;
    while (m < M) {
        int32_t i, j;
        if (t >= cap) { rc = -2; break; }
        raw_draw(L, seed, (uint64_t)t, ddx, ddy, cum, K, &i, &j);
        t++;
        if (ilist_has(&adj[i], j)) continue;       /* multi-edge: reject */
        if (ilist_push(&adj[i], j) || ilist_push(&adj[j], i)) { rc = -1; break; }
        edges[2 * m] = i; edges[2 * m + 1] = j;
        m++;
    }
    if (n_attempts) *n_attempts = t;
out:
    if (adj) for (a = 0; a < N; a++) free(adj[a].v);
    free(adj); free(ddx); free(ddy); free(cum);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Levy graph with free boundaries (Sec. 2: distances within the L x L      */
/* square, no wrap; r_max = L sqrt 2).  A raw draw t takes counter          */
/* (t lo, t hi, 1, P_GRAPH << 24): site i uniform; a displacement d with    */
/* dx, dy in {-(L-1)..L-1}, d != 0, raster order (dy outer, dx inner),      */
/* weight (dx^2+dy^2)^(-rho/2), by the same inversion; j = i + d.  A draw   */
/* with j outside the square is rejected, as is one that repeats a link.    */
/* Every unordered pair {i, j} is then drawn with probability proportional  */
/* to r^-rho (from i with d, or from j with -d).                            */
/* Pinned by: the exact pair law on a 4 x 4 square (brute force), rho = 0   */
/* (every pair equally likely), exact link count and invariants.           */
/* ------------------------------------------------------------------------ */
static int disp_table_free(int L, double rho, int32_t *ddx, int32_t *ddy, double *cum)
{
    int K = 0, dx, dy;
    double acc = 0.0;
    for (dy = -(L - 1); dy <= L - 1; dy++) {
        for (dx = -(L - 1); dx <= L - 1; dx++) {
            double r2;
            if (dx == 0 && dy == 0) continue;
            r2 = (double)(dx * dx + dy * dy);
            acc = acc + pow(r2, -0.5 * rho);
            ddx[K] = dx; ddy[K] = dy; cum[K] = acc;
            K++;
        }
    }
    return K;
}

int oxy_levy_graph_free(int L, int z, double rho, uint64_t seed, int32_t *edges, int64_t *n_attempts)
{
    int64_t N, M, m = 0, t = 0, cap;
    int K, a, rc = 0;
    int32_t *ddx, *ddy;
    double *cum;
    ilist *adj;
    if (L < 2 || z < 1 || !(rho >= 0.0)) return -1;
    N = (int64_t)L * L;
    if ((N * z) % 2 != 0 || z >= N - 1) return -1;
    M = N * z / 2;
    K = (2 * L - 1) * (2 * L - 1) - 1;
    ddx = malloc(sizeof(int32_t) * K); ddy = malloc(sizeof(int32_t) * K);
    cum = malloc(sizeof(double) * K);
    adj = calloc((size_t)N, sizeof(ilist));
    if (!ddx || !ddy || !cum || !adj) { rc = -1; goto out; }
    disp_table_free(L, rho, ddx, ddy, cum);
    cap = 1000 * M + 1000000;
    while (m < M) {
        uint32_t w[4];
        int32_t i, j, xj, yj, k;
        if (t >= cap) { rc = -2; break; }
        draw(seed, (uint32_t)t, (uint32_t)(t >> 32), 1u, (uint32_t)P_GRAPH << 24, w);
        t++;
        i = (int32_t)(((uint64_t)w[0] * (uint64_t)N) >> 32);
        k = first_above(cum, K, u53(w[1], w[2]) * cum[K - 1]);
        xj = i % L + ddx[k]; yj = i / L + ddy[k];
        if (xj < 0 || xj >= L || yj < 0 || yj >= L) continue;   /* outside the square */
        j = yj * L + xj;
        if (ilist_has(&adj[i], j)) continue;                    /* multi-edge: reject */
        if (ilist_push(&adj[i], j) || ilist_push(&adj[j], i)) { rc = -1; break; }
        edges[2 * m] = i; edges[2 * m + 1] = j;
        m++;
    }
    if (n_attempts) *n_attempts = t;
out:
    if (adj) for (a = 0; a < N; a++) free(adj[a].v);
    free(adj); free(ddx); free(ddy); free(cum);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Smallest-last ordering colouring (App. B, "Graph coloring"): repeatedly  */
/* remove a site of minimum remaining degree (ties: smallest index), then   */
/* colour sites in reverse removal order with the smallest colour that no   */
/* already-coloured neighbour has.                                          */
/* Pinned by: properness, Q <= degeneracy+1, square lattice -> 2 colours.   */
/* ------------------------------------------------------------------------ */

/* binary min-heap of (degree, site) */
typedef struct { int64_t key; } hent;
static void heap_push(hent *h, int *n, int64_t key)
{
    int c = (*n)++;
    h[c].key = key;
    while (c > 0) {
        int p = (c - 1) / 2;
        if (h[p].key <= h[c].key) break;
        { hent tmp = h[p]; h[p] = h[c]; h[c] = tmp; }
        c = p;
    }
}
static int64_t heap_pop(hent *h, int *n)
{
    int64_t top = h[0].key;
    int c = 0;
    h[0] = h[--(*n)];
    for (;;) {
        int l = 2 * c + 1, r = l + 1, s = c;
        if (l < *n && h[l].key < h[s].key) s = l;
        if (r < *n && h[r].key < h[s].key) s = r;
        if (s == c) break;
        { hent tmp = h[s]; h[s] = h[c]; h[c] = tmp; }
        c = s;
    }
    return top;
}

int oxy_slo_colour(int n, int m, const int32_t *edges, int32_t *colour)
{
    int *deg = calloc((size_t)n, sizeof(int)), *start = malloc(sizeof(int) * (n + 1));
    int *fill = calloc((size_t)n, sizeof(int)), *nb = malloc(sizeof(int) * (2 * (size_t)m + 1));
    int *order = malloc(sizeof(int) * (n + 1));
    char *removed = calloc((size_t)n, 1);
    hent *heap = malloc(sizeof(hent) * ((size_t)n + 2 * (size_t)m + 1));
    int *used = NULL;
    int e, v, hn = 0, nrem = 0, Q = 0, maxdeg = 0;
    if (!deg || !start || !fill || !nb || !order || !removed || !heap) { Q = -1; goto out; }
    for (e = 0; e < m; e++) { deg[edges[2 * e]]++; deg[edges[2 * e + 1]]++; }
    start[0] = 0;
    for (v = 0; v < n; v++) { start[v + 1] = start[v] + deg[v]; if (deg[v] > maxdeg) maxdeg = deg[v]; }
    for (e = 0; e < m; e++) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        nb[start[a] + fill[a]++] = b;
        nb[start[b] + fill[b]++] = a;
    }
    /* deg[] now serves as the remaining degree */
    for (v = 0; v < n; v++) heap_push(heap, &hn, (int64_t)deg[v] * n + v);
    while (nrem < n) {
        int64_t key = heap_pop(heap, &hn);
        int d = (int)(key / n), u = (int)(key % n), a;
        if (removed[u] || deg[u] != d) continue;   /* stale entry */
        removed[u] = 1;
        order[nrem++] = u;
        for (a = start[u]; a < start[u + 1]; a++) {
            int w = nb[a];
            if (!removed[w]) { deg[w]--; heap_push(heap, &hn, (int64_t)deg[w] * n + w); }
        }
    }
    used = calloc((size_t)maxdeg + 2, sizeof(int));
    if (!used) { Q = -1; goto out; }
    for (v = 0; v < n; v++) colour[v] = -1;
    for (e = n - 1; e >= 0; e--) {
        int u = order[e], a, c;
        for (a = start[u]; a < start[u + 1]; a++) {
            int w = nb[a];
            if (colour[w] >= 0 && colour[w] <= maxdeg) used[colour[w]] = 1;
        }
        c = 0;
        while (used[c]) c++;
        colour[u] = c;
        if (c + 1 > Q) Q = c + 1;
        for (a = start[u]; a < start[u + 1]; a++) {
            int w = nb[a];
            if (colour[w] >= 0 && colour[w] <= maxdeg) used[colour[w]] = 0;
        }
    }
out:
    free(deg); free(start); free(fill); free(nb); free(order); free(removed); free(heap); free(used);
    return Q;
}

/* ------------------------------------------------------------------------ */
/* Single-site moves (App. B): Metropolis with a uniform direction proposal */
/* and over-relaxation (reflection about the local field, Creutz 1987).     */
/* Spins are FP64 unit vectors; only + - * / sqrt are used on the state.    */
/* Pinned by: von Mises law of one spin in a frozen field; OR involution    */
/* and energy conservation.                                                 */
/* ------------------------------------------------------------------------ */

/* Uniform direction: rejection sampling in the unit disk, normalised. */
static void uniform_dir(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                        uint32_t purpose_sub, double *px, double *py)
{
    uint32_t tr;
    for (tr = 0; tr < 64; tr++) {
        uint32_t w[4];
        double x, y, r2, s;
        draw(seed, c0, c1, c2, purpose_sub | tr, w);
        x = 2.0 * u53(w[0], w[1]) - 1.0;
        y = 2.0 * u53(w[2], w[3]) - 1.0;
        r2 = x * x + y * y;
        if (r2 > 1.0 || r2 == 0.0) continue;
        s = sqrt(r2);
        *px = x / s; *py = y / s;
        return;
    }
    *px = 1.0; *py = 0.0;   /* unreachable in practice: p(64 misses) ~ 1e-43 */
}

/* Metropolis move of spin (x,y) in local field (hx,hy) at inverse T beta.
 * Returns 1 if accepted. */
int oxy_met_move(double hx, double hy, double *x, double *y, double beta,
                 uint64_t seed, uint32_t site, uint32_t sweep, uint32_t slot)
{
    double xn, yn, e_old, e_new, dE;
    uint32_t w[4];
    uniform_dir(seed, site, sweep, slot, (uint32_t)P_MET << 24, &xn, &yn);
    e_old = hx * (*x) + hy * (*y);
    e_new = hx * xn + hy * yn;
    dE = e_old - e_new;            /* H = -h.S, so dE = -h.S' + h.S */
    draw(seed, site, sweep, slot, (uint32_t)P_MET_ACC << 24, w);
    if (dE <= 0.0 || u53(w[0], w[1]) < exp(-(beta * dE))) {
        *x = xn; *y = yn;
        return 1;
    }
    return 0;
}

/* Over-relaxation: S' = 2 (S.h / h.h) h - S ; unchanged if h = 0. */
void oxy_or_move(double hx, double hy, double *x, double *y)
{
    double hh = hx * hx + hy * hy, a, t;
    if (hh == 0.0) return;
    a = (hx * (*x) + hy * (*y)) / hh;
    t = 2.0 * a;
    *x = t * hx - *x;
    *y = t * hy - *y;
}

/* ------------------------------------------------------------------------ */
/* Simulation of one graph at n_T temperatures (one replica per T).         */
/* ------------------------------------------------------------------------ */
typedef struct oxy_sim {
    int n, m, L, nT, Q;
    uint64_t seed;
    int32_t *edges;        /* 2m, as given */
    int32_t *colour;       /* n */
    int32_t *cx, *cy;      /* lattice coordinates of each site */
    int *start, *nb;       /* adjacency, each list sorted by (colour, index) */
    int *by_colour;        /* sites sorted by (colour, index) */
    int *col_start;        /* Q+1 */
    double *T, *beta;      /* per temperature index */
    int *slot_of_T, *T_of_slot;
    double *sx, *sy;       /* [slot][site] */
    uint32_t sweep;        /* sweeps done so far */
    int64_t pt_acc[1024], pt_try[1024];
} oxy_sim;

/* sort sites by (colour, index): key = colour * n + index */
static int cmp_i64(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return a < b ? -1 : (a > b);
}

static int sort_by_colour(int *v, int cnt, const int32_t *colour, int n)
{
    int64_t *key = malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
    int a;
    if (!key) return -1;
    for (a = 0; a < cnt; a++) key[a] = (int64_t)colour[v[a]] * n + v[a];
    qsort(key, (size_t)cnt, sizeof(int64_t), cmp_i64);
    for (a = 0; a < cnt; a++) v[a] = (int)(key[a] % n);
    free(key);
    return 0;
}

void oxy_sim_free(oxy_sim *s)
{
    if (!s) return;
    free(s->edges); free(s->colour); free(s->cx); free(s->cy); free(s->start);
    free(s->nb); free(s->by_colour); free(s->col_start); free(s->T); free(s->beta);
    free(s->slot_of_T); free(s->T_of_slot); free(s->sx); free(s->sy);
    free(s);
}

/* coords may be NULL: then site i sits at (i % L, i / L). */
oxy_sim *oxy_sim_create(int n, int m, const int32_t *edges, const int32_t *colour,
                        const int32_t *coords, int L, int nT, const double *T,
                        uint64_t seed)
{
    oxy_sim *s = calloc(1, sizeof(oxy_sim));
    int *fill = NULL, v, e, k;
    if (!s || n < 1 || m < 0 || nT < 1 || nT > 1024 || L < 1) { free(s); return NULL; }
    s->n = n; s->m = m; s->L = L; s->nT = nT; s->seed = seed;
    s->edges = malloc(sizeof(int32_t) * (2 * (size_t)m + 1));
    s->colour = malloc(sizeof(int32_t) * n);
    s->cx = malloc(sizeof(int32_t) * n); s->cy = malloc(sizeof(int32_t) * n);
    s->start = calloc((size_t)n + 1, sizeof(int));
    s->nb = malloc(sizeof(int) * (2 * (size_t)m + 1));
    s->by_colour = malloc(sizeof(int) * n);
    s->T = malloc(sizeof(double) * nT); s->beta = malloc(sizeof(double) * nT);
    s->slot_of_T = malloc(sizeof(int) * nT); s->T_of_slot = malloc(sizeof(int) * nT);
    s->sx = malloc(sizeof(double) * (size_t)n * nT); s->sy = malloc(sizeof(double) * (size_t)n * nT);
    fill = calloc((size_t)n, sizeof(int));
    if (!s->edges || !s->colour || !s->cx || !s->cy || !s->start || !s->nb || !s->by_colour ||
        !s->T || !s->beta || !s->slot_of_T || !s->T_of_slot || !s->sx || !s->sy || !fill) {
        free(fill); oxy_sim_free(s); return NULL;
    }
    memcpy(s->edges, edges, sizeof(int32_t) * 2 * (size_t)m);
    memcpy(s->colour, colour, sizeof(int32_t) * n);
    s->Q = 0;
    for (v = 0; v < n; v++) {
        if (colour[v] + 1 > s->Q) s->Q = colour[v] + 1;
        if (coords) { s->cx[v] = coords[2 * v]; s->cy[v] = coords[2 * v + 1]; }
        else { s->cx[v] = v % L; s->cy[v] = v / L; }
    }
    for (e = 0; e < m; e++) { s->start[edges[2 * e] + 1]++; s->start[edges[2 * e + 1] + 1]++; }
    for (v = 0; v < n; v++) s->start[v + 1] += s->start[v];
    for (e = 0; e < m; e++) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        s->nb[s->start[a] + fill[a]++] = b;
        s->nb[s->start[b] + fill[b]++] = a;
    }
    free(fill);
    for (v = 0; v < n; v++)
        if (sort_by_colour(s->nb + s->start[v], s->start[v + 1] - s->start[v], s->colour, n)) {
            oxy_sim_free(s); return NULL;
        }
    for (v = 0; v < n; v++) s->by_colour[v] = v;
    if (sort_by_colour(s->by_colour, n, s->colour, n)) { oxy_sim_free(s); return NULL; }
    s->col_start = calloc((size_t)s->Q + 1, sizeof(int));
    if (!s->col_start) { oxy_sim_free(s); return NULL; }
    for (v = 0; v < n; v++) s->col_start[colour[v] + 1]++;
    for (k = 0; k < s->Q; k++) s->col_start[k + 1] += s->col_start[k];
    for (k = 0; k < nT; k++) {
        s->T[k] = T[k];
        s->beta[k] = 1.0 / T[k];
        s->slot_of_T[k] = k; s->T_of_slot[k] = k;
        s->pt_acc[k] = 0; s->pt_try[k] = 0;
    }
    for (v = 0; v < n * nT; v++) { s->sx[v] = 1.0; s->sy[v] = 0.0; }
    s->sweep = 0;
    return s;
}

int oxy_sim_n_colours(const oxy_sim *s) { return s->Q; }

/* Random initial state: an independent uniform direction per (slot, site). */
void oxy_sim_init_random(oxy_sim *s)
{
    int r, i;
    for (r = 0; r < s->nT; r++)
        for (i = 0; i < s->n; i++)
            uniform_dir(s->seed, (uint32_t)i, 0u, (uint32_t)r, (uint32_t)P_INIT << 24,
                        &s->sx[(size_t)r * s->n + i], &s->sy[(size_t)r * s->n + i]);
}

/* xy: [slot][site][2]; perm: slot_of_T (may be NULL = identity) */
void oxy_sim_set_state(oxy_sim *s, const double *xy, const int32_t *slot_of_T, uint32_t sweep)
{
    size_t a;
    int k;
    for (a = 0; a < (size_t)s->n * s->nT; a++) { s->sx[a] = xy[2 * a]; s->sy[a] = xy[2 * a + 1]; }
    for (k = 0; k < s->nT; k++) {
        s->slot_of_T[k] = slot_of_T ? slot_of_T[k] : k;
        s->T_of_slot[s->slot_of_T[k]] = k;
    }
    s->sweep = sweep;
}

void oxy_sim_get_state(const oxy_sim *s, double *xy, int32_t *slot_of_T, uint32_t *sweep)
{
    size_t a;
    int k;
    for (a = 0; a < (size_t)s->n * s->nT; a++) { xy[2 * a] = s->sx[a]; xy[2 * a + 1] = s->sy[a]; }
    if (slot_of_T) for (k = 0; k < s->nT; k++) slot_of_T[k] = s->slot_of_T[k];
    if (sweep) *sweep = s->sweep;
}

static void local_field(const oxy_sim *s, int r, int i, double *hx, double *hy)
{
    const double *X = s->sx + (size_t)r * s->n, *Y = s->sy + (size_t)r * s->n;
    double ax = 0.0, ay = 0.0;
    int a;
    for (a = s->start[i]; a < s->start[i + 1]; a++) { ax = ax + X[s->nb[a]]; ay = ay + Y[s->nb[a]]; }
    *hx = ax; *hy = ay;
}

/* Energy H = -sum_links S_i.S_j of the spins in slot r (Eq. HXY, J=1). */
double oxy_sim_energy(const oxy_sim *s, int r)
{
    const double *X = s->sx + (size_t)r * s->n, *Y = s->sy + (size_t)r * s->n;
    double E = 0.0;
    int e;
    for (e = 0; e < s->m; e++) {
        int i = s->edges[2 * e], j = s->edges[2 * e + 1];
        E = E - (X[i] * X[j] + Y[i] * Y[j]);
    }
    return E;
}

/* Observables of slot r: E, |m|^2, |m|^4, F_x, F_y, m_x, m_y, 0.
 * m = (1/N) sum S_j (Sec. 3); F = |sum_j S_j e^{i k.r_j}|^2 / N for
 * k = (2pi/L, 0) and (0, 2pi/L) -- the Fourier transform of the two-point
 * function at k_min (Sec. 3, definition of xi_2). */
static void observe(const oxy_sim *s, int r, double *o)
{
    const double *X = s->sx + (size_t)r * s->n, *Y = s->sy + (size_t)r * s->n;
    double mx = 0.0, my = 0.0, fx[4] = {0, 0, 0, 0}, fy[4] = {0, 0, 0, 0};
    const double two_pi = 6.283185307179586476925286766559;
    double N = (double)s->n, m2;
    int i;
    for (i = 0; i < s->n; i++) {
        double cx = cos(two_pi * s->cx[i] / s->L), sx = sin(two_pi * s->cx[i] / s->L);
        double cy = cos(two_pi * s->cy[i] / s->L), sy = sin(two_pi * s->cy[i] / s->L);
        mx += X[i]; my += Y[i];
        fx[0] += X[i] * cx; fx[1] += X[i] * sx; fx[2] += Y[i] * cx; fx[3] += Y[i] * sx;
        fy[0] += X[i] * cy; fy[1] += X[i] * sy; fy[2] += Y[i] * cy; fy[3] += Y[i] * sy;
    }
    mx /= N; my /= N;
    m2 = mx * mx + my * my;
    o[0] = oxy_sim_energy(s, r);
    o[1] = m2;
    o[2] = m2 * m2;
    o[3] = (fx[0] * fx[0] + fx[1] * fx[1] + fx[2] * fx[2] + fx[3] * fx[3]) / N;
    o[4] = (fy[0] * fy[0] + fy[1] * fy[1] + fy[2] * fy[2] + fy[3] * fy[3]) / N;
    o[5] = mx; o[6] = my; o[7] = 0.0;
}

/* out: [nT][8], indexed by temperature */
void oxy_sim_measure(const oxy_sim *s, double *out)
{
    int k;
    for (k = 0; k < s->nT; k++) observe(s, s->slot_of_T[k], out + 8 * (size_t)k);
}

/* Parallel tempering (Hukushima-Nemoto; App. B): on sweep number w, the
 * pairs (k, k+1) with k = w mod 2, k+2, ... are attempted; a swap exchanges
 * the temperature labels of the two slots with probability
 * min(1, exp((beta_k - beta_{k+1}) (E_k - E_{k+1}))). */
static void pt_step(oxy_sim *s, uint8_t *pt_log)
{
    double E[1024];
    int r, k;
    for (r = 0; r < s->nT; r++) E[r] = oxy_sim_energy(s, r);
    for (k = (int)(s->sweep % 2u); k + 1 < s->nT; k += 2) {
        int a = s->slot_of_T[k], b = s->slot_of_T[k + 1], acc;
        double d = (s->beta[k] - s->beta[k + 1]) * (E[a] - E[b]);
        uint32_t w[4];
        draw(s->seed, (uint32_t)k, s->sweep, 0u, (uint32_t)P_PT << 24, w);
        acc = (d >= 0.0 || u53(w[0], w[1]) < exp(d));
        s->pt_try[k]++;
        if (acc) {
            s->slot_of_T[k] = b; s->slot_of_T[k + 1] = a;
            s->T_of_slot[b] = k; s->T_of_slot[a] = k + 1;
            s->pt_acc[k]++;
        }
        if (pt_log) pt_log[k] = (uint8_t)(acc ? 1 : 2);
    }
}

/* Runs n_sweeps sweeps.  One sweep = 1 Metropolis sub-sweep then n_or OR
 * sub-sweeps; each sub-sweep visits colours 0..Q-1 in order (sites of one
 * colour are mutually unlinked, so their order does not matter).  After the
 * sweep: PT if pt_every > 0 and (sweep+1) % pt_every == 0; then a record if
 * meas_every > 0 and (sweep+1) % meas_every == 0.
 *   records : [max_rec][nT][8]        (may be NULL)
 *   met_log : [n_sweeps][nT][n] bytes, 1 = accepted, 0 = rejected, indexed
 *             by slot and lattice site (may be NULL)
 *   pt_log  : [n_sweeps][nT] bytes, 1 = swap accepted, 2 = rejected,
 *             0 = not attempted, indexed by the lower T of the pair (may be NULL)
 * Returns the number of records written. */
int oxy_sim_run(oxy_sim *s, int n_sweeps, int n_or, int pt_every, int meas_every,
                double *records, int max_rec, uint8_t *met_log, uint8_t *pt_log)
{
    int w, nrec = 0;
    for (w = 0; w < n_sweeps; w++) {
        int sub;
        for (sub = 0; sub <= n_or; sub++) {
            int c;
            for (c = 0; c < s->Q; c++) {
                int a;
                for (a = s->col_start[c]; a < s->col_start[c + 1]; a++) {
                    int i = s->by_colour[a], r;
                    for (r = 0; r < s->nT; r++) {
                        double hx, hy;
                        double *x = &s->sx[(size_t)r * s->n + i], *y = &s->sy[(size_t)r * s->n + i];
                        local_field(s, r, i, &hx, &hy);
                        if (sub == 0) {
                            int acc = oxy_met_move(hx, hy, x, y, s->beta[s->T_of_slot[r]],
                                                   s->seed, (uint32_t)i, s->sweep, (uint32_t)r);
                            if (met_log) met_log[((size_t)w * s->nT + r) * s->n + i] = (uint8_t)acc;
                        } else {
                            oxy_or_move(hx, hy, x, y);
                        }
                    }
                }
            }
        }
        if (pt_log) memset(pt_log + (size_t)w * s->nT, 0, (size_t)s->nT);
        if (pt_every > 0 && (s->sweep + 1) % (uint32_t)pt_every == 0)
            pt_step(s, pt_log ? pt_log + (size_t)w * s->nT : NULL);
        s->sweep++;
        if (meas_every > 0 && s->sweep % (uint32_t)meas_every == 0) {
            if (records && nrec < max_rec) oxy_sim_measure(s, records + (size_t)nrec * s->nT * 8);
            nrec++;
        }
    }
    return nrec < max_rec ? nrec : max_rec;
}

void oxy_sim_pt_counts(const oxy_sim *s, int64_t *acc, int64_t *tries)
{
    int k;
    for (k = 0; k < s->nT; k++) { acc[k] = s->pt_acc[k]; tries[k] = s->pt_try[k]; }
}

/* Batched Philox for tests: ctr[4n], key[2n] -> out[4n]. */
void oxy_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    int64_t a;
    for (a = 0; a < n; a++) oxy_philox(ctr + 4 * a, key + 2 * a, out + 4 * a);
}

/* Metropolis / OR moves of one spin in a frozen field, n_moves times, for
 * the detailed-balance tests; angle after each move in ang_out (radians,
 * atan2 -- test output only, not on the state path). */
int oxy_frozen_field_chain(double hx, double hy, double beta, uint64_t seed,
                           int n_moves, int or_every, double *ang_out)
{
    double x = 1.0, y = 0.0;
    int t, acc = 0;
    for (t = 0; t < n_moves; t++) {
        if (or_every > 0 && (t % or_every) == or_every - 1) oxy_or_move(hx, hy, &x, &y);
        else acc += oxy_met_move(hx, hy, &x, &y, beta, seed, 0u, (uint32_t)t, 0u);
        ang_out[t] = atan2(y, x);
    }
    return acc;
}

/* ------------------------------------------------------------------------ */
/* Random walks on the graph (Sec. 2, spectral dimension; App. A).  P(tau), */
/* the probability that a walker is back at its starting site after tau     */
/* steps, behaves as tau^(-dbar/2), dbar the spectral dimension.            */
/*                                                                          */
/* Walker w (0..n_walkers-1) starts at                                      */
/*   start_mode 0: the lattice centre, site (L/2) L + L/2;                  */
/*   start_mode 1: the k-th site, in lattice order, of degree larger than   */
/*     two, k = (x count) >> 32, x word 0 of the draw (w, 0, 0, P_RW_START).*/
/* Step t (t = 0 .. n_steps-1) moves from the current site to its neighbour */
/* number (x deg) >> 32, neighbours in ascending lattice index, x word      */
/* t mod 4 of the draw (w, t / 4, 0, P_RW).  A walker on a site of degree 0 */
/* stays.  hist[t] (t = 0 .. n_steps) counts the walkers at their start     */
/* after t steps, so hist[0] = n_walkers.  starts (may be NULL) receives    */
/* the starting sites.                                                      */
/* Pinned by: the square lattice, whose return probability after 2n steps   */
/* is (C(2n,n)/4^n)^2 and after an odd number 0, and the start-site rule.   */
/* Returns 0, -1 on bad arguments, -2 without an eligible start, -3 on      */
/* allocation failure.                                                      */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b)
{
    const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int oxy_random_walk(int n, int m, const int32_t *edges, int L, int n_walkers, int n_steps,
                    uint64_t seed, int start_mode, uint64_t *hist, int32_t *starts)
{
    int32_t *deg, *off, *nbr, *fill, *elig = NULL;
    int i, e, w, t, n_elig = 0, rc = 0;
    if (n < 1 || m < 0 || n_walkers < 0 || n_steps < 0 || (start_mode != 0 && start_mode != 1)) return -1;
    if (start_mode == 0 && (L < 2 || L * L != n)) return -1;
    deg = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    off = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    fill = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
    if (!deg || !off || !fill || !nbr) { rc = -3; goto done; }
    for (e = 0; e < m; e++) { deg[edges[2 * e]]++; deg[edges[2 * e + 1]]++; }
    for (i = 0; i < n; i++) off[i + 1] = off[i] + deg[i];
    for (e = 0; e < m; e++) {
        const int32_t a = edges[2 * e], b = edges[2 * e + 1];
        nbr[off[a] + fill[a]++] = b;
        nbr[off[b] + fill[b]++] = a;
    }
    for (i = 0; i < n; i++) qsort(nbr + off[i], (size_t)deg[i], sizeof(int32_t), cmp_i32);
    if (start_mode == 1) {
        elig = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        if (!elig) { rc = -3; goto done; }
        for (i = 0; i < n; i++) if (deg[i] > 2) elig[n_elig++] = i;
        if (n_elig == 0) { rc = -2; goto done; }
    }
    for (t = 0; t <= n_steps; t++) hist[t] = 0;
    for (w = 0; w < n_walkers; w++) {
        uint32_t x[4];
        int32_t s0, cur;
        if (start_mode == 0) {
            s0 = (L / 2) * L + L / 2;
        } else {
            draw(seed, (uint32_t)w, 0u, 0u, (uint32_t)P_RW_START << 24, x);
            s0 = elig[(uint32_t)(((uint64_t)x[0] * (uint64_t)n_elig) >> 32)];
        }
        if (starts) starts[w] = s0;
        cur = s0;
        hist[0]++;
        for (t = 0; t < n_steps; t++) {
            if ((t & 3) == 0) draw(seed, (uint32_t)w, (uint32_t)(t >> 2), 0u, (uint32_t)P_RW << 24, x);
            if (deg[cur] > 0) cur = nbr[off[cur] + (int32_t)(((uint64_t)x[t & 3] * (uint64_t)deg[cur]) >> 32)];
            if (cur == s0) hist[t + 1]++;
        }
    }
done:
    free(deg); free(off); free(fill); free(nbr); free(elig);
    return rc;
}
