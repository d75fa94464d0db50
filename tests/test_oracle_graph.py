"""Pins of the oracle's Levy-graph builder and SLO colouring (CPU only).

What fixes the graph, independently of the oracle's own code:
* exact link count Nz/2, no self-loops, no multi-edges (Sec. 1.1, Sec. 2);
* rho -> infinity at z = 4 is the square lattice, every degree 4 (Sec. 2,
  text after Eq. Levyi); at z = 6 the 2N nearest-neighbour links plus
  diagonal links;
* rho = 0 is the Erdos-Renyi graph: degree law Binomial(N-1, z/(N-1)), i.e.
  Poisson(z) for large N (Sec. 2, the rho = 0 limit);
* the raw draws (before rejection) follow |r|^-rho over the minimum-image
  displacements, checked against a direct enumeration of all site pairs;
* the total weight sum_r r^-rho equals values computed independently of this
  code (6.850 at L=16, rho=3.5; 11.02 at L=16, rho=2.5; 7.008 at L=256, rho=3.5).
Colouring (App. B "Graph coloring"): properness, the greedy (Grundy)
property, Q <= degeneracy + 1, and 2 colours on the square lattice
(the paper reports 2 colours at rho = infinity).
Parity: pinned.
"""
import numpy as np
import pytest
from scipy import stats

import oracle


def _check_simple(edges, n, m):
    assert edges.shape == (m, 2)
    assert edges.min() >= 0 and edges.max() < n
    assert np.all(edges[:, 0] != edges[:, 1])
    key = np.minimum(edges[:, 0], edges[:, 1]).astype(np.int64) * n + np.maximum(edges[:, 0], edges[:, 1])
    assert np.unique(key).size == m


def _min_image(d, L):
    d = np.abs(d) % L
    return np.minimum(d, L - d)


@pytest.mark.parametrize("L,z,rho,seed", [(16, 6, 3.5, 1), (32, 6, 2.5, 7), (16, 4, 0.0, 3), (64, 6, 4.5, 0)])
def test_link_count_simple_graph(L, z, rho, seed):
    n = L * L
    e, att = oracle.levy_graph(L, z, rho, seed)
    _check_simple(e, n, n * z // 2)
    assert att >= n * z // 2


def test_rho_infinite_is_square_lattice():
    L = 16
    n = L * L
    e, _ = oracle.levy_graph(L, 4, 60.0, 3)
    _check_simple(e, n, 2 * n)
    deg = np.bincount(e.ravel(), minlength=n)
    assert np.all(deg == 4)
    xi, yi = e[:, 0] % L, e[:, 0] // L
    xj, yj = e[:, 1] % L, e[:, 1] // L
    r2 = _min_image(xi - xj, L) ** 2 + _min_image(yi - yj, L) ** 2
    assert np.all(r2 == 1)


def test_rho_large_z6_fills_nearest_then_diagonal():
    L = 16
    n = L * L
    e, _ = oracle.levy_graph(L, 6, 20.0, 5)
    xi, yi = e[:, 0] % L, e[:, 0] // L
    xj, yj = e[:, 1] % L, e[:, 1] // L
    r2 = _min_image(xi - xj, L) ** 2 + _min_image(yi - yj, L) ** 2
    assert np.sum(r2 == 1) == 2 * n            # every nearest-neighbour pair
    assert np.sum(r2 == 2) >= n - 3            # the rest is (almost) all diagonal


def test_rho_zero_degree_law_is_binomial():
    L, z = 128, 6
    n = L * L
    degs = []
    for seed in (11, 12):
        e, _ = oracle.levy_graph(L, z, 0.0, seed)
        degs.append(np.bincount(e.ravel(), minlength=n))
    deg = np.concatenate(degs)
    kmax = 14
    obs = np.array([np.sum(deg == k) for k in range(kmax)] + [np.sum(deg >= kmax)], dtype=float)
    p = stats.binom.pmf(np.arange(kmax), n - 1, z / (n - 1))
    p = np.append(p, 1 - p.sum())
    exp = p * deg.size
    chi2 = np.sum((obs - exp) ** 2 / exp)
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4, (obs, exp)
    assert abs(deg.mean() - z) < 1e-12


@pytest.mark.parametrize("L,rho", [(16, 3.5), (16, 2.5), (32, 1.0)])
def test_raw_draw_law_matches_enumeration(L, rho):
    n = L * L
    ndraw = 400_000
    ij = oracle.levy_raw_draws(L, rho, 99, ndraw)
    # site i is uniform
    cnt = np.bincount(ij[:, 0], minlength=n)
    chi2 = np.sum((cnt - ndraw / n) ** 2 / (ndraw / n))
    assert stats.chi2.sf(chi2, n - 1) > 1e-4
    # displacement law: enumerate every target site j != 0 of site 0 on the torus
    xs, ys = np.meshgrid(np.arange(L), np.arange(L))
    xs, ys = xs.ravel(), ys.ravel()
    r2 = (_min_image(xs, L) ** 2 + _min_image(ys, L) ** 2).astype(float)
    w = np.zeros(n)
    w[1:] = r2[1:] ** (-rho / 2)
    p = w / w.sum()
    # translate each draw so that i sits at the origin
    dx = (ij[:, 1] % L - ij[:, 0] % L) % L
    dy = (ij[:, 1] // L - ij[:, 0] // L) % L
    obs = np.bincount(dy * L + dx, minlength=n).astype(float)
    assert obs[0] == 0
    # group by distance shell to keep expected counts large
    shells = np.unique(r2[1:])
    o_sh = np.array([obs[r2 == s].sum() for s in shells])
    e_sh = np.array([p[r2 == s].sum() for s in shells]) * ndraw
    big = e_sh >= 20
    o_fold, e_fold = o_sh[big], e_sh[big]
    if (~big).any():
        o_fold = np.append(o_fold, o_sh[~big].sum())
        e_fold = np.append(e_fold, e_sh[~big].sum())
    chi2 = np.sum((o_fold - e_fold) ** 2 / e_fold)
    assert stats.chi2.sf(chi2, len(o_fold) - 1) > 1e-4
    # within a shell, every displacement equally likely (covers sign/axis errors)
    for s in shells[:3]:
        sel = (r2 == s)
        sub = obs[sel]
        assert stats.chisquare(sub).pvalue > 1e-4


@pytest.mark.parametrize("L,rho,total", [(16, 3.5, 6.850), (16, 2.5, 11.02), (256, 3.5, 7.008),
                                         (128, 2.5, 13.75), (512, 4.5, 5.456)])
def test_weight_total(L, rho, total):
    assert abs(oracle.levy_weight_total(L, rho) - total) < 6e-3


def _degeneracy(n, edges):
    """k-core peeling (a different algorithm from SLO): largest k with a
    non-empty k-core."""
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    deg = np.array([len(x) for x in adj])
    alive = np.ones(n, bool)
    k = 0
    while alive.any():
        k += 1
        changed = True
        while changed:
            changed = False
            dead = np.nonzero(alive & (deg < k))[0]
            for v in dead:
                alive[v] = False
                changed = True
                for w in adj[v]:
                    if alive[w]:
                        deg[w] -= 1
        if not alive.any():
            return k - 1
    return k


@pytest.mark.parametrize("L,z,rho,seed", [(16, 6, 3.5, 1), (32, 6, 2.5, 2), (32, 6, 4.5, 4), (16, 6, 0.0, 9)])
def test_slo_colouring_properties(L, z, rho, seed):
    n = L * L
    e, _ = oracle.levy_graph(L, z, rho, seed)
    col, q = oracle.slo_colour(n, e)
    assert col.min() == 0 and col.max() == q - 1
    assert np.all(col[e[:, 0]] != col[e[:, 1]])           # proper
    # Grundy property: a site of colour c sees every colour below c
    nbc = [set() for _ in range(n)]
    for a, b in e:
        nbc[a].add(col[b])
        nbc[b].add(col[a])
    for v in range(n):
        assert set(range(col[v])) <= nbc[v]
    assert q <= _degeneracy(n, e) + 1


def test_square_lattice_two_colours():
    e, _ = oracle.levy_graph(16, 4, 60.0, 3)
    col, q = oracle.slo_colour(256, e)
    assert q == 2
    assert np.all(col[e[:, 0]] != col[e[:, 1]])


def test_slo_tiny_graphs():
    # path 0-1-2: SLO removes 0 (deg 1, smallest index), then 1 (deg 1), then 2;
    # colours in reverse: 2 -> 0, 1 -> 1, 0 -> 0
    col, q = oracle.slo_colour(3, np.array([[0, 1], [1, 2]]))
    assert list(col) == [0, 1, 0] and q == 2
    col, q = oracle.slo_colour(4, np.array([[0, 1], [1, 2], [2, 0], [0, 3], [1, 3], [2, 3]]))
    assert q == 4 and sorted(col) == [0, 1, 2, 3]
    col, q = oracle.slo_colour(3, np.zeros((0, 2), dtype=np.int32))
    assert q == 1 and list(col) == [0, 0, 0]


# --- free boundaries (Sec. 2: distances within the open L x L square) -------

def _pair_weights_open_square(L, rho):
    """Every unordered pair {i, j} of the open L x L square with weight r^-rho."""
    n = L * L
    xs, ys = np.arange(n) % L, np.arange(n) // L
    i, j = np.triu_indices(n, 1)
    r2 = (xs[i] - xs[j]) ** 2 + (ys[i] - ys[j]) ** 2
    return i, j, r2.astype(np.float64) ** (-rho / 2)


def test_free_boundary_pair_law_brute_force():
    """The first accepted draw of a graph is an unordered pair {i, j} with
    probability proportional to r^-rho over all pairs of the open square."""
    L, rho, n_graphs = 4, 2.5, 30000
    i, j, w = _pair_weights_open_square(L, rho)
    index = {(a, b): k for k, (a, b) in enumerate(zip(i, j))}
    counts = np.zeros(i.size)
    for seed in range(n_graphs):
        e, _ = oracle.levy_graph(L, 1, rho, seed, boundary="free")
        a, b = sorted(e[0])
        counts[index[(a, b)]] += 1
    expect = n_graphs * w / w.sum()
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert stats.chi2.sf(chi2, i.size - 1) > 1e-3, chi2


@pytest.mark.parametrize("L,z,rho,seed", [(16, 6, 3.5, 1), (17, 4, 2.5, 3), (12, 4, 14 / 3, 5), (20, 6, 0.0, 2)])
def test_free_boundary_invariants(L, z, rho, seed):
    e, att = oracle.levy_graph(L, z, rho, seed, boundary="free")
    n = L * L
    assert e.shape == (n * z // 2, 2) and att >= e.shape[0]
    assert (e >= 0).all() and (e < n).all() and (e[:, 0] != e[:, 1]).all()
    key = np.minimum(e[:, 0], e[:, 1]) * n + np.maximum(e[:, 0], e[:, 1])
    assert np.unique(key).size == key.size
    dx = e[:, 0] % L - e[:, 1] % L
    dy = e[:, 0] // L - e[:, 1] // L
    assert (np.hypot(dx, dy) <= (L - 1) * np.sqrt(2) + 1e-12).all()
    # with free boundaries no link wraps: its length is the plain distance,
    # and the periodic graph of the same seed is a different graph
    ep, _ = oracle.levy_graph(L - (L % 2), z, rho, seed)
    assert L % 2 or not np.array_equal(e, ep)


def test_free_boundary_rho_zero_is_erdos_renyi():
    """rho = 0: every pair equally likely, as for the periodic graph (the
    paper notes the Erdos-Renyi limit does not depend on the boundary)."""
    L, z = 32, 4
    n = L * L
    deg = np.concatenate([np.bincount(oracle.levy_graph(L, z, 0.0, s, boundary="free")[0].ravel(), minlength=n)
                          for s in range(20)])
    kmax = 12
    obs = np.bincount(np.minimum(deg, kmax), minlength=kmax + 1)
    p = stats.binom.pmf(np.arange(kmax + 1), n - 1, z / (n - 1))
    p[kmax] = stats.binom.sf(kmax - 1, n - 1, z / (n - 1))
    chi2 = np.sum((obs - deg.size * p) ** 2 / (deg.size * p))
    # sites are not independent (fixed link count), so the bound is loose
    assert stats.chi2.sf(chi2, kmax) > 1e-4, chi2
