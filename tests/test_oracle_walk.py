"""Pins of the oracle's random walks (Sec. 2, spectral dimension; App. A).

The z = 4, large-rho Levy graph is the square lattice (pinned in the graph
tests), on which a simple random walk is back at its start after 2n steps with
probability (C(2n, n) / 4^n)^2 (the two coordinates of the rotated lattice
walk are independent one-dimensional walks) and never after an odd number of
steps.  The start rule and the spectral-dimension fit are pinned as well.
"""
from math import comb

import numpy as np

import oracle
from paper_1211_3991_amd import analysis


def _square(L):
    e, _ = oracle.levy_graph(L, 4, 60.0, 3)
    return L * L, e


def test_square_lattice_return_probability():
    n, e = _square(64)
    W, T = 20000, 64
    h = oracle.random_walk(n, e, 64, W, T, seed=5, start_mode=0)
    assert h[0] == W and not h[1::2].any()            # bipartite: no odd returns
    for t in range(2, T + 1, 2):
        p = (comb(t, t // 2) / 4 ** (t // 2)) ** 2
        sigma = np.sqrt(p * (1 - p) / W)
        assert abs(h[t] / W - p) < 4.5 * sigma, (t, h[t] / W, p)


def test_start_rule_and_determinism():
    L = 32
    e, _ = oracle.levy_graph(L, 4, 3.5, 11)
    n = L * L
    deg = np.bincount(e.ravel(), minlength=n)
    h1, s1 = oracle.random_walk(n, e, L, 5000, 50, seed=9, start_mode=1, return_starts=True)
    h2, s2 = oracle.random_walk(n, e, L, 5000, 50, seed=9, start_mode=1, return_starts=True)
    assert np.array_equal(h1, h2) and np.array_equal(s1, s2)
    assert (deg[s1] > 2).all()
    # every eligible site is reachable as a start and the choice is uniform
    elig = np.flatnonzero(deg > 2)
    counts = np.bincount(np.searchsorted(elig, s1), minlength=elig.size)
    chi2 = np.sum((counts - s1.size / elig.size) ** 2) / (s1.size / elig.size)
    assert chi2 < elig.size + 5 * np.sqrt(2 * elig.size)
    # a different seed gives different walks
    assert not np.array_equal(h1, oracle.random_walk(n, e, L, 5000, 50, seed=10, start_mode=1))


def test_isolated_start_site_stays():
    # a site of degree 0 is never eligible; with the centre start on a graph
    # whose centre is isolated, the walker stays and returns at every step
    L = 4
    edges = np.array([[0, 1], [1, 2]], dtype=np.int32)       # centre (2, 2) = site 10 is isolated
    h = oracle.random_walk(L * L, edges, L, 3, 5, seed=1, start_mode=0)
    assert np.array_equal(h, np.full(6, 3, dtype=np.uint64))


def test_spectral_dimension_of_the_square_lattice():
    n, e = _square(128)
    h = oracle.random_walk(n, e, 128, 20000, 256, seed=7, start_mode=0)
    d, err = analysis.spectral_dimension(h, 16, 256)
    assert abs(d - 2.0) < max(0.1, 4 * err), (d, err)
