"""Host analysis (jackknife, U4, xi_2, c): CPU tests.

Pins: the jackknife reproduces the standard error of the mean exactly for a
linear observable, and its bias correction of a square equals the closed
form mean^2 - s^2/n; on infinite-temperature oracle records (independent
uniform spins) U4 = 1 - 1/N, chi(0)/chi(k_min) = 1 and xi_2 = 0 within errors.
"""
import numpy as np

import oracle
from paper_1211_3991_amd import analysis


def test_jackknife_linear_is_standard_error():
    rng = np.random.default_rng(3)
    b = rng.normal(size=40)
    v, e = analysis.jackknife(lambda x: x, [b])
    assert abs(v - b.mean()) < 1e-14
    assert abs(e - b.std(ddof=1) / np.sqrt(len(b))) < 1e-14


def test_jackknife_bias_correction_of_square():
    rng = np.random.default_rng(4)
    b = rng.normal(loc=0.3, size=25)
    v, _ = analysis.jackknife(lambda x: x * x, [b])
    n = len(b)
    assert abs(v - (b.mean() ** 2 - b.var(ddof=1) / n)) < 1e-13


def test_infinite_temperature_cumulants():
    L = 16
    n = L * L
    e, _ = oracle.levy_graph(L, 6, 3.5, 1)
    col, _ = oracle.slo_colour(n, e)
    sim = oracle.Sim(n, e, col, L, np.array([1e30]), 21)
    sim.init_random()
    rec = sim.run(20_000, meas_every=1)["records"][:, None]          # [n, G=1, T=1, 8]
    out = analysis.thermal(rec, n, [1e30], L, 3.5, n_bins=40, discard=0.0)
    U4, eU = out["U4"]
    assert abs(U4[0, 0] - (1 - 1 / n)) < 4.5 * eU[0, 0]
    r, er = out["ratio"]
    assert abs(r[0, 0] - 1) < 4.5 * er[0, 0]
    assert abs(out["chi"][0][0, 0] - 1) < 4.5 * out["chi"][1][0, 0]
    d = analysis.disorder(np.repeat(rec, 4, axis=1)[:, :, :, :], n, np.array([1e30]), L, 3.5)
    assert d["U4"][0].shape == (1,)


def test_psi():
    assert analysis.psi_of(2.5) == 0.5 and analysis.psi_of(3.5) == 1.5 and analysis.psi_of(4.5) == 2.0
