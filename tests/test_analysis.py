"""Host analysis (jackknife, U4, xi_2, c): CPU tests.

Pins: the jackknife reproduces the standard error of the mean exactly for a
linear observable, and its bias correction of a square equals the closed
form mean^2 - s^2/n; on infinite-temperature oracle records (independent
uniform spins) U4 = 1 - 1/N, chi(0)/chi(k_min) = 1 and xi_2 = 0 within errors.
"""
import numpy as np
import pytest

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


def test_crossing_of_two_lines():
    T = np.linspace(1.0, 3.0, 9)
    assert abs(analysis.crossing(T, 0.5 + 0.1 * (T - 2.13), 0.5 + 0.4 * (T - 2.13)) - 2.13) < 1e-12
    assert analysis.crossing(T, T, T + 1.0) is None


def _u4_records(T, slope, G, n_rec=8, noise=None):
    """Records whose thermal U4 is 0.5 + slope (T - 2.05) in every sample
    (|m|^2 = 1, |m|^4 = 1 + U4), optionally with per-sample noise."""
    u = 0.5 + slope * (np.asarray(T) - 2.05)
    rec = np.zeros((n_rec, G, len(T), 8))
    rec[:, :, :, 1] = 1.0
    rec[:, :, :, 2] = 1.0 + u
    if noise is not None:
        rec[:, :, :, 2] += noise[None, :, None]
    return rec


def test_u4_crossing_exact_and_jackknife():
    T = np.linspace(1.6, 2.4, 11)
    est, err = analysis.u4_crossing(T, _u4_records(T, -0.2, 6), _u4_records(T, -0.6, 5))
    assert abs(est - 2.05) < 1e-12 and err < 1e-12
    # sample-to-sample scatter of the large size only: the crossing moves with
    # the mean shift and the jackknife error is the shift's standard error
    # divided by the slope difference (linear curves)
    noise = np.random.default_rng(2).normal(scale=0.01, size=40)
    est, err = analysis.u4_crossing(T, _u4_records(T, -0.2, 6), _u4_records(T, -0.6, 40, noise=noise))
    assert abs(est - (2.05 + noise.mean() / 0.4)) < 1e-9
    assert abs(err - noise.std(ddof=1) / np.sqrt(40) / 0.4) < 1e-9


def test_fss_tc_recovers_the_law():
    N = np.array([256.0, 1024.0, 4096.0])
    tc, c = analysis.fss_tc(N, 1.93 + 3.0 * N ** -0.5, 2.0)
    assert abs(tc - 1.93) < 1e-12 and abs(c - 3.0) < 1e-10


def test_bethe_tc():
    # I1/I0 at beta = 1 and 0.1 (tabulated Bessel ratios) give T = 1 and 10
    assert abs(analysis.bethe_tc(1.0 / 0.446389965896535) - 1.0) < 1e-10
    assert abs(analysis.bethe_tc(1.0 / 0.049937603987939) - 10.0) < 1e-8
    # the analytic value for the Erdos-Renyi graph of mean degree 4 (Sec. 4)
    assert abs(analysis.bethe_tc(4.0) - 1.9361) < 1e-4


def test_degree_distribution_pins():
    # the z = 4, large-rho periodic graph is the square lattice: P(k) = delta(k - 4)
    e, _ = oracle.levy_graph(16, 4, 60.0, 1)
    p = analysis.degree_distribution(e, 256)
    assert p.size == 5 and p[4] == 1.0
    # any graph: the mean degree is 2M/N = z exactly
    for boundary in ("periodic", "free"):
        e, _ = oracle.levy_graph(24, 6, 3.5, 2, boundary=boundary)
        p = analysis.degree_distribution(e, 576)
        assert abs(np.sum(np.arange(p.size) * p) - 6.0) < 1e-12 and abs(p.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("rho", [0.5, 1.0, 7 / 3, 10 / 3, 14 / 3])
def test_colour_classes_at_most_six_at_z4(rho):
    """App. B: for N <= 2^16 and z = 4 the colouring never needs more than 6
    colours; the classes partition the sites."""
    for L, seeds in ((64, range(4)), (256, range(2))):
        for s in seeds:
            e, _ = oracle.levy_graph(L, 4, rho, s)
            colour, q = oracle.slo_colour(L * L, e)
            f = analysis.colour_fractions(colour)
            assert q <= 6 and f.size == q and abs(f.sum() - 1.0) < 1e-12 and (f > 0).all()


def _scaling_records(T, N, G, u_fn, m2_fn, rng=None):
    """Records [n_rec, G, n_T, 8] whose thermal |m|^2 is m2_fn(T) and U4 is
    u_fn(T) (|m|^4 = (1 + U4) |m|^2^2), optionally with per-sample noise."""
    m2 = m2_fn(T)
    u = u_fn(T)
    rec = np.zeros((4, G, T.size, 8))
    rec[:, :, :, 1] = m2
    rec[:, :, :, 2] = (1.0 + u) * m2 ** 2
    if rng is not None:
        rec[:, :, :, 2] *= 1.0 + 0.01 * rng.normal(size=(1, G, 1))
    return rec


def test_nu_bar_and_gamma_over_nu_from_exact_scaling():
    """U4 = 0.6 - 0.5 (T - 1.9) N^(1/2) and chi(T) = N^(1/2) c(T): nu_bar = 2
    and gamma/nu_bar = 1/2 come out exactly (linear curves, no noise)."""
    T = np.linspace(1.7, 2.2, 21)
    N = [256, 1024, 4096, 16384]
    recs = [_scaling_records(T, n, 5, lambda t, n=n: 0.6 - 0.5 * (t - 1.9) * n ** 0.5,
                             lambda t, n=n: n ** -0.5 * (3.0 - t)) for n in N]
    nu, err = analysis.nu_bar_from_u4(T, N, recs, u_target=0.6, discard=0.0)
    assert abs(nu - 2.0) < 1e-10 and err < 1e-10
    g, gerr = analysis.gamma_over_nu_bar(T, N, recs, T_ref=1.93, discard=0.0)
    assert abs(g - 0.5) < 1e-12 and gerr < 1e-12
    # sample-to-sample noise gives a finite jackknife error around the same value
    rng = np.random.default_rng(3)
    recs = [_scaling_records(T, n, 30, lambda t, n=n: 0.6 - 0.5 * (t - 1.9) * n ** 0.5,
                             lambda t, n=n: n ** -0.5 * (3.0 - t), rng) for n in N]
    nu, err = analysis.nu_bar_from_u4(T, N, recs, u_target=0.6, discard=0.0)
    assert 0 < err < 0.2 and abs(nu - 2.0) < 5 * err


def test_u4_slope_at():
    T = np.array([1.0, 2.0, 3.0])
    t, s = analysis.u4_slope_at(T, np.array([0.9, 0.5, 0.1]), 0.6)
    assert abs(t - 1.75) < 1e-12 and abs(s + 0.4) < 1e-12
    assert analysis.u4_slope_at(T, np.array([0.9, 0.8, 0.7]), 0.1) is None


def test_eta_and_kt_temperature_from_exact_scaling():
    """chi = L^(2 - eta(T)) (ln L)^(-1/8) c(T) with eta(T) = 1/4 + 1.5 (T - 0.894)
    (the square-lattice form of Sec. 4, Eq. chi_SR): eta_of_T returns eta(T)
    and t_eta the temperature where eta = 1/4, exactly; with per-sample noise
    the jackknife error is finite and covers it.  A dropped log correction
    (r = 0) moves the answer, so the correction is pinned too."""
    T = np.linspace(0.80, 1.00, 11)
    L = [16, 32, 64, 128]
    eta = 0.25 + 1.5 * (T - 0.894)

    def recs(G, rng=None):
        out = []
        for l in L:
            m2 = l ** (-eta) * np.log(l) ** (-1.0 / 8) * (1.2 - 0.1 * T)
            out.append(_scaling_records(T, l * l, G, lambda t: np.zeros_like(t), lambda t, m2=m2: m2, rng))
            if rng is not None:
                out[-1][:, :, :, 1] *= 1.0 + 0.002 * rng.normal(size=(1, G, 1))
        return out

    r = recs(4)
    assert np.allclose(analysis.eta_of_T(T, L, r, discard=0.0), eta, atol=1e-12)
    t, err = analysis.t_eta(T, L, r, discard=0.0)
    assert abs(t - 0.894) < 1e-12 and err < 1e-12
    t0, _ = analysis.t_eta(T, L, r, r=0.0, discard=0.0)
    assert abs(t0 - 0.894) > 0.005
    t, err = analysis.t_eta(T, L, recs(24, np.random.default_rng(5)), discard=0.0)
    assert 0 < err < 0.01 and abs(t - 0.894) < 5 * err
