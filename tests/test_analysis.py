"""Host analysis (jackknife, U4, xi_2, c): CPU tests.

Pins: the jackknife reproduces the standard error of the mean exactly for a
linear observable, and its bias correction of a square equals the closed
form mean^2 - s^2/n; on infinite-temperature oracle records (independent
uniform spins) U4 = 1 - 1/N, chi(0)/chi(k_min) = 1 and xi_2 = 0 within errors.
"""
import json

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
    """chi = L^(2 - eta(T)) (ln L)^(1/8) c(T) with eta(T) = 1/4 + 1.5 (T - 0.894)
    (the square-lattice form of Sec. 4, Eq. chi_SR, with the KT exponent
    r = -1/16): eta_of_T returns eta(T) and t_eta the temperature where
    eta = 1/4, exactly; with per-sample noise the jackknife error is finite
    and covers it.  A dropped log correction (r = 0) or the opposite sign
    moves the answer, so the correction is pinned too."""
    T = np.linspace(0.80, 1.00, 11)
    L = [16, 32, 64, 128]
    eta = 0.25 + 1.5 * (T - 0.894)

    def recs(G, rng=None):
        out = []
        for l in L:
            m2 = l ** (-eta) * np.log(l) ** (1.0 / 8) * (1.2 - 0.1 * T)
            out.append(_scaling_records(T, l * l, G, lambda t: np.zeros_like(t), lambda t, m2=m2: m2, rng))
            if rng is not None:
                out[-1][:, :, :, 1] *= 1.0 + 0.002 * rng.normal(size=(1, G, 1))
        return out

    r = recs(4)
    assert np.allclose(analysis.eta_of_T(T, L, r, discard=0.0), eta, atol=1e-12)
    t, err = analysis.t_eta(T, L, r, discard=0.0)
    assert abs(t - 0.894) < 1e-12 and err < 1e-12
    for r_wrong in (0.0, 1.0 / 16):
        t0, _ = analysis.t_eta(T, L, r, r=r_wrong, discard=0.0)
        assert abs(t0 - 0.894) > 0.005
    t, err = analysis.t_eta(T, L, recs(24, np.random.default_rng(5)), discard=0.0)
    assert 0 < err < 0.01 and abs(t - 0.894) < 5 * err


def test_compare_chains_calibrated_and_detects_bias():
    """compare_chains on synthetic chains with known law: two independent
    sets of AR(1) chains (autocorrelation time 5 records, bins of 50) with
    equal means give z-scores with the standard normal's tails (fraction
    beyond 3 sigma near 0.27%, chi^2/dof near 1), for the per-sample and the
    disorder-paired comparisons; a shift of 6 standard errors planted in one
    (temperature, observable) of one set is flagged there, and only there,
    by the disorder-paired comparison."""
    rng = np.random.default_rng(7)
    n, G, R, Q = 1000, 64, 12, 5
    phi = np.exp(-1 / 5)

    def ar1():
        x = np.empty((n, G, R, Q))
        x[0] = rng.standard_normal((G, R, Q))
        e = rng.standard_normal((n, G, R, Q)) * np.sqrt(1 - phi ** 2)
        for t in range(1, n):
            x[t] = phi * x[t - 1] + e[t]
        return x

    disorder = rng.standard_normal((1, G, R, Q)) * 3.0        # sample-to-sample offsets, shared by both sets
    a, b = ar1() + disorder, ar1() + disorder
    res = analysis.compare_chains(a, b, n_bins=20)
    ps, dis = res["per_sample"], res["disorder"]
    assert ps["n"] == G * R * Q and dis["n"] == R * Q
    assert ps["frac_gt"] < 0.01 and 0.85 < ps["chi2_dof"] < 1.2, ps
    assert dis["chi2_dof"] < 1.6 and dis["max_abs"] < 4.0, dis
    # planted bias: set b shifted at (T index 3, observable 1) by 6 standard
    # errors of the disorder mean of the difference
    sd = np.sqrt(2 * (1 + phi) / (1 - phi) / n)               # error of one chain's mean
    shift = 6 * sd * np.sqrt(2) / np.sqrt(G)
    b2 = b.copy()
    b2[:, :, 3, 1] += shift
    res2 = analysis.compare_chains(a, b2, n_bins=20)
    flagged = {idx for idx, _ in res2["disorder"]["outliers"]}
    assert (3, 1) in flagged and len(flagged) <= 2, res2["disorder"]["outliers"]
    # a shift of one chain by 8 of its own errors is a per-sample outlier
    b3 = b.copy()
    b3[:, 5, 7, 2] += 8 * sd * np.sqrt(2)
    res3 = analysis.compare_chains(a, b3, n_bins=20)
    assert (5, 7, 2) in {idx for idx, _ in res3["per_sample"]["outliers"]}
    # drift: a chain that moves between the two halves of its records is flagged
    b4 = b.copy()
    b4[n // 2:, 9, 0, 0] += 10 * sd * np.sqrt(2)
    res4 = analysis.compare_chains(a, b4, n_bins=20)
    assert (1, 9, 0, 0) in {idx for idx, _ in res4["drift"]["outliers"]}


def test_comparison_bars_are_calibrated():
    """The bars the statistical comparisons use, checked by simulation under
    the null: the family-wise |z| bar and the chi^2/dof bar (without its 1.5
    floor) are each exceeded by about alpha of the families of independent
    normal z, and by at most a few alpha when the z are Student t with the
    stated degrees of freedom; the fixed 1.5 on 20 normal z would false-fail
    several percent of the time (the reason for the quantile)."""
    rng = np.random.default_rng(11)
    alpha, trials = 0.01, 40000
    for n, dof in ((20, np.inf), (20, 15), (80, 31), (120, 63)):
        z = rng.standard_normal((trials, n)) if not np.isfinite(dof) else rng.standard_t(dof, (trials, n))
        zb = analysis.familywise_z_bar(n, dof, alpha)
        cb = analysis.chi2_dof_bar(n, dof, alpha, floor=0.0)
        p_max = np.mean(np.abs(z).max(axis=1) > zb)
        p_chi = np.mean((z ** 2).mean(axis=1) > cb)
        assert 0.5 * alpha < p_max < 1.5 * alpha, (n, dof, p_max)
        assert (0.5 * alpha < p_chi < 1.5 * alpha) if not np.isfinite(dof) else (p_chi < 4 * alpha), (n, dof, p_chi)
    z = rng.standard_normal((trials, 20))
    assert np.mean((z ** 2).mean(axis=1) > 1.5) > 0.05
    # comparison_ok applies them to compare_chains summaries
    few = {"n": 20, "n_undefined": 0, "frac_gt": 0.05, "chi2_dof": 1.65, "max_abs": 2.99}
    assert analysis.comparison_ok(few, "few", dof=15)
    assert not analysis.comparison_ok(dict(few, max_abs=6.0), "few", dof=15)
    assert not analysis.comparison_ok(dict(few, chi2_dof=2.7), "few", dof=15)
    assert not analysis.comparison_ok(few, "many")
    assert analysis.comparison_ok(dict(few, n=2000, frac_gt=0.008, chi2_dof=1.1), "many")
    assert not analysis.comparison_ok(dict(few, n_undefined=1), "few", dof=15)


def test_hotelling_reduces_to_t_test_and_is_calibrated():
    """analysis.hotelling: with one observable its p-value is the two-sided
    one-sample t-test's (paired) and Welch-free two-sample t with the
    conservative nu (unpaired); under the null with strongly correlated
    observables (|m|^2 and |m|^4 move together) its family-wise bar rejects
    about alpha of the data sets, where a chi^2 of the marginal z would
    reject many times more; a shift of Mahalanobis length 8 along one
    temperature's observables is detected."""
    from scipy import stats
    rng = np.random.default_rng(5)
    x = rng.standard_normal((40, 3, 1)) + 0.3
    mv = analysis.hotelling(x)
    for t in range(3):
        assert np.isclose(mv["pval"][t], stats.ttest_1samp(x[:, t, 0], 0.0).pvalue, rtol=1e-9)
    y = rng.standard_normal((40, 3, 1))
    mv2 = analysis.hotelling(x, y)
    for t in range(3):
        tt = (x[:, t, 0].mean() - y[:, t, 0].mean()) / np.sqrt(x[:, t, 0].var(ddof=1) / 40 + y[:, t, 0].var(ddof=1) / 40)
        assert np.isclose(mv2["T2"][t], tt * tt, rtol=1e-12)
        assert np.isclose(mv2["pval"][t], 2 * stats.t.sf(abs(tt), 39), rtol=1e-9)
    # correlated observables: E, m2, m4 with correlations -0.9, -0.9, 0.99
    C = np.eye(5)
    C[0, 1] = C[1, 0] = C[0, 2] = C[2, 0] = -0.9
    C[1, 2] = C[2, 1] = 0.99
    A = np.linalg.cholesky(C)
    alpha, trials, G, n_T = 0.01, 2000, 64, 8
    rej_mv = rej_chi = 0
    for _ in range(trials):
        d = rng.standard_normal((G, n_T, 5)) @ A.T
        mv = analysis.hotelling(d, alpha=alpha)
        rej_mv += not analysis.hotelling_ok(mv, alpha)
        z = d.mean(0) / (d.std(0, ddof=1) / np.sqrt(G))
        rej_chi += np.mean(z ** 2) > analysis.chi2_dof_bar(z.size, G - 1, alpha, floor=0.0)
    assert rej_mv / trials < 2.5 * alpha, rej_mv / trials
    assert rej_chi / trials > 3 * alpha, rej_chi / trials
    d = rng.standard_normal((G, n_T, 5)) @ A.T
    d[:, 3] += (8.0 / np.sqrt(G)) * A[:, 1]          # a correlated move of one temperature, Mahalanobis 8
    mv = analysis.hotelling(d)
    assert not analysis.hotelling_ok(mv) and int(np.argmin(mv["pval"])) == 3


def _fss_records(T, L, nu_bar=2.0, tc=1.93, bn=0.125, dbn=0.1, G=8, n_rec=4, noise=0.0, seed=0):
    """Records of one size whose disorder-averaged U4 follows exact scaling,
    U4(T, N) = 0.5 - 0.02 (T - tc) N^(1/nu_bar) (linear in T, so ladder
    interpolation is exact), and whose <|m|^2> = 0.3 N^(-2 x(T)) with
    x(T) = bn + dbn (T - tc) (Eq. mscaling with beta/nu_bar = x(tc))."""
    N = float(L * L)
    T = np.asarray(T)
    u = 0.5 - 0.02 * (T - tc) * N ** (1.0 / nu_bar)
    m2 = 0.3 * N ** (-2.0 * (bn + dbn * (T - tc)))
    rec = np.zeros((n_rec, G, len(T), 8))
    rng = np.random.default_rng(seed)
    scale = 1.0 + noise * rng.standard_normal(G)        # per-sample scatter of |m|^2, U4 unchanged per sample
    rec[:, :, :, 1] = m2[None, None, :] * scale[None, :, None]
    rec[:, :, :, 2] = (1.0 + u)[None, None, :] * rec[:, :, :, 1] ** 2
    return rec


def test_app_c_joint_fits_recover_exact_scaling():
    """App. C on synthetic exact scaling: the joint fit of Eq. Tfsscaling over
    three U4 sets (common exponent, free exponents, fixed exponent) returns
    T_c and x = 1/nu_bar; Eq. scaling_lndotU4 with a common slope returns
    nu_bar; Eq. mscaling and Eq. chiscaling return x(T) and 1 - 2 x(T)
    (Rushbrooke-Widom: gamma/nu_bar = 1 - 2 beta/nu_bar) at every ladder
    temperature, and beta_over_nu_bar its value at T_c."""
    T = np.linspace(1.5, 2.4, 19)                       # 1.93 is not a ladder point; 1.95 is
    Ls = [16, 32, 64, 128]
    Ns = [L * L for L in Ls]
    recs = [_fss_records(T, L) for L in Ls]
    targets = [0.4, 0.5, 0.6]
    for kw in ({}, {"common_x": False}, {"x_fixed": 0.5}):
        r = analysis.tc_from_u4_sets(T, Ns, recs, targets, **kw)
        assert abs(r["T_c"] - 1.93) < 1e-9, (kw, r["T_c"])
        assert np.allclose(r["x"], 0.5, atol=1e-7), (kw, r["x"])
        assert r["T_c_error"] < 1e-9
    nu, nu_err = analysis.nu_bar_joint(T, Ns, recs, targets)
    assert abs(nu - 2.0) < 1e-10 and nu_err < 1e-10
    x_m, e_m = analysis.size_exponent_curve(T, Ns, recs, "m")
    x_c, _ = analysis.size_exponent_curve(T, Ns, recs, "chi")
    assert np.allclose(x_m, 0.125 + 0.1 * (T - 1.93), atol=1e-12) and np.all(e_m < 1e-12)
    assert np.allclose(x_c, 1.0 - 2.0 * x_m, atol=1e-12)
    b, _ = analysis.beta_over_nu_bar(T, Ns, recs, 1.95)
    assert abs(b - (0.125 + 0.1 * 0.02)) < 1e-12
    g, _ = analysis.gamma_over_nu_bar(T, Ns, recs, 1.95)
    assert abs(g - (1.0 - 2.0 * b)) < 1e-12


def test_tf_joint_fit_free_exponents_and_errors():
    """Eq. Tfsscaling with exponents that differ between the U4 sets (the
    paper's choice for rho > 3.75) is recovered exactly; per-sample scatter of
    |m|^2 (U4 per sample unchanged) leaves T_c exact; scatter of U4 gives a
    jackknife error that shrinks as 1/sqrt(samples)."""
    N = np.array([256.0, 1024.0, 4096.0, 16384.0, 65536.0])
    A, x = np.array([0.8, -0.3, 1.5]), np.array([0.35, 0.5, 0.7])
    Tf = 1.75 + A[None, :] * N[:, None] ** (-x[None, :])
    r = analysis.tf_joint_fit(Tf, N, common_x=False)
    assert abs(r["T_c"] - 1.75) < 1e-8 and np.allclose(r["x"], x, atol=1e-6) and np.allclose(r["A"], A, atol=1e-6)
    T = np.linspace(1.5, 2.4, 19)
    Ls = [16, 32, 64]
    recs = [_fss_records(T, L, noise=0.05, seed=L) for L in Ls]
    r = analysis.tc_from_u4_sets(T, [L * L for L in Ls], recs, [0.45, 0.55])
    assert abs(r["T_c"] - 1.93) < 1e-9
    errs = []
    for G in (16, 64):
        recs = []
        for L in Ls:
            rec = _fss_records(T, L, G=G, seed=L)
            rng = np.random.default_rng(100 + L + G)
            rec[:, :, :, 2] += 0.02 * rng.standard_normal(G)[None, :, None] * rec[:, :, :, 1] ** 2
            recs.append(rec)
        errs.append(analysis.tc_from_u4_sets(T, [L * L for L in Ls], recs, [0.45, 0.55])["T_c_error"])
    assert errs[0] > 0 and 1.3 < errs[0] / errs[1] < 3.2, errs


def test_graph_reports():
    """The Fig. 1 / Fig. 15 report entry point on small sizes: every P(k)
    sums to 1 with mean degree exactly z; rho = 1/2 is close to the Poisson
    law of mean z (Sec. 2: the rho -> 0 limit is Erdos-Renyi); colour-class
    fractions sum to 1, sorted largest first, at most 6 classes (App. B)."""
    from paper_1211_3991_amd import reports
    d = reports.degree_report(L=64, rhos=(0.5, 14 / 3), samples=2)
    assert len(d["curves"]) == 4
    for c in d["curves"]:
        P = np.asarray(c["P"])
        assert abs(P.sum() - 1.0) < 1e-12 and abs(c["mean_degree"] - 4.0) < 1e-12
    mf = np.asarray(d["curves"][0]["P"])
    pois = np.asarray(d["poisson"][:mf.size])
    assert np.max(np.abs(mf - pois)) < 0.02
    c = reports.colour_report(exps=(8, 10), samples=2)
    for s in c["sizes"]:
        f = np.asarray(s["fractions"])
        assert abs(f.sum() - 1.0) < 1e-12 and np.all(np.diff(f) <= 0) and f.size <= 6
        assert s["spread"] == pytest.approx(f[0] - f[-1], abs=0.05)
    json.dumps(d), json.dumps(c)
