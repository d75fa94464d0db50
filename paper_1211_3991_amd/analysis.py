"""Host analysis of measurement records (Sec. 3 observables, Sec. 4 method).

Records come from ``Batch.records()``: float64 [n_rec, G, n_T, 8] with
columns E, |m|^2, |m|^4, F_x, F_y, m_x, m_y, 0.  Thermal averages use the
second half of the records (the last exponential time window, Sec. 4) and
errors come from a jackknife over contiguous time bins (per sample) or over
samples (disorder averages).

Definitions (Sec. 3):
  c    = (<H^2> - <H>^2) / (N T^2)                       Eq. (specificheat)
  chi  = N <|m|^2>  (and N(<|m|^2> - |<m>|^2) with the m vector)   Eq. (chi)
  U4   = <m^4> / <m^2>^2 - 1      (per sample; disorder: mean<m^4> / mean(<m^2>^2) - 1)
  xi_2 = [chi(0)/chi(k_min) - 1]^(1/psi) / (2 sin(|k_min|/2)),  chi(k) = <F(k)>,
         chi(0) = N <|m|^2>, |k_min| = 2 pi / L, psi = rho - 2 for rho < 3.75 else 2
"""
import numpy as np

E, M2, M4, FX, FY, MX, MY = range(7)


def psi_of(rho):
    """Long-range exponent psi of the correlation length (rho - d in the
    long-range regime, 2 in the short-range one; d = 2, boundary rho = 3.75)."""
    return rho - 2.0 if rho < 3.75 else 2.0


def bin_means(x, n_bins):
    """Means of n_bins contiguous bins along axis 0 (trailing remainder dropped)."""
    x = np.asarray(x, dtype=np.float64)
    nb = x.shape[0] // n_bins
    if nb < 1:
        raise ValueError(f"need at least {n_bins} records, have {x.shape[0]}")
    return x[: nb * n_bins].reshape((n_bins, nb) + x.shape[1:]).mean(axis=1)


def jackknife(fn, blocks):
    """Jackknife of fn over the first axis of each array in `blocks` (one entry
    per bin or per sample).  Returns (bias-corrected estimate, error)."""
    blocks = [np.asarray(b, dtype=np.float64) for b in blocks]
    n = blocks[0].shape[0]
    full = fn(*[b.mean(axis=0) for b in blocks])
    tot = [b.sum(axis=0) for b in blocks]
    loo = np.array([fn(*[(t - b[i]) / (n - 1) for t, b in zip(tot, blocks)]) for i in range(n)])
    mean_loo = loo.mean(axis=0)
    est = n * full - (n - 1) * mean_loo
    err = np.sqrt((n - 1) / n * np.sum((loo - mean_loo) ** 2, axis=0))
    return est, err


def _observables(N, T, L, rho):
    """Functions of the bin means (E, E^2, m2, m4, F) for one sample/temperature."""
    beta = 1.0 / T
    psi = psi_of(rho)
    s = 2.0 * np.sin(np.pi / L)

    def xi2(m2, f):
        r = N * m2 / f - 1.0
        return np.where(r > 0, np.abs(r) ** (1.0 / psi), np.nan) / s

    return {
        "e": lambda e, e2, m2, m4, f: e / N,
        "c": lambda e, e2, m2, m4, f: beta * beta * (e2 - e * e) / N,
        "chi": lambda e, e2, m2, m4, f: N * m2,
        "U4": lambda e, e2, m2, m4, f: m4 / (m2 * m2) - 1.0,
        "ratio": lambda e, e2, m2, m4, f: N * m2 / f,
        "xi2": lambda e, e2, m2, m4, f: xi2(m2, f),
    }


def thermal(records, N, T, L, rho, n_bins=20, discard=0.5):
    """Per-sample thermal averages with jackknife errors.

    records: [n_rec, G, n_T, 8]; N, L, rho: per-sample sequences (or scalars);
    T: [n_T] or [G, n_T].  Returns {name: (value[G, n_T], error[G, n_T])}."""
    rec = np.asarray(records, dtype=np.float64)
    rec = rec[int(rec.shape[0] * discard):]
    n_rec, G, R, _ = rec.shape
    N = np.broadcast_to(np.asarray(N, dtype=np.float64), (G,))
    L = np.broadcast_to(np.asarray(L, dtype=np.float64), (G,))
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (G,))
    T = np.broadcast_to(np.asarray(T, dtype=np.float64), (G, R))
    out = {}
    for g in range(G):
        for k in range(R):
            x = rec[:, g, k]
            f = 0.5 * (x[:, FX] + x[:, FY])
            series = [x[:, E], x[:, E] ** 2, x[:, M2], x[:, M4], f]
            blocks = [bin_means(sr, n_bins) for sr in series]
            for name, fn in _observables(N[g], T[g, k], L[g], rho[g]).items():
                v, e = jackknife(fn, blocks)
                if name not in out:
                    out[name] = (np.full((G, R), np.nan), np.full((G, R), np.nan))
                out[name][0][g, k] = v
                out[name][1][g, k] = e
    return out


def disorder(records, N, T, L, rho, discard=0.5):
    """Disorder averages over the G samples (same N, L, rho) with a jackknife
    over samples.  U4 is the ratio of disorder averages as printed in Sec. 3:
    mean <m^4> / mean(<m^2>^2) - 1.  Returns {name: (value[n_T], error[n_T])}."""
    rec = np.asarray(records, dtype=np.float64)
    rec = rec[int(rec.shape[0] * discard):]
    th = rec.mean(axis=0)                                  # [G, n_T, 8] thermal averages
    e2 = (rec[:, :, :, E] ** 2).mean(axis=0)               # [G, n_T]
    T = np.asarray(T, dtype=np.float64)
    beta = 1.0 / T
    psi = psi_of(rho)
    s = 2.0 * np.sin(np.pi / L)
    f = 0.5 * (th[:, :, FX] + th[:, :, FY])
    var = e2 - th[:, :, E] ** 2                            # per-sample <H^2> - <H>^2
    blocks = [th[:, :, E], var, th[:, :, M2], th[:, :, M4], th[:, :, M2] ** 2, f]
    fns = {
        "e": lambda e, v, m2, m4, m2sq, ff: e / N,
        "c": lambda e, v, m2, m4, m2sq, ff: beta * beta * v / N,
        "chi": lambda e, v, m2, m4, m2sq, ff: N * m2,
        "U4": lambda e, v, m2, m4, m2sq, ff: m4 / m2sq - 1.0,
        "xi2": lambda e, v, m2, m4, m2sq, ff: np.abs(N * m2 / ff - 1.0) ** (1.0 / psi) / s,
    }
    return {name: jackknife(fn, blocks) for name, fn in fns.items()}


def crossing(T, ya, yb):
    """Temperature where the curves ya(T) and yb(T) cross: the first sign change
    of ya - yb along the ladder T (ascending), linearly interpolated.  None if
    they do not cross."""
    T = np.asarray(T, dtype=np.float64)
    d = np.asarray(ya, dtype=np.float64) - np.asarray(yb, dtype=np.float64)
    for k in range(len(T) - 1):
        if d[k] == 0.0:
            return float(T[k])
        if d[k] * d[k + 1] < 0.0:
            return float(T[k] - d[k] * (T[k + 1] - T[k]) / (d[k + 1] - d[k]))
    return float(T[-1]) if d[-1] == 0.0 else None


def u4_samples(records, discard=0.5):
    """Per-sample thermal <m^4> and <m^2>^2 ([G, n_T] each) of records
    [n_rec, G, n_T, 8], after discarding the first part (Sec. 4)."""
    rec = np.asarray(records, dtype=np.float64)
    rec = rec[int(rec.shape[0] * discard):]
    th = rec.mean(axis=0)
    return th[:, :, M4], th[:, :, M2] ** 2


def u4_crossing(T, rec_small, rec_large, discard=0.5):
    """Crossing temperature of the disorder-averaged U4 (Sec. 3, ratio of
    disorder averages) of two sizes, with a jackknife error over the samples
    of both sizes (independent sets: the leave-one-out variances add).
    Sec. 4 estimates T_c from the crossing of U4(T, N) with U4(T, N/4)."""
    a4, a2 = u4_samples(rec_small, discard)
    b4, b2 = u4_samples(rec_large, discard)

    def cross(a4m, a2m, b4m, b2m):
        return crossing(T, a4m / a2m - 1.0, b4m / b2m - 1.0)

    est = cross(a4.mean(0), a2.mean(0), b4.mean(0), b2.mean(0))
    if est is None:
        return None, None
    var = 0.0
    for x4, x2, other, first in ((a4, a2, (b4.mean(0), b2.mean(0)), True), (b4, b2, (a4.mean(0), a2.mean(0)), False)):
        n = x4.shape[0]
        s4, s2 = x4.sum(0), x2.sum(0)
        loo = []
        for i in range(n):
            m4, m2 = (s4 - x4[i]) / (n - 1), (s2 - x2[i]) / (n - 1)
            c = cross(m4, m2, *other) if first else cross(*other, m4, m2)
            if c is not None:
                loo.append(c)
        loo = np.asarray(loo)
        if loo.size > 1:
            var += (n - 1) / n * np.sum((loo - loo.mean()) ** 2)
    return est, float(np.sqrt(var))


def fss_tc(N, T_cross, nu_bar):
    """T_c from crossing temperatures T(N) under T(N) = C N^(-1/nu_bar) + T_c
    (Sec. 4): least squares in (N^(-1/nu_bar), T).  Returns (T_c, C)."""
    x = np.asarray(N, dtype=np.float64) ** (-1.0 / nu_bar)
    A = np.stack([np.ones_like(x), x], axis=1)
    (tc, c), *_ = np.linalg.lstsq(A, np.asarray(T_cross, dtype=np.float64), rcond=None)
    return float(tc), float(c)


def bethe_tc(excess_degree):
    """Critical temperature of the XY model on a locally tree-like random
    graph in the Bethe approximation: I1(beta)/I0(beta) = 1 / excess degree
    (the excess degree <k^2>/<k> - 1 is z for a Poisson degree of mean z)."""
    from scipy.optimize import brentq
    from scipy.special import i0e, i1e
    f = lambda b: i1e(b) / i0e(b) - 1.0 / excess_degree
    return 1.0 / brentq(f, 1e-9, 50.0)


def spectral_dimension(hist, t_min, t_max):
    """Spectral dimension from a self-return histogram (Sec. 2, spectral
    dimension; App. A): P(tau) ~ tau^(-dbar/2), so dbar = -2 x the slope of
    log hist against log tau over t_min <= tau <= t_max (times with no return
    are skipped, e.g. odd times on a bipartite graph).  Weighted least squares
    with Poisson weights (variance of log count ~ 1 / count).  Returns
    (dbar, its standard error from the fit)."""
    h = np.asarray(hist, dtype=np.float64)
    t = np.arange(h.size, dtype=np.float64)
    sel = (t >= t_min) & (t <= t_max) & (h > 0)
    if sel.sum() < 3:
        raise ValueError("need at least three times with returns in the window")
    x, y, w = np.log(t[sel]), np.log(h[sel]), h[sel]
    A = np.stack([np.ones_like(x), x], axis=1)
    Aw = A * w[:, None]
    cov = np.linalg.inv(A.T @ Aw)
    coef = cov @ (Aw.T @ y)
    return float(-2.0 * coef[1]), float(2.0 * np.sqrt(cov[1, 1]))


def degree_distribution(edges, n):
    """P(k), the fraction of the n sites with k links (Sec. 2, the degree
    distributions of the dilute graphs): float64[k_max + 1]."""
    e = np.asarray(edges).reshape(-1, 2)
    deg = np.bincount(e.ravel(), minlength=n)
    return np.bincount(deg) / float(n)


def colour_fractions(colour):
    """Fraction of the sites in each colour class (App. B, "Graph coloring":
    the sizes of the sets updated in parallel): float64[Q]."""
    c = np.asarray(colour)
    return np.bincount(c) / float(c.size)


def _u4_curve(m4, m2sq):
    """Disorder-averaged U4 (ratio of averages, Sec. 3) from per-sample arrays."""
    return m4.mean(0) / m2sq.mean(0) - 1.0


def u4_slope_at(T, U, u_target):
    """(T*, dU/dT at T*) where the curve U(T) first crosses u_target, from
    the linear segment of the ladder that brackets it; None if it does not."""
    T = np.asarray(T, dtype=np.float64)
    d = np.asarray(U, dtype=np.float64) - u_target
    for k in range(len(T) - 1):
        if d[k] == 0.0 or d[k] * d[k + 1] < 0.0:
            slope = (d[k + 1] - d[k]) / (T[k + 1] - T[k])
            return float(T[k] - d[k] / slope), float(slope)
    return None


def _jackknife_sizes(est, per_size):
    """est(list of per-size argument tuples of sample means) -> scalar, with a
    jackknife error over the samples of each size (independent sets, the
    leave-one-out variances add).  per_size: list of tuples of [G, ...] arrays."""
    means = [tuple(a.mean(0) for a in arrs) for arrs in per_size]
    value = est(means)
    var = 0.0
    for s, arrs in enumerate(per_size):
        n = arrs[0].shape[0]
        tot = [a.sum(0) for a in arrs]
        loo = []
        for i in range(n):
            trial = list(means)
            trial[s] = tuple((t - a[i]) / (n - 1) for t, a in zip(tot, arrs))
            v = est(trial)
            if v is not None and np.isfinite(v):
                loo.append(v)
        loo = np.asarray(loo)
        if loo.size > 1:
            var += (n - 1) / n * np.sum((loo - loo.mean()) ** 2)
    return value, float(np.sqrt(var))


def nu_bar_from_u4(T, N, records, u_target, discard=0.5):
    """nu_bar from dU4/dT at fixed U4 (Sec. 4, Eq. U4dot): |dU4/dT| at the
    temperature where U4(T, N) = u_target grows as N^(1/nu_bar).  records:
    one [n_rec, G, n_T, 8] array per size N.  Returns (nu_bar, error), the
    error a jackknife over the samples of every size."""
    per_size = [u4_samples(r, discard) for r in records]
    lnN = np.log(np.asarray(N, dtype=np.float64))

    def est(means):
        ln_slopes = []
        for m4, m2sq in means:
            hit = u4_slope_at(T, m4 / m2sq - 1.0, u_target)
            if hit is None:
                return None
            ln_slopes.append(np.log(abs(hit[1])))
        inv_nu = np.polyfit(lnN, ln_slopes, 1)[0]
        return 1.0 / inv_nu

    return _jackknife_sizes(est, per_size)


def gamma_over_nu_bar(T, N, records, T_ref, discard=0.5):
    """gamma / nu_bar from chi = N <|m|^2> at T_ref (Sec. 3, Eq. chi; Sec. 4):
    chi(T_ref, N) ~ N^(gamma/nu_bar), chi linearly interpolated along the
    ladder.  Returns (gamma/nu_bar, jackknife error over samples)."""
    T = np.asarray(T, dtype=np.float64)
    per_size = []
    for r in records:
        rec = np.asarray(r, dtype=np.float64)
        rec = rec[int(rec.shape[0] * discard):]
        per_size.append((rec.mean(axis=0)[:, :, M2],))
    Ns = np.asarray(N, dtype=np.float64)

    def est(means):
        ln_chi = [np.log(n * np.interp(T_ref, T, m2)) for n, (m2,) in zip(Ns, means)]
        return np.polyfit(np.log(Ns), ln_chi, 1)[0]

    return _jackknife_sizes(est, per_size)


def _eta_curve(T, L, m2_means, r):
    """eta at every ladder temperature from the per-size mean |m|^2 curves."""
    Ls = np.asarray(L, dtype=np.float64)
    x = np.log(Ls)
    y = np.stack([np.log(l * l * m2) + 2.0 * r * np.log(np.log(l)) for l, m2 in zip(Ls, m2_means)])
    slope = np.polyfit(x, y, 1)[0]                 # one slope per temperature
    return 2.0 - slope


def eta_of_T(T, L, records, r=-1.0 / 16, discard=0.5):
    """eta(T) on a square L x L lattice (Sec. 4, the square-lattice limit,
    Eq. chi_SR): chi = N <|m|^2> ~ L^(2 - eta) (ln L)^(-2r) at each ladder
    temperature, fitted over the sizes (least squares of ln chi + 2r ln ln L
    against ln L).  r = -1/16 by default: the KT value in this form, chi ~
    L^(7/4) (ln L)^(1/8) at T_c (the paper prints the magnitude 1/16).  records: one [n_rec, G, n_T, 8] array per size
    in L.  Returns eta per temperature (sample means of <|m|^2>)."""
    m2 = []
    for rec in records:
        rec = np.asarray(rec, dtype=np.float64)
        rec = rec[int(rec.shape[0] * discard):]
        m2.append(rec.mean(axis=(0, 1))[:, M2])
    return _eta_curve(T, L, m2, r)


def t_eta(T, L, records, eta_target=0.25, r=-1.0 / 16, discard=0.5):
    """The temperature where eta(T) of eta_of_T reaches eta_target (the KT
    value 1/4 locates T_c, Sec. 4), by linear interpolation along the ladder,
    with a jackknife error over the samples of each size.  Returns (T, error);
    T is None when eta does not cross the target on the ladder."""
    T = np.asarray(T, dtype=np.float64)
    per_size = []
    for rec in records:
        rec = np.asarray(rec, dtype=np.float64)
        rec = rec[int(rec.shape[0] * discard):]
        per_size.append((rec.mean(axis=0)[:, :, M2],))

    def est(means):
        eta = _eta_curve(T, L, [m2 for (m2,) in means], r)
        return crossing(T, eta, np.full_like(eta, eta_target))

    t, err = _jackknife_sizes(est, per_size)
    return t, err


def compare_chains(a, b, n_bins=20, z_bar=3.0):
    """Statistical comparison of two independent sets of Markov chains on the
    same graphs and ladder (e.g. the fixed-point and the FP64 sweep), as the
    thermal averages of Sec. 3 would be compared:

      a, b : kept records [n_rec, G, n_T, n_obs] (the equilibration cut
             already applied), chain (s, k) of a and of b independent.

    Per (sample, temperature, observable): the difference of the two thermal
    averages over its error sigma = sqrt(sigma_a^2 + sigma_b^2), each sigma
    the jackknife (for a mean: batch-means) error over n_bins contiguous time
    bins.  Per (temperature, observable): the disorder-paired difference,
    d_s = <O>_a,s - <O>_b,s averaged over the samples, over its standard
    error from the sample-to-sample spread of d_s (valid whatever the
    autocorrelation inside a chain, since the samples are independent).
    Also the drift of each chain: first against second half of its kept
    records, in units of its error.

    Returns a dict with, for "per_sample", "disorder" and "drift", the number
    of comparisons, the fraction with |z| > z_bar, chi^2/dof = mean(z^2),
    max |z| and the outliers (index tuples and z)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape or a.ndim != 4:
        raise ValueError("a and b must both be [n_rec, G, n_T, n_obs]")
    ba, bb = bin_means(a, n_bins), bin_means(b, n_bins)
    ma, mb = ba.mean(axis=0), bb.mean(axis=0)
    ea = ba.std(axis=0, ddof=1) / np.sqrt(n_bins)
    eb = bb.std(axis=0, ddof=1) / np.sqrt(n_bins)
    with np.errstate(divide="ignore", invalid="ignore"):
        z_ps = (ma - mb) / np.hypot(ea, eb)
        d = ma - mb                                  # [G, n_T, n_obs]
        G = d.shape[0]
        z_dis = d.mean(axis=0) / (d.std(axis=0, ddof=1) / np.sqrt(G))
        h = a.shape[0] // 2
        drift = []
        for x in (a, b):
            q1, q2 = bin_means(x[:h], n_bins // 2), bin_means(x[h:2 * h], n_bins // 2)
            e1 = q1.std(axis=0, ddof=1) / np.sqrt(q1.shape[0])
            e2 = q2.std(axis=0, ddof=1) / np.sqrt(q2.shape[0])
            drift.append((q2.mean(axis=0) - q1.mean(axis=0)) / np.hypot(e1, e2))
        z_drift = np.stack(drift)                    # [2, G, n_T, n_obs]

    def summary(z, max_list=50):
        z = np.asarray(z)
        ok = np.isfinite(z)
        zf = z[ok]
        out_idx = np.argwhere(ok & (np.abs(np.where(ok, z, 0.0)) > z_bar))
        order = np.argsort(-np.abs(z[tuple(out_idx.T)])) if out_idx.size else []
        outliers = [(tuple(int(v) for v in out_idx[k]), float(z[tuple(out_idx[k])])) for k in order[:max_list]]
        return {"n": int(zf.size), "n_undefined": int((~ok).sum()),
                "frac_gt": float(np.mean(np.abs(zf) > z_bar)) if zf.size else 0.0,
                "chi2_dof": float(np.mean(zf ** 2)) if zf.size else 0.0,
                "max_abs": float(np.max(np.abs(zf))) if zf.size else 0.0,
                "mean": float(np.mean(zf)) if zf.size else 0.0, "outliers": outliers}

    dis = summary(z_dis)
    dis["mv"] = hotelling(d)
    return {"per_sample": summary(z_ps), "disorder": dis, "drift": summary(z_drift),
            "z_bar": z_bar, "n_bins": n_bins, "records": int(a.shape[0]),
            "z_per_sample": z_ps, "z_disorder": z_dis, "abs_diff_disorder": np.abs(d.mean(axis=0)),
            "mean_a": ma, "mean_b": mb}


def hotelling(a, b=None, alpha=1e-3):
    """Multivariate test, per temperature, that a mean difference of the
    observables is zero, for observables that move together (E, |m|^2 and
    |m|^4 of one temperature are strongly correlated, so their z-scores are
    not independent and a chi^2 of them is not chi^2-distributed).

      a [n, n_T, p]: paired differences, one row per independent unit (e.g.
                     the samples of a disorder-paired comparison); or, with
      b [n_b, n_T, p]: two independent sets of per-unit means compared
                     unpaired (e.g. independent chains of each precision).

    Per temperature, T^2 = d^T S^-1 d with d the mean difference and S its
    covariance (paired: the sample covariance of the rows / n; unpaired: the
    sum of the two sets' sample covariances over their sizes), on the
    eigen-directions of S above 1e-12 of its largest eigenvalue (p_eff of
    them).  Under the null, (nu - p_eff + 1) T^2 / (p_eff nu) is F(p_eff,
    nu - p_eff + 1) with nu = n - 1 (Hotelling; unpaired: nu = min(n, n_b) - 1,
    a conservative choice for unequal covariances).  Returns dict with T2,
    p_eff and pval per temperature, min_p, and chi2_dof = sum T^2 / sum
    p_eff with its bar: the larger of 1.5 and the 1 - alpha quantile of
    c chi^2_k / k, k = sum p_eff, c = nu / (nu - p - 1) the mean of T^2 / p."""
    from scipy import stats
    a = np.asarray(a, dtype=np.float64)
    if b is None:
        n = a.shape[0]
        d = a.mean(axis=0)
        S = np.einsum("gti,gtj->tij", a - d, a - d) / (n - 1) / n
        nu = n - 1
    else:
        b = np.asarray(b, dtype=np.float64)
        na, nb = a.shape[0], b.shape[0]
        ma, mb = a.mean(axis=0), b.mean(axis=0)
        d = ma - mb
        S = (np.einsum("gti,gtj->tij", a - ma, a - ma) / (na - 1) / na
             + np.einsum("gti,gtj->tij", b - mb, b - mb) / (nb - 1) / nb)
        nu = min(na, nb) - 1
    n_T, p = d.shape
    T2 = np.empty(n_T)
    p_eff = np.empty(n_T, dtype=np.int64)
    pval = np.empty(n_T)
    for t in range(n_T):
        w, V = np.linalg.eigh(S[t])
        keep = w > 1e-12 * max(w.max(), 1e-300)
        y = V[:, keep].T @ d[t]
        k = int(keep.sum())
        T2[t] = float(np.sum(y * y / w[keep])) if k else 0.0
        p_eff[t] = k
        if k == 0 or nu - k + 1 <= 0:
            pval[t] = np.nan
        else:
            pval[t] = float(stats.f.sf((nu - k + 1) * T2[t] / (k * nu), k, nu - k + 1))
    k_tot = int(p_eff.sum())
    c = nu / (nu - p - 1) if nu - p - 1 > 0 else np.inf
    bar = max(1.5, float(c * stats.chi2.isf(alpha, k_tot) / k_tot)) if k_tot else np.inf
    return {"T2": T2.tolist(), "p_eff": p_eff.tolist(), "pval": pval.tolist(),
            "min_p": float(np.nanmin(pval)) if np.any(np.isfinite(pval)) else float("nan"),
            "chi2_dof": float(T2.sum() / max(k_tot, 1)), "chi2_dof_bar": bar, "nu": int(nu), "n_T": int(n_T)}


def hotelling_ok(mv, alpha=1e-3):
    """hotelling's bar: every temperature's p-value above alpha / n_T
    (family-wise over the temperatures) and chi2_dof below its bar."""
    pv = np.asarray(mv["pval"], dtype=np.float64)
    return bool(np.all(np.isfinite(pv)) and pv.min() >= alpha / mv["n_T"] and mv["chi2_dof"] <= mv["chi2_dof_bar"])


def familywise_z_bar(n, dof=np.inf, alpha=1e-3):
    """|z| that the largest of n independent null comparisons exceeds with
    probability alpha (Bonferroni; Student t with dof degrees of freedom
    when the errors are estimated from dof + 1 independent values)."""
    from scipy import stats
    p = alpha / (2 * n)
    return float(stats.norm.isf(p) if not np.isfinite(dof) else stats.t.isf(p, dof))


def chi2_dof_bar(n, dof=np.inf, alpha=1e-3, floor=1.5):
    """Bar on chi^2/dof = mean(z^2) of n comparisons: the larger of `floor`
    (the fixed bar used for many comparisons) and the value the mean of n
    independent squared null z exceeds with probability alpha (the chi^2_n / n
    quantile, times the variance dof / (dof - 2) of a Student t).  For a few
    tens of comparisons a fixed 1.5 is not a 3-sigma test: chi^2_20 / 20
    exceeds it with probability 0.07 even for normal z."""
    from scipy import stats
    var = dof / (dof - 2.0) if np.isfinite(dof) and dof > 2 else 1.0
    return max(floor, float(stats.chi2.isf(alpha, n) / n * var))


def comparison_ok(summary, kind, dof=np.inf, frac=0.01, alpha=1e-3):
    """The bar on one set of comparisons (a summary of compare_chains).
    kind "many" (per (sample, temperature) comparisons, thousands): at most
    `frac` of them beyond 3 sigma and chi^2/dof at most 1.5.  kind "few"
    (disorder-paired ones, tens): the largest |z| below familywise_z_bar,
    with the errors' degrees of freedom, and, when the summary carries the
    multivariate test of the observables of each temperature ("mv", from
    hotelling), hotelling_ok; else chi^2/dof below chi2_dof_bar."""
    n = summary["n"]
    if summary.get("n_undefined", 0) or n == 0:
        return False
    if kind == "many":
        return summary["frac_gt"] <= frac and summary["chi2_dof"] <= 1.5
    if summary["max_abs"] > familywise_z_bar(n, dof, alpha):
        return False
    if "mv" in summary:                      # correlated observables: the per-temperature multivariate test
        return hotelling_ok(summary["mv"], alpha)
    return summary["chi2_dof"] <= chi2_dof_bar(n, dof, alpha)


# ---------------------------------------------------------------------------
# App. C: joint finite-size-scaling fits
# ---------------------------------------------------------------------------
def _u4_target_temps(T, means, u_targets):
    """T_f(U4_j, N) and dU4/dT there for every size (rows) and target
    (columns) from per-size mean curves ((m4, m2sq) pairs); None if a curve
    misses a target."""
    tf = np.empty((len(means), len(u_targets)))
    sl = np.empty_like(tf)
    for a, (m4, m2sq) in enumerate(means):
        U = m4 / m2sq - 1.0
        for j, u in enumerate(u_targets):
            hit = u4_slope_at(T, U, u)
            if hit is None:
                return None, None
            tf[a, j], sl[a, j] = hit
    return tf, sl


def tf_joint_fit(Tf, N, common_x=True, x_fixed=None):
    """Simultaneous fit of T_f(U4_j, N) = T_c + A_j N^(-x_j) (App. C, Eq.
    Tfsscaling) over n_d data sets j (columns of Tf, rows = sizes N): common
    T_c, set-dependent amplitudes A_j, and exponents x_j common to all sets
    (common_x, the paper's choice for rho < 3.75) or one per set; x_fixed
    fixes a common exponent (the fit is then linear).  Returns dict(T_c, A,
    x)."""
    from scipy.optimize import least_squares
    Tf = np.asarray(Tf, dtype=np.float64)
    lnN = np.log(np.asarray(N, dtype=np.float64))
    n_sz, n_d = Tf.shape

    def design(x):
        # columns: T_c, then one amplitude per set
        A = np.zeros((n_sz * n_d, 1 + n_d))
        A[:, 0] = 1.0
        for j in range(n_d):
            A[j::n_d, 1 + j] = np.exp(-np.broadcast_to(x, (n_d,))[j] * lnN)
        return A

    y = Tf.ravel()                                   # size-major: row a, set j -> a * n_d + j
    if x_fixed is not None:
        coef = np.linalg.lstsq(design(float(x_fixed)), y, rcond=None)[0]
        return {"T_c": float(coef[0]), "A": coef[1:].tolist(), "x": [float(x_fixed)] * n_d}
    n_x = 1 if common_x else n_d

    def resid(p):
        x = np.full(n_d, p[0]) if common_x else p[:n_d]
        coef = np.linalg.lstsq(design(x), y, rcond=None)[0]   # T_c and A_j are linear given x
        return design(x) @ coef - y

    fit = least_squares(resid, np.full(n_x, 0.5), bounds=(1e-3, 10.0), xtol=1e-14, ftol=1e-14, gtol=1e-14)
    x = np.full(n_d, fit.x[0]) if common_x else fit.x
    coef = np.linalg.lstsq(design(x), y, rcond=None)[0]
    return {"T_c": float(coef[0]), "A": coef[1:].tolist(), "x": [float(v) for v in x]}


def tc_from_u4_sets(T, N, records, u_targets, common_x=True, x_fixed=None, discard=0.5):
    """T_c by the joint fit of Eq. Tfsscaling (App. C) on the temperatures
    where the disorder-averaged U4 (ratio of averages) of each size reaches
    each value of u_targets; records: one [n_rec, G, n_T, 8] array per size
    N.  Returns dict(T_c, T_c_error, x, x_error, T_f), errors by a jackknife
    over the samples of every size."""
    per_size = [u4_samples(r, discard) for r in records]

    def fit(means):
        tf, _ = _u4_target_temps(T, means, u_targets)
        return None if tf is None else tf_joint_fit(tf, N, common_x, x_fixed)

    full = fit([(a.mean(0), b.mean(0)) for a, b in per_size])
    if full is None:
        raise ValueError("a U4 target lies outside some size's curve on the ladder")
    tc, tc_err = _jackknife_sizes(lambda m: (lambda f: None if f is None else f["T_c"])(fit(m)), per_size)
    x_err = None
    if x_fixed is None and common_x:
        _, x_err = _jackknife_sizes(lambda m: (lambda f: None if f is None else f["x"][0])(fit(m)), per_size)
    tf, _ = _u4_target_temps(T, [(a.mean(0), b.mean(0)) for a, b in per_size], u_targets)
    return {"T_c": full["T_c"], "T_c_error": tc_err, "x": full["x"], "x_error": x_err, "A": full["A"],
            "T_f": tf.tolist(), "u_targets": list(map(float, u_targets))}


def nu_bar_joint(T, N, records, u_targets, discard=0.5):
    """nu_bar from ln dU4/dT at fixed U4 = c_j + (1/nu_bar) ln N (App. C, Eq.
    scaling_lndotU4), fitted simultaneously over the sets U4_j with one
    intercept per set and a common slope.  Returns (nu_bar, jackknife error
    over the samples of every size)."""
    per_size = [u4_samples(r, discard) for r in records]
    lnN = np.log(np.asarray(N, dtype=np.float64))
    n_d = len(u_targets)

    def est(means):
        _, sl = _u4_target_temps(T, means, u_targets)
        if sl is None:
            return None
        y = np.log(np.abs(sl)).ravel()               # size-major
        A = np.zeros((y.size, 1 + n_d))
        A[:, 0] = np.repeat(lnN, n_d)
        for j in range(n_d):
            A[j::n_d, 1 + j] = 1.0
        inv_nu = np.linalg.lstsq(A, y, rcond=None)[0][0]
        return 1.0 / inv_nu

    return _jackknife_sizes(est, per_size)


def size_exponent_curve(T, N, records, kind, discard=0.5):
    """x(T) at every ladder temperature from the sizes' disorder-averaged
    <|m|^2>: kind "chi": ln chi = cte + x ln N with chi = N <|m|^2> (App. C,
    Eq. chiscaling; x(T_c) = gamma/nu_bar); kind "m": (1/2) ln <|m|^2> =
    cte - x ln N (Eq. mscaling; x(T_c) = beta/nu_bar).  Returns (x, error),
    arrays over the ladder, errors by a jackknife over the samples."""
    if kind not in ("chi", "m"):
        raise ValueError("kind is 'chi' or 'm'")
    Ns = np.asarray(N, dtype=np.float64)
    per_size = []
    for r in records:
        rec = np.asarray(r, dtype=np.float64)
        rec = rec[int(rec.shape[0] * discard):]
        per_size.append((rec.mean(axis=0)[:, :, M2],))

    def curve(means):
        if kind == "chi":
            y = np.stack([np.log(n * m2) for n, (m2,) in zip(Ns, means)])
            return np.polyfit(np.log(Ns), y, 1)[0]
        y = np.stack([0.5 * np.log(m2) for (m2,) in means])
        return -np.polyfit(np.log(Ns), y, 1)[0]

    x = curve([(m2.mean(0),) for (m2,) in per_size])
    err = np.array([_jackknife_sizes(lambda m, k=k: curve(m)[k], per_size)[1] for k in range(len(T))])
    return x, err


def beta_over_nu_bar(T, N, records, T_ref, discard=0.5):
    """beta / nu_bar = x(T_ref) of Eq. mscaling (App. C), x linearly
    interpolated along the ladder.  Returns (value, jackknife error)."""
    T = np.asarray(T, dtype=np.float64)
    Ns = np.asarray(N, dtype=np.float64)
    per_size = []
    for r in records:
        rec = np.asarray(r, dtype=np.float64)
        rec = rec[int(rec.shape[0] * discard):]
        per_size.append((rec.mean(axis=0)[:, :, M2],))

    def est(means):
        y = [0.5 * np.log(np.interp(T_ref, T, m2)) for (m2,) in means]
        return -np.polyfit(np.log(Ns), y, 1)[0]

    return _jackknife_sizes(est, per_size)
