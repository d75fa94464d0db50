"""Small statistics helpers for the tests (batch means, jackknife over
batches, and the bars the statistical GPU tests apply).  Test code only; the
product's own analysis lives in the package.

Bars:
* many comparisons (hundreds or more): at most 1% of |z| beyond 3 and
  chi^2/dof = mean(z^2) at most 1.5, every outlier listed (assert_r22);
* few comparisons (pooled means, disorder averages): the largest |z| below
  the quantile a family of that size exceeds with probability 1e-3 under the
  null (Bonferroni, Student t with the errors' degrees of freedom), and
  chi^2/dof below the larger of 1.5 and its own 1e-3 quantile for that many
  comparisons (assert_familywise; analysis.familywise_z_bar, chi2_dof_bar);
* few comparisons of correlated observables (E, |m|^2, |m|^4, F of one
  temperature move together): the family-wise bar on each z, and, per
  temperature, Hotelling's test of the vector of differences, family-wise
  over the temperatures (assert_pooled; analysis.hotelling).
"""
import numpy as np

from paper_1211_3991_amd.analysis import chi2_dof_bar, familywise_z_bar, hotelling, hotelling_ok


def batch_mean_err(x, n_batches=50):
    """Mean of x and its standard error from n_batches contiguous batches."""
    x = np.asarray(x, dtype=np.float64)
    nb = len(x) // n_batches
    b = x[: nb * n_batches].reshape(n_batches, nb).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(n_batches)


def batch_means_err_axis0(x, n_batches=50):
    """Means and standard errors along axis 0 from n_batches contiguous batches."""
    x = np.asarray(x, dtype=np.float64)
    nb = x.shape[0] // n_batches
    b = x[: nb * n_batches].reshape((n_batches, nb) + x.shape[1:]).mean(axis=1)
    return b.mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(n_batches)


def jackknife_fn(fn, series, n_batches=50):
    """Jackknife estimate and error of fn(*batch means) over contiguous batches.
    series: list of 1-d arrays of equal length."""
    arrs = [np.asarray(s, dtype=np.float64) for s in series]
    nb = len(arrs[0]) // n_batches
    bm = [a[: nb * n_batches].reshape(n_batches, nb).mean(axis=1) for a in arrs]
    tot = [b.mean() for b in bm]
    full = fn(*tot)
    loo = np.array([fn(*[(b.sum() - b[i]) / (n_batches - 1) for b in bm]) for i in range(n_batches)])
    err = np.sqrt((n_batches - 1) / n_batches * np.sum((loo - loo.mean()) ** 2))
    return full, err


def _outliers(z, bar, labels=None, limit=30):
    z = np.asarray(z, dtype=np.float64)
    idx = np.argwhere(np.abs(z) > bar)
    order = np.argsort(-np.abs(z[tuple(idx.T)])) if idx.size else []
    out = []
    for k in order[:limit]:
        i = tuple(int(v) for v in idx[k])
        out.append((labels[i] if labels is not None else i, round(float(z[i]), 2)))
    return out


def assert_r22(z, what=""):
    """At most 1% of the |z| beyond 3 and chi^2/dof at most 1.5."""
    z = np.asarray(z, dtype=np.float64)
    assert np.all(np.isfinite(z)), f"{what}: undefined z"
    frac, chi2 = float(np.mean(np.abs(z) > 3)), float(np.mean(z ** 2))
    msg = f"{what}: n={z.size} frac|z|>3={frac:.4f} chi2/dof={chi2:.3f} outliers={_outliers(z, 3.0)}"
    print(msg, flush=True)
    assert frac <= 0.01 and chi2 <= 1.5, msg


def familywise_bar(n, dof=np.inf, alpha=1e-3):
    """|z| that one of n independent null comparisons exceeds with probability alpha."""
    return familywise_z_bar(n, dof, alpha)


def assert_familywise(z, what="", dof=np.inf, alpha=1e-3):
    z = np.asarray(z, dtype=np.float64)
    assert np.all(np.isfinite(z)), f"{what}: undefined z"
    bar = familywise_bar(z.size, dof, alpha)
    chi2, chi2_bar = float(np.mean(z ** 2)), chi2_dof_bar(z.size, dof, alpha)
    msg = f"{what}: n={z.size} max|z|={np.max(np.abs(z)):.2f} (bar {bar:.2f}) chi2/dof={chi2:.3f} " \
          f"(bar {chi2_bar:.2f}) beyond 3: {_outliers(z, 3.0)}"
    print(msg, flush=True)
    assert np.max(np.abs(z)) <= bar, msg
    assert chi2 <= chi2_bar, msg


def assert_pooled(a, b=None, what="", alpha=1e-3):
    """a [n, n_T, p]: paired differences of n independent units; or a, b:
    two independent sets of per-unit means.  Each (temperature, observable)
    z below the family-wise bar, and Hotelling's per-temperature test."""
    a = np.asarray(a, dtype=np.float64)
    if b is None:
        n, d = a.shape[0], a.mean(axis=0)
        se = a.std(axis=0, ddof=1) / np.sqrt(n)
    else:
        b = np.asarray(b, dtype=np.float64)
        n = min(a.shape[0], b.shape[0])
        d = a.mean(axis=0) - b.mean(axis=0)
        se = np.hypot(a.std(axis=0, ddof=1) / np.sqrt(a.shape[0]), b.std(axis=0, ddof=1) / np.sqrt(b.shape[0]))
    z = d / se
    assert np.all(np.isfinite(z)), f"{what}: undefined z"
    bar = familywise_bar(z.size, n - 1, alpha)
    mv = hotelling(a, b, alpha)
    pv = np.round(mv["pval"], 5).tolist()
    msg = (f"{what}: n={z.size} max|z|={np.max(np.abs(z)):.2f} (bar {bar:.2f}) beyond 3: {_outliers(z, 3.0)}; "
           f"Hotelling per T: p={pv} (bar {alpha / mv['n_T']:.1e}), chi2/dof={mv['chi2_dof']:.3f} "
           f"(bar {mv['chi2_dof_bar']:.2f})")
    print(msg, flush=True)
    assert np.max(np.abs(z)) <= bar, msg
    assert hotelling_ok(mv, alpha), msg
