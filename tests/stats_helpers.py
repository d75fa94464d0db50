"""Small statistics helpers for the tests (batch means and jackknife over
batches).  Test code only; the product's own analysis lives in the package."""
import numpy as np


def batch_mean_err(x, n_batches=50):
    """Mean of x and its standard error from n_batches contiguous batches."""
    x = np.asarray(x, dtype=np.float64)
    nb = len(x) // n_batches
    b = x[: nb * n_batches].reshape(n_batches, nb).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(n_batches)


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
