"""Fixed-point sweep against the FP64 sweep at the batched workload shapes
(through the C ABI): 64 samples of L=256 (rho=3.5, 24 temperatures in
[1.0, 2.5]), 32 samples of L=512 (rho=2.5, 16 temperatures in [1.5, 3.5]),
64 samples of L=128 (rho=3.5, 16 temperatures in [1.0, 2.5]) and the 128
uneven samples (L = 32, 64, 128, 256; rho = 2.5, 3.5, 4.5; 32 temperatures in
[0.8, 3.0]; the smaller graphs in the workgroup form, the larger in the phase
form), z = 6, parallel tempering every sweep (App. B), in the launch
configuration the benchmark uses (autotuned form and stream groups, HIP-graph
replay).

Both precisions sweep the same graphs from the ordered start with
independent random keys for the same number of sweeps, measuring E, |m|^2,
|m|^4, F_x, F_y (Sec. 3) every 4 sweeps; the second half of the records is
kept (the last time window, Sec. 4).  A time bin must span several
integrated autocorrelation times for the jackknife errors to hold: at L=512
that time reaches 25-35 sweeps for E and |m|^2 in the slowest chains (median
3.5, 90th percentile 7), so that case runs 4096 sweeps (bins of 102 sweeps;
at 2048, bins of 51 sweeps, a few such chains give too small errors).  The FP64 sweep is the path whose decisions equal the
oracle's bit for bit (tests/test_gpu_fp64_parity.py, also at this L=256
shape), so this ties the fixed-point form, at its real shape, to the oracle's
observables.  The bar: per (sample, temperature, observable) with jackknife
errors over 20 time bins (thousands of comparisons), at most 1% beyond 3
sigma and chi^2/dof at most 1.5; disorder-paired per (temperature,
observable) (tens of comparisons, errors from the sample-to-sample spread),
the largest |z| below the 1e-3 family-wise bar and, per temperature,
Hotelling's test of the five observables together at the family-wise 1e-3
(analysis.comparison_ok); every outlier is printed.  The two chains of a sample follow the same law from the
same initial law, so their windows compare even where a chain is still
relaxing; the first-against-second-quarter drift of the kept records is
printed as the equilibration check.

The L=256 case runs the phase kernel with 24 slots per site (six threads per
site, 42 sites per block); the L=512 case runs its int32-index
instantiation with 4096-site degree windows.
"""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1211_3991_amd import analysis, parity  # noqa: E402

SWEEPS = {"headline_l256": 2048, "large_l512": 4096, "batch_l128": 2048, "uneven_sizes": 1024}


def _report(out):
    for k in ("per_sample", "disorder", "drift"):
        s = out[k]
        print(f"{out['workload']} {k}: n={s['n']} frac|z|>3={s['frac_gt']:.4f} chi2/dof={s['chi2_dof']:.3f} "
              f"max|z|={s['max_abs']:.2f} outliers={s['outliers'][:20]}", flush=True)
    mv = out["disorder"].get("mv")
    if mv:
        print(f"{out['workload']} disorder Hotelling: min p={mv['min_p']:.4g} (bar {1e-3 / mv['n_T']:.2g}) "
              f"chi2/dof={mv['chi2_dof']:.3f} (bar {mv['chi2_dof_bar']:.2f})", flush=True)
    print(json.dumps(out["per_observable"]), flush=True)
    print(json.dumps({"max_rel_dev_disorder": out["max_rel_dev_disorder"],
                      "rel_err_disorder": out["rel_err_disorder"]}), flush=True)
    path = os.environ.get("XY_PARITY_OUT")
    if path:
        with open(os.path.join(path, f"parity_{out['workload']}.json"), "w") as fh:
            json.dump(out, fh, indent=1)


@pytest.mark.parametrize("name", ["headline_l256", "large_l512", "batch_l128", "uneven_sizes"])
def test_fix16_matches_fp64_at_full_shape(name):
    wl = workloads.ALL[name]()
    out, rec16, rec64 = parity.fix16_vs_fp64(wl, SWEEPS[name], meas_every=4, n_bins=20)
    _report(out)
    n_rec = SWEEPS[name] // 4
    assert rec16.shape == rec64.shape == (n_rec, len(wl.samples), wl.n_T, 8)
    assert np.all(np.isfinite(rec16)) and np.all(np.isfinite(rec64))
    G = len(wl.samples)
    for k, kind in (("per_sample", "many"), ("disorder", "few")):
        s = out[k]
        assert s["n_undefined"] == 0, (k, s)
        assert analysis.comparison_ok(s, kind, dof=G - 1), (k, s["frac_gt"], s["chi2_dof"], s["max_abs"],
                                                             s["outliers"])
