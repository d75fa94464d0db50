"""Fixed-point sweep against the FP64 sweep at a workload's full shape.

Both precisions run the method (App. B: Metropolis + over-relaxation sweeps
with parallel tempering every sweep) on the same graphs and temperature
ladder from the ordered start (or the random one), for the same number of sweeps
and the same measurement cadence; their records of E, |m|^2, |m|^4, F_x and
F_y (Sec. 3) are then compared with ``analysis.compare_chains``: per (sample,
temperature) with jackknife errors over time bins, and disorder-paired per
temperature.  The two chains of a sample use independent Philox keys (the
FP64 key is the sample seed plus 2^32), so their difference has the variance
of two independent chains.

The FP64 sweep is the path whose decisions equal the oracle's bit for bit;
this comparison is what ties the fixed-point form to it at sizes the oracle
cannot run.  Run as ``python -m paper_1211_3991_amd.parity --workload W``.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import Batch, Graph, analysis

OBS = (analysis.E, analysis.M2, analysis.M4, analysis.FX, analysis.FY)
OBS_NAMES = ("E", "m2", "m4", "Fx", "Fy")
FP64_KEY_OFFSET = 1 << 32


def build_graphs(samples, threads=None):
    """Graphs of the workload's samples, built on host threads (the library's
    graph calls release the interpreter lock)."""
    threads = threads or min(16, len(os.sched_getaffinity(0)))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda s: Graph.levy(s.L, s.z, s.rho, s.seed), samples))


def cold_state(graphs, n_T, precision):
    """Every spin along x (angle 0) in every slot: the ordered start."""
    if precision == "fp64":
        out = []
        for g in graphs:
            a = np.zeros((n_T, g.n, 2))
            a[:, :, 0] = 1.0
            out.append(a)
        return out
    return [np.zeros((n_T, g.n), np.uint16) for g in graphs]


def run_records(graphs, T, precision, seeds, n_sweeps, meas_every, n_or=5, pt_every=1, tune=False, chunk=0,
                start="cold"):
    """Records [n_rec, G, n_T, 8] of n_sweeps sweeps from the ordered start
    (start="cold") or the library's random start ("random")."""
    import torch
    stream = torch.cuda.Stream()
    b = Batch(graphs, T, precision=precision, seeds=seeds, max_records=n_sweeps // meas_every, stream=stream)
    try:
        if start == "cold":
            b.set_state(cold_state(graphs, np.shape(T)[-1], precision), sweep=0)
        if tune and precision == "fix16":
            b.autotune(sweeps=1, n_or=n_or, use_cache=False, pt_every=pt_every)
        if chunk:
            b.use_graph(chunk)
        b.sweep(n_sweeps, n_or=n_or, pt_every=pt_every, meas_every=meas_every)
        b.synchronize()
        return b.records().cpu().numpy()
    finally:
        b.close()
        torch.cuda.empty_cache()


def compare(rec16, rec64, n_bins=20, keep=0.5):
    """compare_chains on the kept records (the last `keep` fraction) of the
    five observables; adds per-observable summaries and the disorder-averaged
    deviation of each (temperature, observable) with its error."""
    n = rec16.shape[0]
    k0 = n - int(round(n * keep))
    a = rec16[k0:, :, :, list(OBS)]
    b = rec64[k0:, :, :, list(OBS)]
    res = analysis.compare_chains(a, b, n_bins=n_bins)
    zs, zd = res["z_per_sample"], res["z_disorder"]
    per_obs = {}
    for q, name in enumerate(OBS_NAMES):
        z = zs[..., q][np.isfinite(zs[..., q])]
        per_obs[name] = {"frac_gt3": float(np.mean(np.abs(z) > 3)), "chi2_dof": float(np.mean(z ** 2)),
                         "max_abs_z": float(np.max(np.abs(z))),
                         "disorder_max_abs_z": float(np.nanmax(np.abs(zd[:, q])))}
    # disorder-averaged fix16 - FP64 per (temperature, observable), relative to the FP64 value
    ma, mb = res["mean_a"], res["mean_b"]
    d = ma - mb
    G = d.shape[0]
    rel = np.abs(d.mean(axis=0)) / np.maximum(np.abs(mb.mean(axis=0)), 1e-300)
    rel_err = d.std(axis=0, ddof=1) / np.sqrt(G) / np.maximum(np.abs(mb.mean(axis=0)), 1e-300)
    out = {k: res[k] for k in ("per_sample", "disorder", "drift", "z_bar", "n_bins", "records")}
    out["per_observable"] = per_obs
    out["max_rel_dev_disorder"] = {name: float(rel[:, q].max()) for q, name in enumerate(OBS_NAMES)}
    out["rel_err_disorder"] = {name: float(rel_err[:, q].max()) for q, name in enumerate(OBS_NAMES)}
    return out


def fix16_vs_fp64(wl, n_sweeps, meas_every=4, n_bins=20, keep=0.5, graphs=None, chunk=32, tune=True, start="cold"):
    """Runs both precisions on workload wl and compares them; returns the
    summary (JSON-able) and the two record arrays.

    start="cold": both from the ordered state, so that the low-temperature
    chains do not freeze into the twisted (winding) states a random start
    leaves on the torus, which relax only through vortex pairs and would make
    one chain's window differ from another's by far more than its own
    fluctuations; "random": the library's random start."""
    graphs = graphs if graphs is not None else build_graphs(wl.samples)
    seeds16 = np.array([s.seed for s in wl.samples], np.uint64)
    t0 = time.perf_counter()
    rec16 = run_records(graphs, wl.T, "fix16", seeds16, n_sweeps, meas_every, wl.n_or, wl.pt_every, tune=tune,
                        chunk=chunk if chunk % meas_every == 0 else 0, start=start)
    t1 = time.perf_counter()
    rec64 = run_records(graphs, wl.T, "fp64", seeds16 + np.uint64(FP64_KEY_OFFSET), n_sweeps, meas_every, wl.n_or,
                        wl.pt_every, start=start)
    t2 = time.perf_counter()
    out = compare(rec16, rec64, n_bins=n_bins, keep=keep)
    out.update(workload=wl.name, sweeps=n_sweeps, meas_every=meas_every, keep=keep, start=start,
               fix16_s=round(t1 - t0, 2), fp64_s=round(t2 - t1, 2),
               fp64_key="sample seed + 2^32", fix16_key="sample seed")
    return out, rec16, rec64


def r22_ok(summary, n_samples):
    """The bar (analysis.comparison_ok): per (sample, temperature), at most 1%
    of the comparisons beyond 3 sigma and chi^2/dof at most 1.5;
    disorder-paired, the family-wise bar with n_samples - 1 degrees of
    freedom."""
    return (analysis.comparison_ok(summary["per_sample"], "many")
            and analysis.comparison_ok(summary["disorder"], "few", dof=n_samples - 1))


def main(argv=None):
    import workloads
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="headline_l256", choices=sorted(workloads.ALL))
    ap.add_argument("--sweeps", type=int, default=2048)
    ap.add_argument("--meas-every", type=int, default=4)
    ap.add_argument("--bins", type=int, default=20)
    ap.add_argument("--start", choices=["cold", "random"], default="cold")
    ap.add_argument("--out", help="write the summary JSON here")
    args = ap.parse_args(argv)
    wl = workloads.ALL[args.workload]()
    out, _, _ = fix16_vs_fp64(wl, args.sweeps, args.meas_every, args.bins, start=args.start)
    out["r22_ok"] = r22_ok(out, len(wl.samples))
    text = json.dumps(out, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    print(text)
    return 0 if out["r22_ok"] else 1


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    sys.exit(main())
