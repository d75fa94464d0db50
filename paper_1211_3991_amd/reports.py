"""Graph reports of the paper's Sec. 2 and App. B, from the library's graphs.

* degree distributions (Sec. 2, Fig. 1): P(k) of dilute graphs with
  N = 256^2 sites and z = 4, for rho = 1/2, 10/3 and 14/3 (one per critical
  regime), with periodic and free boundaries, beside the Poisson law of mean
  4 (the rho = 0 limit);
* colour classes (App. B, Fig. 15): the fractions of the sites in each colour
  class of the smallest-last colouring of rho = 1, z = 4 graphs with
  N = 2^8 ... 2^14 sites, and how far they are from equal.

    python -m paper_1211_3991_amd.reports degrees      # one JSON document
    python -m paper_1211_3991_amd.reports colours
"""
import argparse
import json
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import Graph, analysis


def _graphs(specs, threads=None):
    threads = threads or min(16, len(os.sched_getaffinity(0)))
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda a: Graph.levy(*a[:4], boundary=a[4]), specs))


def degree_report(L=256, z=4, rhos=(0.5, 10 / 3, 14 / 3), samples=4, seed0=0):
    """P(k) averaged over `samples` graphs per (rho, boundary), with its
    standard error over the graphs, and the Poisson(z) law."""
    out = {"L": L, "N": L * L, "z": z, "samples": samples, "curves": []}
    kmax = 0
    for rho in rhos:
        for boundary in ("periodic", "free"):
            gs = _graphs([(L, z, rho, seed0 + s, boundary) for s in range(samples)])
            ps = [analysis.degree_distribution(g.export()["edges"], g.n) for g in gs]
            k = max(p.size for p in ps)
            kmax = max(kmax, k)
            P = np.zeros((samples, k))
            for a, p in enumerate(ps):
                P[a, :p.size] = p
            mean = P.mean(axis=0)
            ks = np.arange(k)
            out["curves"].append({
                "rho": rho, "boundary": boundary, "P": mean.tolist(),
                "P_err": (P.std(axis=0, ddof=1) / math.sqrt(samples)).tolist() if samples > 1 else None,
                "mean_degree": float(np.sum(ks * mean)), "var_degree": float(np.sum(ks * ks * mean) - np.sum(ks * mean) ** 2),
                "P_at_z": float(mean[z]) if z < k else 0.0, "max_degree": int(k - 1)})
    ks = np.arange(kmax)
    out["poisson"] = [float(math.exp(-z) * z ** int(k) / math.factorial(int(k))) for k in ks]
    return out


def colour_report(rho=1.0, z=4, exps=range(8, 15), samples=8, seed0=0):
    """Colour-class fractions (sorted, largest first) of the smallest-last
    colouring per size N = 2^e (square lattices need even e; odd e use the
    nearest even-sided L with L^2 closest to 2^e), averaged over `samples`
    graphs, with the spread (largest minus smallest fraction) and the
    coefficient of variation of the class sizes."""
    out = {"rho": rho, "z": z, "samples": samples, "sizes": []}
    for e in exps:
        L = int(round(math.sqrt(2 ** e)))
        L += L % 2
        gs = _graphs([(L, z, rho, seed0 + s, "periodic") for s in range(samples)])
        fr = [np.sort(analysis.colour_fractions(g.export()["colour"]))[::-1] for g in gs]
        q = max(f.size for f in fr)
        F = np.zeros((samples, q))
        for a, f in enumerate(fr):
            F[a, :f.size] = f
        spread = [float(f[0] - f[-1]) for f in fr]
        cv = [float(f.std() / f.mean()) for f in fr]
        out["sizes"].append({"log2_N_target": e, "L": L, "N": L * L,
                             "colours": sorted({int(f.size) for f in fr}),
                             "fractions": F.mean(axis=0).tolist(),
                             "spread": float(np.mean(spread)), "spread_err": float(np.std(spread, ddof=1) / math.sqrt(samples)),
                             "cv": float(np.mean(cv))})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("what", choices=["degrees", "colours"])
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--out")
    args = ap.parse_args(argv)
    if args.what == "degrees":
        rep = degree_report(samples=args.samples or 4)
    else:
        rep = colour_report(samples=args.samples or 8)
    text = json.dumps(rep, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
