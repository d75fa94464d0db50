"""Finite-size-scaling run of the paper's method on one family of graphs
(Sec. 4 and App. C): equilibrium sweeps with parallel tempering on the GPU
path for several sizes, then the critical temperature from the crossings of
U4(T, N) with U4(T, N/4) extrapolated with T(N) = C N^(-1/nu_bar) + T_c, nu_bar
from dU4/dT at fixed U4 (Eq. U4dot), and gamma/nu_bar from chi at a
reference temperature.

    python -m paper_1211_3991_amd.fss --rho 0 --z 4            # one JSON line
"""
import argparse
import json
from fractions import Fraction

import numpy as np

from . import analysis


def run(rho, z=4, sizes=(16, 32, 64, 128), samples=64, T=(1.7, 2.2, 16), sweeps=1 << 14, meas_every=16,
        seed_base=10_000, nu_bar=2.0, T_ref=None, boundary="periodic", log=None):
    """Runs the sweeps and returns the FSS estimates as a dict.

    T: (first, last, count) of a linear temperature ladder.  Graph and dynamics
    seeds of sample s at size L are seed_base * L + s.  nu_bar is the exponent
    assumed in the T_c extrapolation; T_ref (default: the extrapolated T_c) is
    where gamma/nu_bar is taken."""
    import torch

    import paper_1211_3991_amd as xy
    ladder = np.linspace(T[0], T[1], int(T[2]))
    rec = {}
    for L in sizes:
        if log:
            log(f"rho={rho} z={z} L={L}: {samples} samples, {sweeps} sweeps")
        seeds = [seed_base * L + s for s in range(samples)]
        graphs = [xy.Graph.levy(L, z, rho, sd, boundary=boundary) for sd in seeds]
        b = xy.Batch(graphs, ladder, precision="fix16", seeds=seeds, max_records=sweeps // meas_every)
        b.sweep(sweeps, n_or=5, pt_every=1, meas_every=meas_every)
        torch.cuda.synchronize()
        rec[L] = b.records().cpu().numpy()
        b.close()
    N, Tx, err = [], [], []
    for a, b_ in zip(sizes[:-1], sizes[1:]):
        t, e = analysis.u4_crossing(ladder, rec[a], rec[b_])
        if t is None:
            raise RuntimeError(f"U4 of L={a} and L={b_} do not cross on the ladder")
        N.append(b_ * b_)
        Tx.append(t)
        err.append(e)
    tc, c = analysis.fss_tc(N, Tx, nu_bar)
    # standard error of T_c: the least-squares fit is linear in the crossings
    x = np.asarray(N, float) ** (-1.0 / nu_bar)
    w = np.linalg.pinv(np.stack([np.ones_like(x), x], axis=1))[0]
    tc_err = float(np.sqrt(np.sum((w * np.asarray(err)) ** 2)))
    m4, m2sq = analysis.u4_samples(rec[sizes[-2]])
    u_star = float(np.interp(Tx[-1], ladder, m4.mean(0) / m2sq.mean(0) - 1.0))
    Ns = [L * L for L in sizes]
    nu, nu_err = analysis.nu_bar_from_u4(ladder, Ns, [rec[L] for L in sizes], u_star)
    t_ref = tc if T_ref is None else T_ref
    g, g_err = analysis.gamma_over_nu_bar(ladder, Ns, [rec[L] for L in sizes], t_ref)
    return {"rho": rho, "z": z, "boundary": boundary, "sizes": list(sizes), "samples": samples,
            "crossings": [float(v) for v in Tx], "crossing_errors": [float(v) for v in err],
            "T_c": float(tc), "T_c_error": tc_err, "C": float(c), "nu_bar_assumed": nu_bar,
            "U4_star": u_star, "nu_bar": float(nu), "nu_bar_error": float(nu_err),
            "T_ref": float(t_ref), "gamma_over_nu_bar": float(g), "gamma_over_nu_bar_error": float(g_err),
            "records": rec}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--rho", type=lambda v: float(Fraction(v)), default=0.0, help="e.g. 0, 7/3, 3.5")
    ap.add_argument("--z", type=int, default=4)
    ap.add_argument("--sizes", type=int, nargs="+", default=[16, 32, 64, 128])
    ap.add_argument("--samples", type=int, default=64)
    ap.add_argument("--T", type=float, nargs=3, default=[1.7, 2.2, 16], metavar=("FIRST", "LAST", "COUNT"))
    ap.add_argument("--sweeps", type=int, default=1 << 14)
    ap.add_argument("--boundary", choices=["periodic", "free"], default="periodic")
    ap.add_argument("--nu-bar", type=float, default=2.0, help="exponent assumed in the T_c extrapolation")
    args = ap.parse_args()
    out = run(args.rho, args.z, tuple(args.sizes), args.samples, tuple(args.T), args.sweeps, nu_bar=args.nu_bar,
              boundary=args.boundary, log=lambda m: print("#", m, flush=True))
    out.pop("records")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
