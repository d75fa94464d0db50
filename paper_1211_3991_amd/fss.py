"""Finite-size-scaling run of the paper's method on one family of graphs
(Sec. 4 and App. C): equilibrium sweeps with parallel tempering on the GPU
path for several sizes, then the critical temperature from the crossings of
U4(T, N) with U4(T, N/4) extrapolated with T(N) = C N^(-1/nu_bar) + T_c, nu_bar
from dU4/dT at fixed U4 (Eq. U4dot), and gamma/nu_bar from chi at a
reference temperature; then the joint fits of App. C (T_c from Eq.
Tfsscaling over several U4 values, nu_bar from Eq. scaling_lndotU4 with a
common slope, beta/nu_bar from Eq. mscaling).

    python -m paper_1211_3991_amd.fss --rho 0 --z 4            # one JSON line
"""
import argparse
import json
from fractions import Fraction

import numpy as np

from . import analysis


def _sweep_records(graphs, ladder, seeds, sweeps, meas_every, chunk):
    """Records of `sweeps` sweeps (1 Metropolis + 5 OR, PT every sweep) of the
    fixed-point path, the sweeps replayed from a HIP graph of `chunk` sweeps
    (a multiple of meas_every; 0: direct launches)."""
    import torch

    import paper_1211_3991_amd as xy
    stream = torch.cuda.Stream()
    b = xy.Batch(graphs, ladder, precision="fix16", seeds=seeds, max_records=sweeps // meas_every, stream=stream)
    try:
        if chunk:
            b.use_graph(chunk)
        b.sweep(sweeps, n_or=5, pt_every=1, meas_every=meas_every)
        b.synchronize()
        return b.records().cpu().numpy()
    finally:
        b.close()


def run(rho, z=4, sizes=(16, 32, 64, 128), samples=64, T=(1.7, 2.2, 16), sweeps=1 << 14, meas_every=16,
        seed_base=10_000, nu_bar=2.0, T_ref=None, boundary="periodic", log=None, chunk=256):
    """Runs the sweeps and returns the FSS estimates as a dict.

    T: (first, last, count) of a linear temperature ladder.  Graph and dynamics
    seeds of sample s at size L are seed_base * L + s.  nu_bar is the exponent
    assumed in the T_c extrapolation; T_ref (default: the extrapolated T_c) is
    where gamma/nu_bar is taken.  chunk: sweeps per HIP-graph replay (a
    multiple of meas_every; 0 for direct launches)."""
    import paper_1211_3991_amd as xy
    ladder = np.linspace(T[0], T[1], int(T[2]))
    rec = {}
    for L in sizes:
        if log:
            log(f"rho={rho} z={z} L={L}: {samples} samples, {sweeps} sweeps")
        seeds = [seed_base * L + s for s in range(samples)]
        graphs = [xy.Graph.levy(L, z, rho, sd, boundary=boundary) for sd in seeds]
        rec[L] = _sweep_records(graphs, ladder, seeds, sweeps, meas_every, chunk)
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
    recs = [rec[L] for L in sizes]
    g, g_err = analysis.gamma_over_nu_bar(ladder, Ns, recs, t_ref)
    out = {"rho": rho, "z": z, "boundary": boundary, "sizes": list(sizes), "samples": samples,
           "crossings": [float(v) for v in Tx], "crossing_errors": [float(v) for v in err],
           "T_c": float(tc), "T_c_error": tc_err, "C": float(c), "nu_bar_assumed": nu_bar,
           "U4_star": u_star, "nu_bar": float(nu), "nu_bar_error": float(nu_err),
           "T_ref": float(t_ref), "gamma_over_nu_bar": float(g), "gamma_over_nu_bar_error": float(g_err)}
    out.update(app_c_fits(ladder, Ns, recs, u_star, rho, t_ref))
    out["records"] = rec
    return out


def u4_targets(T, records, u_center, n_d=3, span=0.6):
    """n_d values of U4 around u_center inside the range every size's
    disorder-averaged U4 curve covers on the ladder (the middle `span` of the
    common range, shifted to contain u_center when it can)."""
    lo, hi = -np.inf, np.inf
    for r in records:
        m4, m2sq = analysis.u4_samples(r)
        U = m4.mean(0) / m2sq.mean(0) - 1.0
        lo, hi = max(lo, U.min()), min(hi, U.max())
    if not hi > lo:
        return []
    half = 0.5 * span * (hi - lo)
    c = min(max(u_center, lo + half), hi - half)
    return list(np.linspace(c - half, c + half, n_d))


def app_c_fits(T, N, records, u_star, rho, T_ref):
    """The joint fits of App. C on the records of every size: T_c from Eq.
    Tfsscaling over three U4 sets (exponent common to the sets for
    rho < 3.75, one per set above), nu_bar from Eq. scaling_lndotU4 with a
    common slope, and beta/nu_bar = x(T_ref) of Eq. mscaling (with
    gamma/nu_bar, the Rushbrooke-Widom sum gamma/nu_bar + 2 beta/nu_bar)."""
    out = {}
    targets = u4_targets(T, records, u_star)
    if targets:
        try:
            r = analysis.tc_from_u4_sets(T, N, records, targets, common_x=rho < 3.75)
            out.update(T_c_joint=r["T_c"], T_c_joint_error=r["T_c_error"], x_joint=r["x"],
                       x_joint_error=r["x_error"], u4_sets=r["u_targets"])
            nj, nj_err = analysis.nu_bar_joint(T, N, records, targets)
            out.update(nu_bar_joint=float(nj), nu_bar_joint_error=float(nj_err))
        except ValueError:
            pass
    b, b_err = analysis.beta_over_nu_bar(T, N, records, T_ref)
    g, _ = analysis.gamma_over_nu_bar(T, N, records, T_ref)
    out.update(beta_over_nu_bar=float(b), beta_over_nu_bar_error=float(b_err),
               rushbrooke_widom=float(g + 2 * b))
    return out


def kt_eta_run(sizes=(32, 64, 128, 256, 384), samples=32, T=(0.80, 1.00, 16), sweeps=1 << 14, meas_every=16,
               seed_base=20_000, r_values=(-1.0 / 16, 0.0, 1.0 / 16), log=None, chunk=256):
    """The square-lattice limit (rho -> infinity, z = 4: every link a nearest
    neighbour; rho = 60 gives exactly the square lattice) and the temperature
    where eta(T) = 1/4 (Sec. 4, square-lattice limit, Eq. chi_SR):
    chi = N <|m|^2> ~ L^(2 - eta) (ln L)^(-2r) fitted over the sizes at every
    ladder temperature, for each log-correction exponent r in r_values.
    Returns dict(T_eta={r: (T, error)}, eta={r: eta(T) per ladder T}, ...)."""
    import paper_1211_3991_amd as xy
    ladder = np.linspace(T[0], T[1], int(T[2]))
    recs = []
    for L in sizes:
        if log:
            log(f"square lattice L={L}: {samples} chains, {sweeps} sweeps")
        seeds = [seed_base * L + s for s in range(samples)]
        g = xy.Graph.levy(L, 4, 60.0, seeds[0])
        recs.append(_sweep_records([g] * samples, ladder, seeds, sweeps, meas_every, chunk))
    out = {"sizes": list(sizes), "samples": samples, "sweeps": sweeps, "T": ladder.tolist(), "T_eta": {}, "eta": {}}
    for r in r_values:
        t, e = analysis.t_eta(ladder, list(sizes), recs, 0.25, r)
        out["T_eta"][str(r)] = (t, e)
        out["eta"][str(r)] = analysis.eta_of_T(ladder, list(sizes), recs, r).tolist()
    rec_last = np.asarray(recs[-1])[len(recs[-1]) // 2:]
    out["E_per_site_largest"] = (rec_last[:, :, :, analysis.E].mean(axis=(0, 1)) / (sizes[-1] ** 2)).tolist()
    out["records"] = recs
    return out


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
