"""Validation of the GPU path against the paper's critical temperature in the
Erdos-Renyi limit (Sec. 5, subsection on the Erdos-Renyi limit; Table 2,
column rho = 0).

A Levy graph with rho = 0 and z = 4 is an Erdos-Renyi graph of mean degree 4
(Sec. 2).  The paper finds T_c = 1.93(1) from the temperatures T(N) where
U4(T, N) crosses U4(T, N/4), extrapolated with T(N) = C N^(-1/nu) + T_c and
the mean-field nu = 2, in agreement with the analytic value 1.9361 (the Bethe
condition I1(beta)/I0(beta) = 1/4 for an excess degree of 4).

Here: 64 samples each of L = 16, 32, 64, 128, 16 temperatures in [1.7, 2.2],
PT every sweep, 2^14 sweeps of 1 Metropolis + 5 OR (first half discarded),
measurement every 16 sweeps, on the fixed-point path.  The extrapolated T_c
must agree with the analytic value within three standard errors (jackknife
over samples, propagated through the fit) plus the paper's own 0.01.  The
same run gives the mean-field exponents the paper reports for this graph:
nu_bar = 2 from dU4/dT at fixed U4 (Eq. U4dot; paper 2.00(2)), within three
standard errors plus 0.1, and gamma/nu_bar = 1/2 from chi at T_c, within
three standard errors plus 0.05 (finite-size corrections at these sizes).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1211_3991_amd as xy  # noqa: E402
from paper_1211_3991_amd import analysis  # noqa: E402

SIZES = (16, 32, 64, 128)
G, N_SWEEPS, MEAS = 64, 1 << 14, 16


def _run(L, T):
    seeds = [10_000 * L + s for s in range(G)]
    graphs = [xy.Graph.levy(L, 4, 0.0, sd) for sd in seeds]
    b = xy.Batch(graphs, T, precision="fix16", seeds=seeds, max_records=N_SWEEPS // MEAS)
    b.sweep(N_SWEEPS, n_or=5, pt_every=1, meas_every=MEAS)
    torch.cuda.synchronize()
    rec = b.records().cpu().numpy()
    b.close()
    return rec


def test_erdos_renyi_z4_critical_temperature():
    T = workloads.linear_ladder(1.7, 2.2, 16)
    rec = {}
    for L in SIZES:
        print(f"ER z=4 L={L}: {G} samples, {N_SWEEPS} sweeps", flush=True)
        rec[L] = _run(L, T)
        assert rec[L].shape[0] == N_SWEEPS // MEAS
    N, Tx, err = [], [], []
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        t, e = analysis.u4_crossing(T, rec[a], rec[b])
        print(f"U4 crossing L={a}/{b}: T = {t} +- {e}", flush=True)
        assert t is not None, f"U4 of L={a} and L={b} do not cross in [1.7, 2.2]"
        N.append(b * b)
        Tx.append(t)
        err.append(e)
    nu = 2.0
    tc, c = analysis.fss_tc(N, Tx, nu)
    # standard error of T_c: the fit is linear in the crossing temperatures
    x = np.asarray(N, float) ** (-1.0 / nu)
    A = np.stack([np.ones_like(x), x], axis=1)
    w = np.linalg.pinv(A)[0]
    sigma = float(np.sqrt(np.sum((w * np.asarray(err)) ** 2)))
    ref = analysis.bethe_tc(4.0)
    print(f"T_c = {tc:.4f} +- {sigma:.4f} (C = {c:.3f}); analytic {ref:.4f}, paper 1.93(1)", flush=True)
    assert abs(tc - ref) <= 3.0 * sigma + 0.01

    # nu_bar from dU4/dT at fixed U4 (Eq. U4dot), at the U4 value of the
    # largest pair's crossing; mean field (and the paper's 2.00(2)): 2
    m4, m2sq = analysis.u4_samples(rec[SIZES[-2]])
    u_star = float(np.interp(Tx[-1], T, m4.mean(0) / m2sq.mean(0) - 1.0))
    Ns = [L * L for L in SIZES]
    nu, nu_err = analysis.nu_bar_from_u4(T, Ns, [rec[L] for L in SIZES], u_star)
    print(f"nu_bar = {nu:.3f} +- {nu_err:.3f} at U4 = {u_star:.3f}; mean field 2, paper 2.00(2)", flush=True)
    assert abs(nu - 2.0) <= 3.0 * nu_err + 0.1
    # gamma / nu_bar from chi at the analytic T_c; mean field: 1 / 2
    g, g_err = analysis.gamma_over_nu_bar(T, Ns, [rec[L] for L in SIZES], ref)
    print(f"gamma/nu_bar = {g:.3f} +- {g_err:.3f}; mean field 0.5", flush=True)
    assert abs(g - 0.5) <= 3.0 * g_err + 0.05
