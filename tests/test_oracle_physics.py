"""Pins of the oracle's dynamics and measurement against closed forms (CPU).

The method is a Markov-chain sampler, so what fixes its output is the
Boltzmann law of H = -sum_links S_i.S_j (Sec. 2, Eq. HXY; Sec. 3):
* one spin in a frozen field h follows the von Mises law
  P(theta) ~ exp(beta |h| cos(theta - phi_h)) -- tests the Metropolis move and
  its detailed balance, with and without over-relaxation;
* tiny graphs: exact E and C = beta^2 Var(H) from Bessel closed forms (tree:
  Z ~ I0(beta)^(n-1); n-cycle: Z ~ sum_k I_k(beta)^n) and by quadrature (K4);
  with and without parallel tempering;
* low T: E/N -> -z/2 + (1 - n_c/N) T/2 (harmonic equipartition);
* high T: E/N = -(M/N) t - (n_tri/N) 6 t^2 t' - (n_sq/N) 8 t^3 t' + O(t^5),
  t = I1/I0 (high-temperature cycle expansion);
* measurement: all-aligned state, spin wave along x, infinite temperature
  (<|m|^2> = 1/N, <F> = 1, U4 = 1 - 1/N exactly);
* over-relaxation is an energy-conserving involution (Creutz).
Parity: pinned.
"""
import numpy as np
import pytest
from scipy import special

import oracle
from stats_helpers import batch_mean_err, jackknife_fn

TS = np.array([0.8, 1.2, 1.6, 2.0])


# ----------------------------------------------------------------- exact values
def tree_exact(beta, n_links):
    t = special.iv(1, beta) / special.iv(0, beta)
    var1 = 1.0 - t / beta - t * t
    return -n_links * t, beta * beta * n_links * var1


def cycle_exact(beta, n, kmax=40):
    k = np.arange(-kmax, kmax + 1)
    f = special.iv(k, beta)
    f1 = 0.5 * (special.iv(k - 1, beta) + special.iv(k + 1, beta))
    f2 = 0.25 * (special.iv(k - 2, beta) + 2 * special.iv(k, beta) + special.iv(k + 2, beta))
    Z = np.sum(f ** n)
    Z1 = np.sum(n * f ** (n - 1) * f1)
    Z2 = np.sum(n * (n - 1) * f ** (n - 2) * f1 ** 2 + n * f ** (n - 1) * f2)
    E = -Z1 / Z
    var = Z2 / Z - (Z1 / Z) ** 2
    return E, beta * beta * var


def quadrature_exact(beta, n, edges, M=48):
    """Trapezoid rule on the torus with theta_0 = 0 (spectrally accurate)."""
    g = 2 * np.pi * np.arange(M) / M
    grids = np.meshgrid(*([g] * (n - 1)), indexing="ij")
    th = [np.zeros_like(grids[0])] + list(grids)
    H = np.zeros_like(grids[0])
    for a, b in edges:
        H -= np.cos(th[a] - th[b])
    w = np.exp(-beta * (H - H.min()))
    Z = w.sum()
    E = (w * H).sum() / Z
    var = (w * H * H).sum() / Z - E * E
    return E, beta * beta * var


GRAPHS = {
    "link": (2, [(0, 1)]),
    "chain3": (3, [(0, 1), (1, 2)]),
    "triangle": (3, [(0, 1), (1, 2), (2, 0)]),
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "K4": (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]),
}


def exact(name, beta):
    n, e = GRAPHS[name]
    if name in ("link", "chain3"):
        return tree_exact(beta, len(e))
    if name in ("triangle", "cycle4"):
        return cycle_exact(beta, n)
    return quadrature_exact(beta, n, e)


def test_exact_values_agree_with_each_other():
    # closed forms and quadrature are independent routes to the same numbers
    for beta in 1 / TS:
        for name in ("link", "triangle", "cycle4"):
            n, e = GRAPHS[name]
            a = exact(name, beta)
            b = quadrature_exact(beta, n, e, M=64)
            assert np.allclose(a, b, rtol=1e-10, atol=1e-12)
    # published-by-nobody sanity: link energy at beta = 1 is -I1/I0 = -0.44638996...
    assert abs(tree_exact(1.0, 1)[0] + 0.446389965896535) < 1e-14


# ------------------------------------------------------------------ the moves
@pytest.mark.parametrize("hx,hy,beta,or_every", [(1.2, -0.7, 1.5, 0), (0.3, 0.2, 2.0, 0),
                                                 (-2.0, 1.0, 0.7, 2), (0.0, 3.0, 1.0, 3)])
def test_frozen_field_von_mises(hx, hy, beta, or_every):
    ang, acc = oracle.frozen_field_chain(hx, hy, beta, 17, 400_000, or_every)
    kappa = beta * np.hypot(hx, hy)
    d = ang - np.arctan2(hy, hx)
    for f, target in ((np.cos(d), special.iv(1, kappa) / special.iv(0, kappa)),
                      (np.cos(2 * d), special.iv(2, kappa) / special.iv(0, kappa)),
                      (np.sin(d), 0.0), (np.sin(2 * d), 0.0)):
        m, e = batch_mean_err(f, 100)
        assert abs(m - target) < 4.5 * e + 1e-12, (m, target, e)


def test_or_involution_and_energy():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        hx, hy = rng.normal(size=2) * 3
        th = rng.uniform(0, 2 * np.pi)
        x, y = np.cos(th), np.sin(th)
        x1, y1 = oracle.or_move(hx, hy, x, y)
        assert abs((hx * x1 + hy * y1) - (hx * x + hy * y)) <= 1e-13 * np.hypot(hx, hy)
        assert abs(np.hypot(x1, y1) - 1) < 1e-14
        x2, y2 = oracle.or_move(hx, hy, x1, y1)
        assert abs(x2 - x) < 1e-14 and abs(y2 - y) < 1e-14
    assert oracle.or_move(0.0, 0.0, 0.6, 0.8) == (0.6, 0.8)


# ------------------------------------------------------------- tiny graphs
def _run_tiny(name, pt_every, n_sweeps=120_000, T=TS, seed=3):
    n, e = GRAPHS[name]
    e = np.array(e, dtype=np.int32)
    col, _ = oracle.slo_colour(n, e)
    sim = oracle.Sim(n, e, col, n, T, seed)
    sim.init_random()
    out = sim.run(n_sweeps, n_or=5, pt_every=pt_every, meas_every=1)
    return sim, out["records"]


@pytest.mark.parametrize("name", list(GRAPHS))
def test_tiny_graph_energy_and_heat(name):
    _, rec = _run_tiny(name, 0)
    rec = rec[rec.shape[0] // 10:]
    for k, T in enumerate(TS):
        beta = 1 / T
        E_ex, C_ex = exact(name, beta)
        E = rec[:, k, 0]
        mE, eE = batch_mean_err(E)
        C, eC = jackknife_fn(lambda a, b: beta * beta * (b - a * a), [E, E * E])
        assert abs(mE - E_ex) < 4.5 * eE, (name, T, mE, E_ex, eE)
        assert abs(C - C_ex) < 4.5 * eC, (name, T, C, C_ex, eC)


@pytest.mark.parametrize("name", ["triangle", "K4"])
def test_tiny_graph_with_parallel_tempering(name):
    sim, rec = _run_tiny(name, 1, seed=8)
    rec = rec[rec.shape[0] // 10:]
    for k, T in enumerate(TS):
        E_ex, _ = exact(name, 1 / T)
        mE, eE = batch_mean_err(rec[:, k, 0])
        assert abs(mE - E_ex) < 4.5 * eE, (name, T, mE, E_ex, eE)
    acc, tries = sim.pt_counts()
    assert tries[:3].min() > 10_000 and acc[:3].min() > 0


def test_equal_temperatures_every_swap_accepted():
    n, e = GRAPHS["cycle4"]
    e = np.array(e, dtype=np.int32)
    col, _ = oracle.slo_colour(n, e)
    sim = oracle.Sim(n, e, col, n, np.full(5, 1.3), 2)
    sim.init_random()
    out = sim.run(101, pt_every=1, meas_every=0, pt_log=True)
    acc, tries = sim.pt_counts()
    assert np.array_equal(acc, tries) and tries.sum() == 101 * 2
    assert np.all(out["pt_log"][out["pt_log"] > 0] == 1)


# ---------------------------------------------------------------- limits
def _levy(L=16, z=6, rho=3.5, seed=1):
    e, _ = oracle.levy_graph(L, z, rho, seed)
    col, _ = oracle.slo_colour(L * L, e)
    return e, col


def _components(n, e):
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a, b in e:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    return len({find(a) for a in range(n)})


def test_low_temperature_equipartition():
    L = 16
    n = L * L
    e, col = _levy(L)
    T = np.array([0.05, 0.1])
    sim = oracle.Sim(n, e, col, L, T, 4)
    sim.set_state(np.tile([1.0, 0.0], (2, n, 1)))
    rec = sim.run(6000, meas_every=1)["records"][3000:]
    nc = _components(n, e)
    for k, t in enumerate(T):
        target = -len(e) / n + (1 - nc / n) * t / 2
        m, err = batch_mean_err(rec[:, k, 0] / n)
        # next order is O(T^2): (M/N) T^2 / 8 per link-ish
        assert abs(m - target) < 4 * err + 0.5 * (len(e) / n) * t * t, (t, m, target)
    # T = 0: the aligned state is the ground state, E = -M exactly
    assert sim.energy(0) <= -len(e) * (1 - 0.2)


def test_high_temperature_series():
    L = 16
    n = L * L
    e, col = _levy(L)
    beta = 0.05
    sim = oracle.Sim(n, e, col, L, np.array([1 / beta]), 6)
    sim.init_random()
    rec = sim.run(60_000, meas_every=1)["records"][1000:]
    A = np.zeros((n, n))
    A[e[:, 0], e[:, 1]] = 1
    A[e[:, 1], e[:, 0]] = 1
    n_tri = np.trace(A @ A @ A) / 6
    A2 = A @ A
    c = np.triu(A2, 1)
    n_sq = 0.5 * np.sum(c * (c - 1) / 2)
    t = special.iv(1, beta) / special.iv(0, beta)
    tp = 1 - t / beta - t * t
    target = -(len(e) / n) * t - (n_tri / n) * 6 * t * t * tp - (n_sq / n) * 8 * t ** 3 * tp
    m, err = batch_mean_err(rec[:, 0, 0] / n)
    assert abs(m - target) < 4.5 * err, (m, target, err)
    assert abs(-(len(e) / n) * beta / 2 - target) < 0.01       # leading order -(z/2)(beta/2)


# ----------------------------------------------------------- measurement
def test_measure_aligned_and_spin_wave():
    L = 16
    n = L * L
    e, col = _levy(L)
    sim = oracle.Sim(n, e, col, L, np.array([1.0, 2.0]), 1)
    xy = np.zeros((2, n, 2))
    xy[0, :, 0] = 1.0
    X = np.arange(n) % L
    xy[1, :, 0] = np.cos(2 * np.pi * X / L)
    xy[1, :, 1] = np.sin(2 * np.pi * X / L)
    sim.set_state(xy)
    o = sim.measure()
    assert o[0, 0] == -len(e)
    assert abs(o[0, 1] - 1) < 1e-15 and abs(o[0, 2] - 1) < 1e-15
    assert o[0, 3] < 1e-20 and o[0, 4] < 1e-20
    assert abs(o[1, 3] - n / 2) < 1e-9 * n and o[1, 4] < 1e-20
    assert abs(o[1, 1]) < 1e-25


def test_infinite_temperature_moments():
    L = 16
    n = L * L
    e, col = _levy(L)
    sim = oracle.Sim(n, e, col, L, np.array([1e30]), 12)
    sim.init_random()
    rec = sim.run(30_000, meas_every=1)["records"]
    m2, e2 = batch_mean_err(rec[:, 0, 1])
    assert abs(m2 * n - 1) < 4.5 * e2 * n
    F, eF = batch_mean_err(0.5 * (rec[:, 0, 3] + rec[:, 0, 4]))
    assert abs(F - 1) < 4.5 * eF
    U4, eU = jackknife_fn(lambda a, b: b / (a * a) - 1, [rec[:, 0, 1], rec[:, 0, 2]])
    assert abs(U4 - (1 - 1 / n)) < 4.5 * eU


# ------------------------------------------------------- initial state (pinned)
def test_initial_directions_uniform_and_independent():
    """The random start (the workloads' "spins initialised uniform in
    [0, 2 pi)") is an independent uniform direction per (seed, slot, site):
    unit norm; the angle's Fourier moments <cos k theta>, <sin k theta> vanish
    for k = 1..8 (a point drawn in the square instead of the disk leaves
    <cos 4 theta> = 3 - pi = -0.14); the angle passes a Kolmogorov-Smirnov
    test against U[0, 2 pi); and angles of lattice neighbours, of two slots of
    one site and of two seeds are uncorrelated (a shared or reused stream
    would correlate them)."""
    from scipy import stats
    L, n_T = 64, 8
    n = L * L
    e = np.array([(i, (i + 1) % n) for i in range(0, n, 2)], np.int32)   # any graph: the start ignores links
    col = np.zeros(n, np.int32)
    col[1::2] = 1
    T = np.linspace(1.0, 2.0, n_T)
    angles = []
    for seed in (3, 4):
        sim = oracle.Sim(n, e, col, L, T, seed)
        sim.init_random()
        xy_, _, sw = sim.get_state()
        assert sw == 0
        assert np.allclose(np.hypot(xy_[..., 0], xy_[..., 1]), 1.0, rtol=0, atol=4e-16)
        angles.append(np.arctan2(xy_[..., 1], xy_[..., 0]) % (2 * np.pi))   # [slot, site]
    th = np.concatenate([a.ravel() for a in angles])
    se = 1.0 / np.sqrt(2 * th.size)             # std of <cos k theta> for uniform theta
    for k in range(1, 9):
        assert abs(np.cos(k * th).mean()) < 4.5 * se, k
        assert abs(np.sin(k * th).mean()) < 4.5 * se, k
    assert stats.kstest(th / (2 * np.pi), "uniform").pvalue > 1e-4
    a = angles[0]
    grid = a.reshape(n_T, L, L)
    pairs = {"x neighbours": (grid[:, :, :-1], grid[:, :, 1:]), "y neighbours": (grid[:, :-1, :], grid[:, 1:, :]),
             "slots 0/1": (a[0], a[1]), "seeds 3/4": (angles[0], angles[1])}
    for name, (u, v) in pairs.items():
        c = np.cos(u - v).ravel()                # uniform and independent: <cos(u - v)> = 0
        assert abs(c.mean()) < 4.5 / np.sqrt(2 * c.size), name
        assert not np.array_equal(u, v), name
