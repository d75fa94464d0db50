"""GPU tests of the temperature-ladder argument of xy_sweep and of HIP-graph
replay, through the C ABI.

* A ladder change between sweep calls (App. B: the replicas keep their
  temperature labels, PT keeps exchanging them) is exact on the FP64 path: the
  state and labels equal the oracle's when the oracle is rebuilt with the new
  ladder from the state it had reached.
* Replayed chunks equal direct launches for tempering / record periods whose
  pattern repeats with lcm(pt_every, meas_every) rather than their maximum,
  for chunks that are and are not multiples of that period, with calls of
  uneven lengths, and with kernel timing on (a replay is timed as a whole).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1211_3991_amd as xy  # noqa: E402


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.mark.parametrize("pt_every", [0, 1])
def test_ladder_change_mid_run_exact(pt_every):
    L, z, rho, seed = 16, 6, 3.5, 1
    T1 = np.array([0.8, 1.2, 1.6, 2.0])
    T2 = np.array([0.7, 1.0, 1.9, 2.6])
    g = xy.Graph.levy(L, z, rho, seed)
    b = xy.Batch([g], T1, precision="fp64", seeds=[seed])
    b.sweep(7, n_or=5, pt_every=pt_every, meas_every=0)
    b.sweep(9, n_or=5, pt_every=pt_every, meas_every=0, T=T2)
    st, sot, sw = b.get_state()

    e, _ = oracle.levy_graph(L, z, rho, seed)
    col, _ = oracle.slo_colour(L * L, e)
    first = oracle.Sim(L * L, e, col, L, T1, seed)
    first.init_random()
    first.run(7, n_or=5, pt_every=pt_every, meas_every=0)
    mid, mid_sot, mid_sw = first.get_state()
    second = oracle.Sim(L * L, e, col, L, T2, seed)     # the oracle rebuilt with the new ladder
    second.set_state(mid, mid_sot, mid_sw)
    second.run(9, n_or=5, pt_every=pt_every, meas_every=0)
    ref, ref_sot, ref_sw = second.get_state()
    assert sw == ref_sw == 16
    assert np.array_equal(sot[0], ref_sot)
    assert np.array_equal(_bits(st[0]), _bits(ref))
    # the new ladder is what a measurement reports by temperature: E at the
    # lowest new temperature is the replica holding index 0
    o = b.measure().cpu().numpy()[0]
    second_meas = second.measure()
    assert np.allclose(o[:, :5], second_meas[:, :5], rtol=1e-11, atol=1e-12)
    assert np.array_equal(b.T[0], T2)


def test_ladder_argument_rejects_bad_temperatures():
    g = xy.Graph.levy(16, 6, 3.5, 1)
    b = xy.Batch([g], [1.0, 2.0], precision="fix16", seeds=[1])
    b.sweep(2, pt_every=1, meas_every=0)
    before = b.get_state()
    for bad in ([1.0, 0.0], [1.0, -2.0], [np.nan, 1.0], [np.inf, 1.0]):
        with pytest.raises(xy.XYError):
            b.sweep(1, pt_every=1, meas_every=0, T=bad)
    after = b.get_state()      # rejected calls ran nothing
    assert after[2] == before[2] == 2
    assert all(np.array_equal(x, y) for x, y in zip(after[0], before[0]))
    with pytest.raises(ValueError):
        b.sweep(1, T=[1.0, 2.0, 3.0])


def _fix16_graphs(kind):
    if kind == "phase":        # every sample in the phase form: independent stream groups
        return [xy.Graph.levy(128, 6, 3.5, s) for s in range(4)]
    return [xy.Graph.levy(32, 6, 3.5, s) for s in range(4)]   # one workgroup per replica


@pytest.mark.parametrize("kind", ["phase", "workgroup"])
@pytest.mark.parametrize("pt_every,meas_every,chunk", [(3, 4, 4), (2, 3, 3), (2, 3, 6), (3, 4, 12),
                                                       (1, 32, 20), (0, 5, 7)])
def test_replay_equals_direct_for_any_period(kind, pt_every, meas_every, chunk):
    graphs = _fix16_graphs(kind)
    T = workloads.linear_ladder(1.0, 2.5, 8)
    calls = [5, 13, 20, 3, 27, 40]
    n_rec = sum(calls) // meas_every + 1
    direct = xy.Batch(graphs, T, precision="fix16", seeds=np.arange(4) + 20, max_records=n_rec,
                      stream=torch.cuda.Stream())
    graph = xy.Batch(graphs, T, precision="fix16", seeds=np.arange(4) + 20, max_records=n_rec,
                     stream=torch.cuda.Stream())
    graph.use_graph(chunk)
    graph.kernel_timing(True)
    done = 0
    for k, n in enumerate(calls):
        direct.sweep(n, pt_every=pt_every, meas_every=meas_every)
        graph.sweep(n, pt_every=pt_every, meas_every=meas_every)
        done += n
        a, b_ = direct.get_state(), graph.get_state()
        assert a[2] == b_[2] == done
        assert all(np.array_equal(x, y) for x, y in zip(a[0], b_[0])), (k, done)
        assert np.array_equal(a[1], b_[1]), (k, done)
        ca, cb = direct.counters(), graph.counters()
        assert ca[0] == cb[0] and np.array_equal(ca[1], cb[1]) and np.array_equal(ca[2], cb[2]), (k, done)
        assert np.array_equal(direct.records().cpu().numpy(), graph.records().cpu().numpy()), (k, done)
    ms, n_timed = graph.kernel_time()
    graph.kernel_timing(False)
    assert ms > 0 and n_timed == done      # every sweep is inside one timed event pair


def test_replay_after_ladder_change_equals_direct():
    """The captured kernels read 1/T from device memory: a ladder change needs
    no new capture, and replays continue to equal direct launches."""
    graphs = _fix16_graphs("phase")
    T1 = workloads.linear_ladder(1.0, 2.5, 8)
    T2 = workloads.linear_ladder(0.9, 3.0, 8)
    runs = []
    for chunk in (0, 8):
        b = xy.Batch(graphs, T1, precision="fix16", seeds=np.arange(4) + 5, max_records=8,
                     stream=torch.cuda.Stream())
        if chunk:
            b.use_graph(chunk)
        b.sweep(16, pt_every=1, meas_every=8)
        b.sweep(16, pt_every=1, meas_every=8, T=T2)
        runs.append((b.get_state(), b.records().cpu().numpy(), b.counters()))
    (sa, ra, ca), (sb, rb, cb) = runs
    assert sa[2] == sb[2] == 32 and np.array_equal(sa[1], sb[1])
    assert all(np.array_equal(x, y) for x, y in zip(sa[0], sb[0]))
    assert np.array_equal(ra, rb) and np.array_equal(ca[1], cb[1])
