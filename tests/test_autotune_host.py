"""Host logic of the tuners (no GPU), with stand-ins for the device parts.
Phase-form threshold: the candidate thresholds, one trial batch per
candidate created under that threshold, the environment restored afterwards
(also when a trial fails), the fastest candidate chosen and cached, and no
candidates when the temperature count rules the phase form out (the GPU runs
it in `bench.py --workload uneven`).  Stream-group trials of autotune(): the
candidate arrangements, each scored by the faster of its two launch modes,
the fewer groups on a tie within 0.5%, replayed trials of at most 256 group
sweeps, direct launches only on the null stream, and the cached choice."""
import json
import os
import types

import numpy as np
import pytest

import paper_1211_3991_amd as xy
from paper_1211_3991_amd import autotune


class _G:
    def __init__(self, n):
        self.n = n


@pytest.fixture
def fake_device(monkeypatch, tmp_path):
    """Stand-ins for the device calls of tune_phase_threshold; returns the
    log of trial batches (threshold in force, close called)."""
    import torch
    monkeypatch.setenv("XY_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(torch.cuda, "get_device_properties",
                        lambda dev: types.SimpleNamespace(gcnArchName="gfx950:sramecc+:xnack-"))
    monkeypatch.setattr(torch.cuda, "Stream", lambda *a, **k: object())
    monkeypatch.setattr(torch.cuda, "empty_cache", lambda: None)
    log = []
    cost = {}

    class FakeBatch:
        def __init__(self, graphs, T, precision, seeds=None, device=None, stream=None):
            assert precision == "fix16" and stream is not None
            self.thr = int(os.environ["XY_FIX16_PHASE_MIN"])
            self.entry = {"thr": self.thr, "closed": False}
            log.append(self.entry)

        def get_state(self):
            return ("state", self.thr)

        def close(self):
            self.entry["closed"] = True

    tuned = []
    monkeypatch.setattr(xy, "Batch", FakeBatch)
    monkeypatch.setattr(autotune, "autotune", lambda b, **kw: tuned.append(kw))
    monkeypatch.setattr(autotune, "_time", lambda b, sweeps, n_or, saved: cost[b.thr])
    return types.SimpleNamespace(log=log, cost=cost, tuned=tuned, path=tmp_path / "tune.json")


def test_candidates():
    gs = [_G(1024)] * 3 + [_G(16384)] * 2 + [_G(4096)]
    assert autotune.threshold_candidates(gs, 8) == [1024, 4096, 16384, 16385]
    assert autotune.threshold_candidates(gs, 6) == []
    assert autotune.threshold_candidates([_G(65536)], 24) == [65536, 65537]


def test_picks_fastest_restores_env_and_caches(fake_device, monkeypatch):
    monkeypatch.setenv("XY_FIX16_PHASE_MIN", "777")
    gs = [_G(1024)] * 6 + [_G(16384)] * 4
    fake_device.cost.update({1024: 2.0, 16384: 1.5, 16385: 3.0})
    rep = autotune.tune_phase_threshold(gs, np.linspace(1.0, 2.5, 8))
    assert rep["phase_min"] == 16384 and not rep["cached"]
    assert rep["ms_per_sweep"] == {"1024": 2.0, "16384": 1.5, "16385": 3.0}
    assert [e["thr"] for e in fake_device.log] == [1024, 16384, 16385]
    assert all(e["closed"] for e in fake_device.log)
    # every trial batch is tuned by direct launches only
    assert fake_device.tuned and all(kw.get("replay") is False for kw in fake_device.tuned)
    assert os.environ["XY_FIX16_PHASE_MIN"] == "777"
    cache = json.load(open(fake_device.path))
    (key, entry), = cache.items()
    assert key == "gfx950|R=8|1024x6,16384x4|phase_min" and entry["phase_min"] == 16384
    n_trials = len(fake_device.log)
    again = autotune.tune_phase_threshold(gs, np.linspace(1.0, 2.5, 8))
    assert again["cached"] and again["phase_min"] == 16384 and len(fake_device.log) == n_trials


def test_env_restored_when_a_trial_fails(fake_device, monkeypatch):
    monkeypatch.delenv("XY_FIX16_PHASE_MIN", raising=False)
    gs = [_G(1024), _G(16384)]

    def boom(b, sweeps, n_or, saved):
        raise RuntimeError("trial failed")
    monkeypatch.setattr(autotune, "_time", boom)
    with pytest.raises(RuntimeError):
        autotune.tune_phase_threshold(gs, np.linspace(1.0, 2.5, 4), use_cache=False)
    assert "XY_FIX16_PHASE_MIN" not in os.environ
    assert fake_device.log and all(e["closed"] for e in fake_device.log)


def test_no_phase_form_for_ladders_not_a_multiple_of_four(fake_device):
    rep = autotune.tune_phase_threshold([_G(16384)] * 2, np.arange(1.0, 4.0))
    assert rep["phase_min"] is None and not fake_device.log


class _TuneBatch:
    """Stand-in for a fixed-point batch whose every sample is in the phase
    form: records the arrangement and (cos, sin) form the tuner sets."""
    precision = "fix16"
    device = "cuda:0"
    R = 8

    def __init__(self, n_samples):
        self.graphs = [_G(16384)] * n_samples
        self.arr = (1, 1)
        self.trig = None
        self.calls = []

    def forms(self):
        return np.ones(len(self.graphs), dtype=np.int32)

    def get_state(self):
        return ("state",)

    def set_fix16_form(self, trig, allow_unit):
        self.trig = trig

    def set_phase_streams(self, n, slices=1):
        self.arr = (n, slices)
        self.calls.append(self.arr)

    def phase_streams(self):
        return self.arr[0]

    def phase_slices(self):
        return self.arr[1]

    def _s(self):
        return types.SimpleNamespace(value=1234)


@pytest.fixture
def fake_tuning(monkeypatch, tmp_path):
    import torch
    monkeypatch.setenv("XY_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(torch.cuda, "get_device_properties",
                        lambda dev: types.SimpleNamespace(gcnArchName="gfx950:sramecc+:xnack-"))
    t = types.SimpleNamespace(direct={}, replay={}, trig={2: 1.0, 1: 1.3, 0: 1.2}, replay_sweeps=[])

    def fake_time(batch, sweeps, n_or, saved, pt_every=0):
        if batch.calls:
            return t.direct[batch.arr]
        return t.trig.get(batch.trig, 1.0)     # the probe and the (cos, sin) trials come first

    def fake_replay(batch, sweeps, n_or, saved, pt_every=0):
        t.replay_sweeps.append((batch.arr, sweeps))
        return t.replay[batch.arr]
    monkeypatch.setattr(autotune, "_time", fake_time)
    monkeypatch.setattr(autotune, "_time_replay", fake_replay)
    return t


def test_group_trials_pick_fastest_mode_and_cap_replays(fake_tuning):
    b = _TuneBatch(10)
    arrs = [(1, 1), (2, 1), (3, 1), (2, 2), (3, 2), (2, 4)]
    fake_tuning.direct.update(dict(zip(arrs, [1.00, 0.95, 0.96, 0.99, 0.97, 1.10])))
    fake_tuning.replay.update(dict(zip(arrs, [0.99, 0.96, 0.90, 0.98, 0.904, 1.20])))
    rep = autotune.autotune(b, sweeps=3)
    assert rep["trig"] == 2 and b.trig == 2
    assert set(rep["phase_streams_ms_per_sweep"]) == {"1", "2", "3", "2x2", "3x2", "2x4"}
    assert rep["phase_streams_ms_per_sweep"]["3"] == 0.9 and rep["phase_streams_launch"]["3"] == "replay"
    assert rep["phase_streams_launch"]["2"] == "direct" and rep["phase_streams_launch"]["2x4"] == "direct"
    # 3 streams wins; 3x2 (0.904) is within 0.5% but has more groups and comes later
    assert (rep["phase_streams"], rep["phase_slices"]) == (3, 1) and b.arr == (3, 1)
    # every replayed trial holds at most 256 group sweeps (and at least 2 sweeps)
    for (n, k), sweeps in fake_tuning.replay_sweeps:
        assert 2 <= sweeps <= max(2, 256 // (n * k))
    assert dict(fake_tuning.replay_sweeps)[(2, 4)] == 32
    # the cached choice is applied to a fresh batch without trials
    b2 = _TuneBatch(10)
    n_trials = len(fake_tuning.replay_sweeps)
    again = autotune.autotune(b2)
    assert again["cached"] and b2.arr == (3, 1) and b2.trig == 2 and len(fake_tuning.replay_sweeps) == n_trials


def test_group_trials_tie_goes_to_fewer_groups(fake_tuning):
    b = _TuneBatch(4)
    arrs = [(1, 1), (2, 1), (3, 1), (2, 2)]
    fake_tuning.direct.update(dict(zip(arrs, [1.004, 1.0, 1.02, 1.03])))
    fake_tuning.replay.update(dict(zip(arrs, [1.05, 1.05, 1.05, 1.05])))
    rep = autotune.autotune(b, sweeps=2, use_cache=False)
    assert set(rep["phase_streams_ms_per_sweep"]) == {"1", "2", "3", "2x2"}     # (2, 4) needs 8 samples
    assert (rep["phase_streams"], rep["phase_slices"]) == (1, 1)


def test_group_trials_direct_only_on_the_null_stream(fake_tuning):
    b = _TuneBatch(4)
    b._s = lambda: types.SimpleNamespace(value=None)
    fake_tuning.direct.update({(1, 1): 1.0, (2, 1): 0.9, (3, 1): 0.95, (2, 2): 0.97})
    rep = autotune.autotune(b, sweeps=2, use_cache=False)
    assert not fake_tuning.replay_sweeps and set(rep["phase_streams_launch"].values()) == {"direct"}
    assert rep["phase_streams"] == 2
