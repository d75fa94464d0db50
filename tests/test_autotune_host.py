"""Host logic of the phase-form threshold tuner (no GPU): the candidate
thresholds, one trial batch per candidate created under that threshold, the
environment restored afterwards (also when a trial fails), the fastest
candidate chosen and cached, and no candidates when the temperature count
rules the phase form out.  The device parts (trial batches, their timing and
tuning) are stand-ins here; the GPU runs them in `bench.py --workload uneven`."""
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
