"""Autotuner of the fixed-point sweep configuration.

The candidates are the (cos, sin) form (hardware sine/cosine, 2048-entry
LDS table, two-level LDS table), which every sample uses, times, for batches
with workgroup-form samples, the storage form (unit vectors in LDS where a
replica fits, or angles); then, for phase-form samples, the number of stream
groups (1 to 3 streams, and, when every sample is in the phase form, two or
three streams with two or four groups each swept one after the other), which
changes only how the colour-phase launches overlap and how much state is
swept at a time.
Each candidate is timed on the live batch with HIP events
(``xy_kernel_timing``); a group count is timed both by direct launches and by
the replay of a captured HIP graph of its sweeps (how far the groups'
launches overlap differs between the two), and keeps the better of the two.
The form trials run without tempering or records, the group trials temper as
the run does; the spins, permutations and sweep counter are restored
afterwards, so tuning does not change the trajectory's inputs.  The choice is
cached in a JSON file keyed by the GPU architecture and the batch shape (the
multiset of graph sizes and the number of temperatures).
"""
import json
import os

CANDIDATES = [(2, 1), (1, 1), (0, 1), (2, 0), (1, 0), (0, 0)]   # (trig, allow_unit)


def cache_path():
    return os.environ.get("XY_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "xy_levy_autotune.json"))


def signature(batch):
    import torch
    arch = torch.cuda.get_device_properties(batch.device).gcnArchName.split(":")[0]
    sizes = {}
    for g in batch.graphs:
        sizes[g.n] = sizes.get(g.n, 0) + 1
    shape = ",".join(f"{n}x{c}" for n, c in sorted(sizes.items()))
    return f"{arch}|R={batch.R}|{shape}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _time(batch, sweeps, n_or, saved, pt_every=0):
    batch.sweep(1, n_or=n_or, pt_every=pt_every, meas_every=0)    # first launch of a kernel variant
    batch.kernel_timing(True)
    batch.sweep(sweeps, n_or=n_or, pt_every=pt_every, meas_every=0)
    ms, n = batch.kernel_time()
    batch.kernel_timing(False)
    batch.set_state(*saved)
    return ms / max(n, 1)


def _time_replay(batch, sweeps, n_or, saved, pt_every=0):
    """ms per sweep of one replay of a HIP graph of `sweeps` sweeps (captured
    and run once first)."""
    kw = dict(n_or=n_or, pt_every=pt_every, meas_every=0)
    batch.use_graph(sweeps)
    batch.sweep(sweeps, **kw)                                      # capture, run once
    batch.kernel_timing(True)
    batch.sweep(sweeps, **kw)                                      # one replay
    ms, n = batch.kernel_time()
    batch.kernel_timing(False)
    batch.use_graph(0)
    batch.set_state(*saved)
    return ms / max(n, 1)


def autotune(batch, sweeps=3, n_or=5, use_cache=True, pt_every=1, replay=True):
    """Picks and applies the fastest (trig, allow_unit) and stream-group count;
    returns a report dict.  The stream-group trials temper every pt_every
    sweeps, as the run will (their swaps add to the batch's PT counters; the
    state, labels and sweep counter are restored); with replay, each count
    is also timed by HIP-graph replay and scored by the faster of the two
    launch modes (the report names the faster mode per count; a batch on the
    null stream, which cannot be captured, is timed by direct launches only).
    The batch is left with direct launches (use_graph(0))."""
    if batch.precision != "fix16":
        return {"tuned": False, "reason": "fp64 batch"}
    forms = batch.forms()
    n_phase = int(forms.sum())
    key = signature(batch)
    path = cache_path()
    cache = _load(path) if use_cache else {}
    if key in cache and "phase_streams" in cache[key]:
        c = cache[key]
        if "trig" in c:
            batch.set_fix16_form(c["trig"], c["allow_unit"])
        batch.set_phase_streams(c["phase_streams"], c.get("phase_slices", 1))
        return {"tuned": True, "cached": True, "trig": c.get("trig"), "allow_unit": c.get("allow_unit"),
                "phase_streams": c["phase_streams"], "phase_slices": c.get("phase_slices", 1), "key": key}
    saved = batch.get_state()
    rep = {"tuned": True, "cached": False, "key": key}
    entry = {}
    if not forms.all():
        times = {}
        for trig, unit in CANDIDATES:
            batch.set_fix16_form(trig, unit)
            times[(trig, unit)] = _time(batch, sweeps, n_or, saved)
        (trig, unit), _ = min(times.items(), key=lambda kv: kv[1])
        batch.set_fix16_form(trig, unit)
        rep.update(trig=trig, allow_unit=unit,
                   ms_per_sweep={f"trig{t}_unit{u}": round(v, 4) for (t, u), v in times.items()})
        entry.update(trig=trig, allow_unit=unit, ms_per_sweep=rep["ms_per_sweep"])
    n_sw = n_sw_groups = sweeps
    if n_phase >= 1:
        # the candidates differ by a few percent: each trial runs about 40 ms
        # of sweeps (at least 2 x sweeps), twice, keeping the faster; the
        # stream-group counts, a percent or two apart, about 100 ms
        probe = _time(batch, sweeps, n_or, saved)
        n_sw = int(min(256, max(2 * sweeps, 40.0 / max(probe, 1e-3))))
        n_sw_groups = int(min(512, max(2 * sweeps, 100.0 / max(probe, 1e-3))))
    if forms.all():
        # every sample in the phase form: the (cos, sin) form alone
        times = {}
        for trig in (2, 1, 0):
            batch.set_fix16_form(trig, 1)
            times[trig] = min(_time(batch, n_sw, n_or, saved) for _ in range(2))
        trig = min(times, key=times.get)
        batch.set_fix16_form(trig, 1)
        rep.update(trig=trig, allow_unit=1, trig_ms_per_sweep={f"trig{t}": round(v, 4) for t, v in times.items()})
        entry.update(trig=trig, allow_unit=1, trig_ms_per_sweep=rep["trig_ms_per_sweep"])
    best = (batch.phase_streams(), batch.phase_slices())
    if n_phase >= 2:
        # (trials temper as the run does: each group runs its own energies and
        # tempering after its colour phases, and those tails overlap the other
        # groups' phases; the caller's stream plus three others fill the four
        # hardware queues a process gets by default: one to three streams.
        # With every sample in the phase form, also two or three streams in
        # slices of groups swept one after the other, which shrinks the state
        # swept at a time for the memory-side caches.  The fastest, the fewer
        # groups on a tie within 0.5%.)
        cands = [(n, 1) for n in range(1, min(3, n_phase) + 1)]
        if forms.all():
            cands += [(n, k) for n, k in ((2, 2), (3, 2), (2, 4)) if n * k <= n_phase]
        st, mode = {}, {}
        n_rep = min(n_sw_groups, 128)          # the replayed graph: at most 128 sweeps of launches
        replay = replay and bool(batch._s().value)   # graph capture needs a stream other than the null one
        for c in cands:
            batch.set_phase_streams(*c)
            d = min(_time(batch, n_sw_groups, n_or, saved, pt_every) for _ in range(2))
            # (and at most 256 group sweeps, about ten thousand launches: the
            # one abort of unknown cause came in a larger trial graph)
            n_c = max(2, min(n_rep, 256 // (c[0] * c[1])))
            r = min(_time_replay(batch, n_c, n_or, saved, pt_every) for _ in range(2)) if replay else float("inf")
            st[c], mode[c] = (r, "replay") if r < d else (d, "direct")
        fastest = min(st.values())
        best = next(c for c in cands if st[c] <= 1.005 * fastest)
        label = {c: (str(c[0]) if c[1] == 1 else f"{c[0]}x{c[1]}") for c in cands}
        rep["phase_streams_ms_per_sweep"] = {label[c]: round(v, 4) for c, v in st.items()}
        rep["phase_streams_launch"] = {label[c]: m for c, m in mode.items()}
        entry["phase_streams_ms_per_sweep"] = rep["phase_streams_ms_per_sweep"]
    batch.set_phase_streams(*best)
    rep["phase_streams"], rep["phase_slices"] = best
    entry["phase_streams"], entry["phase_slices"] = best
    if use_cache:
        cache[key] = entry
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    return rep


def threshold_candidates(graphs, R):
    """Phase-form thresholds worth trying for a batch: every distinct graph
    size (the smallest graphs of that size and all larger ones take the phase
    form), plus "none" (every sample in a workgroup per replica); only when
    the temperature count allows the phase form (a multiple of 4)."""
    if R % 4:
        return []
    sizes = sorted({g.n for g in graphs})
    return sizes + [sizes[-1] + 1]


def tune_phase_threshold(graphs, T, seeds=None, sweeps=4, n_or=5, use_cache=True, device="cuda"):
    """Chooses the graph size from which samples take the phase form (site-
    major state, a launch per colour phase) instead of a workgroup per
    replica, for this batch: builds a trial batch per candidate threshold
    (threshold_candidates), tunes it and times `sweeps` sweeps with the
    kernel-event timer (direct launches; see below), and returns the
    fastest threshold with the timings.
    The form is fixed when a batch is created, so the caller creates its
    batch with the result (environment variable XY_FIX16_PHASE_MIN, which
    xy_batch_sizes and xy_batch_init read).  Cached like autotune()."""
    import numpy as np
    import torch

    from . import Batch
    T = np.asarray(T, dtype=np.float64)
    R = T.shape[-1]
    cands = threshold_candidates(graphs, R)
    if not cands:
        return {"phase_min": None, "reason": "n_T is not a multiple of 4"}
    arch = torch.cuda.get_device_properties(torch.device(device)).gcnArchName.split(":")[0]
    sizes = {}
    for g in graphs:
        sizes[g.n] = sizes.get(g.n, 0) + 1
    key = f"{arch}|R={R}|" + ",".join(f"{n}x{c}" for n, c in sorted(sizes.items())) + "|phase_min"
    path = cache_path()
    cache = _load(path) if use_cache else {}
    if key in cache:
        return dict(cache[key], cached=True)
    old = os.environ.get("XY_FIX16_PHASE_MIN")
    times = {}
    try:
        for thr in cands:
            os.environ["XY_FIX16_PHASE_MIN"] = str(thr)
            b = Batch(graphs, T, precision="fix16", seeds=seeds, device=device, stream=torch.cuda.Stream())
            try:
                # (trial batches are tuned by direct launches only: a
                # replayed trial of a batch of small graphs captures up to
                # 128 sweeps of very short launches, tens of thousands of
                # graph nodes, and one such trial ended the process with an
                # abort whose cause is not known)
                autotune(b, sweeps=2, n_or=n_or, use_cache=False, replay=False)
                saved = b.get_state()
                times[thr] = min(_time(b, sweeps, n_or, saved) for _ in range(2))
            finally:
                b.close()
                torch.cuda.empty_cache()
    finally:
        if old is None:
            os.environ.pop("XY_FIX16_PHASE_MIN", None)
        else:
            os.environ["XY_FIX16_PHASE_MIN"] = old
    best = min(times, key=times.get)
    out = {"phase_min": int(best), "ms_per_sweep": {str(k): round(v, 4) for k, v in times.items()}, "cached": False}
    if use_cache:
        cache[key] = {k: v for k, v in out.items() if k != "cached"}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    return out
