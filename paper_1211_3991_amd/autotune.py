"""Autotuner of the fixed-point sweep configuration.

The candidates are the (cos, sin) form (hardware sine/cosine, 2048-entry LDS
table, two-level LDS table) times the storage form (unit vectors in LDS where a
replica fits, or angles).  Each candidate is timed on the live batch with HIP
events around the sweep kernel (``xy_kernel_timing``).  Trial sweeps run
without tempering or records, and the spins, permutations and sweep counter are
restored afterwards, so tuning does not change the trajectory's inputs.  The
choice is cached in a JSON file keyed by the GPU architecture and the batch
shape (the multiset of graph sizes and the number of temperatures).
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


def autotune(batch, sweeps=3, n_or=5, use_cache=True):
    """Picks and applies the fastest (trig, allow_unit); returns a report dict."""
    if batch.precision != "fix16":
        return {"tuned": False, "reason": "fp64 batch"}
    if batch.forms().all():
        return {"tuned": False, "reason": "every sample is in the phase form, which these choices do not affect"}
    key = signature(batch)
    path = cache_path()
    cache = _load(path) if use_cache else {}
    if key in cache:
        trig, unit = cache[key]["trig"], cache[key]["allow_unit"]
        batch.set_fix16_form(trig, unit)
        return {"tuned": True, "cached": True, "trig": trig, "allow_unit": unit, "key": key}
    saved = batch.get_state()
    times = {}
    for trig, unit in CANDIDATES:
        batch.set_fix16_form(trig, unit)
        batch.sweep(1, n_or=n_or, pt_every=0, meas_every=0)       # first launch of a kernel variant
        batch.kernel_timing(True)
        batch.sweep(sweeps, n_or=n_or, pt_every=0, meas_every=0)
        ms, n = batch.kernel_time()
        batch.kernel_timing(False)
        times[(trig, unit)] = ms / max(n, 1)
        batch.set_state(*saved)
    (trig, unit), best = min(times.items(), key=lambda kv: kv[1])
    batch.set_fix16_form(trig, unit)
    rep = {"tuned": True, "cached": False, "trig": trig, "allow_unit": unit, "key": key,
           "ms_per_sweep": {f"trig{t}_unit{u}": round(v, 4) for (t, u), v in times.items()}}
    if use_cache:
        cache[key] = {"trig": trig, "allow_unit": unit, "ms_per_sweep": rep["ms_per_sweep"]}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path + ".tmp", "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
            os.replace(path + ".tmp", path)
        except OSError:
            pass
    return rep
