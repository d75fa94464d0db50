"""Throughput of the XY / Levy-graph Monte Carlo hot path on one MI355X.

A step is one sweep of the whole hot path over the batch: 1 Metropolis + 5
over-relaxation sub-sweeps of every spin of every (sample, temperature),
energies, a parallel-tempering step, and every 32nd sweep the measurement of
E, |m|^2, |m|^4, F(k_min) (the paper's cadence, Sec. 4).  Graph sampling,
colouring and upload happen once, before the timed region, as in the paper.

Workload (default): 64 samples of L=256 Levy graphs, z=6, rho=3.5, 24
temperatures in [1.0, 2.5], 16-bit fixed-point angles (the batched form).
The FP64 plain path is timed on the same workload for the speedup, and the
oracle (sequential FP64 C) on a bounded slice on the host cores.

Prints one JSON line (rank 0; one GPU only).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fix16_sweep_L256.json")


def alg_bytes_per_update(b_s, z, R):
    """Gather-inclusive algorithmic bytes of one spin update: own read + write,
    z neighbour reads, and the CSR (z int32 columns + one row pointer) shared
    by the R replicas of a sample."""
    return 2 * b_s + z * b_s + (4 * z + 4) / R


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("kernels_fix16.hip", "kernels.hpp", "xy_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1211_3991_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_gpu(wl, precision, steps, warmup, graphs, torch, xy):
    stream = torch.cuda.Stream()
    b = xy.Batch(graphs, wl.T, precision=precision, seeds=[s.seed for s in wl.samples],
                 max_records=max(1, (steps + warmup) // wl.meas_every + 1), stream=stream)
    tune = b.autotune(n_or=wl.n_or, use_cache=False) if precision == "fix16" else None
    b.sweep(warmup, n_or=wl.n_or, pt_every=wl.pt_every, meas_every=wl.meas_every)
    b.synchronize()
    b.kernel_timing(True)
    with torch.cuda.stream(stream):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        b.sweep(steps, n_or=wl.n_or, pt_every=wl.pt_every, meas_every=wl.meas_every)
        t1.record(stream)
        torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    k_ms, k_n = b.kernel_time()
    b.kernel_timing(False)
    nrec, acc, tries = b.counters()
    rec = b.records().cpu().numpy()
    b.close()
    return {"ms": ms, "kernel_ms": k_ms / max(k_n, 1), "kernel_n": k_n, "records": rec,
            "pt_rate": float(acc.sum()) / max(float(tries.sum()), 1.0), "autotune": tune}


def cpu_baseline(wl, seconds):
    """The oracle, single-threaded, on sample 0 of the workload (all its
    temperatures), as many whole sweeps as fit in about `seconds`."""
    import oracle
    s = wl.samples[0]
    e, _ = oracle.levy_graph(s.L, s.z, s.rho, s.seed)
    col, _ = oracle.slo_colour(s.L * s.L, e)
    sim = oracle.Sim(s.L * s.L, e, col, s.L, wl.T, s.seed)
    sim.init_random()
    t = time.perf_counter()
    sim.run(1, n_or=wl.n_or, pt_every=wl.pt_every, meas_every=0)
    one = time.perf_counter() - t
    n = max(1, int(seconds / max(one, 1e-9)) - 1)
    t = time.perf_counter()
    sim.run(n, n_or=wl.n_or, pt_every=wl.pt_every, meas_every=0)
    dt = time.perf_counter() - t
    upd = s.L * s.L * wl.n_T * (1 + wl.n_or) * n
    return {"value": upd / (dt * 1e9), "unit": "spin updates/ns", "cores": 1, "kind": "oracle",
            "sample": f"sample 0 of the workload (L={s.L}, {wl.n_T} T), {n} sweeps with PT, "
                      f"{upd} updates in {dt:.1f} s, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="headline_l256", choices=sorted(workloads.ALL))
    ap.add_argument("--precision", default="fix16", choices=["fix16", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=8, help="sweeps of the FP64 plain comparison (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle time budget (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the samples are independent and a multi-GPU "
              "run would shard them with no communication; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n, "copies": 5}))
        return
    import paper_1211_3991_amd as xy

    wl = workloads.ALL[args.workload]()
    t = time.perf_counter()
    graphs = [xy.Graph.levy(s.L, s.z, s.rho, s.seed) for s in wl.samples]
    setup_s = time.perf_counter() - t
    print(f"# graphs built in {setup_s:.1f} s; colours per sample: "
          f"{sorted(set(g.n_colours for g in graphs))}", file=sys.stderr, flush=True)

    upd_per_sweep = wl.updates_per_sweep()
    main_run = time_gpu(wl, args.precision, args.steps, args.warmup, graphs, torch, xy)
    value = upd_per_sweep * args.steps / (main_run["ms"] * 1e6)
    print(f"# {args.precision}: {main_run['ms'] / args.steps:.3f} ms/sweep, {value:.1f} updates/ns",
          file=sys.stderr, flush=True)

    z = wl.samples[0].z
    b_s = 2 if args.precision == "fix16" else 16
    bpu = alg_bytes_per_update(b_s, z, wl.n_T)
    k_ms = main_run["kernel_ms"]
    achieved = bpu * upd_per_sweep / (k_ms * 1e6)   # GB/s, one sweep kernel launch = one sweep
    traffic = None
    if args.precision == "fix16" and os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("kernel_digest") == kernel_source_digest() and tr.get("workload") == wl.name:
            traffic = tr["bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": ("k_fix16_sweep (one launch = one sweep of every (sample, slot))" if args.precision == "fix16"
                           else "k_fp64_phase (all colour-phase launches of a sweep)"),
                "kernel_ms": round(k_ms, 4), "alg_bytes_per_update": round(bpu, 3),
                "updates_per_launch": upd_per_sweep}

    fp64 = None
    if args.precision == "fix16" and args.fp64_steps > 0:
        r = time_gpu(wl, "fp64", args.fp64_steps, 2, graphs, torch, xy)
        v64 = upd_per_sweep * args.fp64_steps / (r["ms"] * 1e6)
        fp64 = {"value": round(v64, 2), "unit": "spin updates/ns", "ms_per_step": round(r["ms"] / args.fp64_steps, 3),
                "state": "FP64 unit vectors", "speedup_fix16_over_fp64": round(value / v64, 2)}
        print(f"# fp64 plain: {r['ms'] / args.fp64_steps:.3f} ms/sweep, {v64:.2f} updates/ns",
              file=sys.stderr, flush=True)

    cpu = cpu_baseline(wl, args.cpu_seconds) if args.cpu_seconds > 0 else None
    s0 = wl.samples[0]
    out = {
        "metric": "spin updates/ns at L=256 rho=3.5 (fixed-point batched vs FP64 plain), %HBM roof",
        "value": round(value, 2), "unit": "spin updates/ns", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(main_run["ms"] / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fix16" else "f64", "data": "synthetic",
        "config": {"workload": wl.name, "samples": len(wl.samples), "L": s0.L, "z": s0.z, "rho": s0.rho,
                   "n_T": wl.n_T, "T": [float(wl.T[0]), float(wl.T[-1])], "sweep": f"1 Metropolis + {wl.n_or} OR",
                   "pt_every": wl.pt_every, "meas_every": wl.meas_every,
                   "state": "uint16 angles, FP32 fields, FP64 accumulators" if args.precision == "fix16"
                   else "FP64 unit vectors", "parallelism": "samples x temperatures on one GPU"},
        "roofline": roofline,
        "fp64_plain": fp64,
        "cpu_baseline": cpu,
        "pt_acceptance": round(main_run["pt_rate"], 4),
        "autotune": main_run["autotune"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
