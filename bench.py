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
import csv
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
VALU_PEAK_TLANE = 78.64    # published FP32 vector 157.3 TFLOP/s / 2 flops per FMA: FMA lane-instructions, 1e12/s
# Measured on MI355X with a standalone probe (independent chains, 8 waves per
# SIMD): v_fma_f32 issues at 51.7e12 lane-instructions/s (3.04 cycles per
# wave instruction per SIMD at 2.4 GHz), v_sin_f32 at 15.5e12 (10.2 cycles).
VALU_FMA_ISSUE_TLANE = 51.7
TRANS_COST = 10.17 / 3.04  # one transcendental in FMA issue slots
# transcendentals per update of the phase kernel, from its code path at the
# mean degree 6, per sweep of 1 Metropolis and 5 over-relaxation sub-sweeps:
# every update takes the (cos, sin) of 6 neighbours (12); a Metropolis update
# also those of the own and the proposed angle and one 2^x (5); an
# over-relaxation update one reciprocal for the axis, and the last sub-sweep
# the proposed angle's (cos, sin) for the energy (2); the over-relaxation
# moves the test surely accepts (about 96% of the waves) skip the rest
TRANS_PER_UPDATE = 12 + (5 + 5 * 1 + 2) / 6.0


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def uses_phase_form(wl):
    """The library's rule for the fix16 site-major phase form (does any sample
    use it): graphs of at least XY_FIX16_PHASE_MIN (16384) sites with the
    temperature count a multiple of 4; XY_FIX16_PHASE=1 / 0 forces it on / off."""
    mode = os.environ.get("XY_FIX16_PHASE", "")
    n_min = int(os.environ.get("XY_FIX16_PHASE_MIN", "") or 16384)
    if wl.n_T % 4 or mode == "0":
        return False
    return mode not in ("",) or any(s.L * s.L >= n_min for s in wl.samples)


def alg_bytes_per_update(b_s, z, R):
    """Gather-inclusive algorithmic bytes of one spin update: own read + write,
    z neighbour reads, and the CSR (z int32 columns + one row pointer) shared
    by the R replicas of a sample."""
    return 2 * b_s + z * b_s + (4 * z + 4) / R


def kernel_source_digest():
    h = hashlib.sha256()
    # the kernel sources and the runtime that groups its launches
    for f in ("kernels_phase.hip", "fix16_common.hpp", "kernels.hpp", "xy_internal.hpp", "runtime.hip"):
        with open(os.path.join(ROOT, "paper_1211_3991_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_gpu(wl, precision, steps, warmup, graphs, torch, xy, n_or=None, form=None, phase_streams=0, replay=True,
             direct=True, phase_slices=1):
    """Times `steps` sweeps (fix16: autotunes first, or takes `form` =
    (trig, allow_unit) from an earlier tuning; phase_streams > 0 then fixes
    the stream count of the phase-form sample groups, and phase_slices the
    number of group slices swept one after the other).

    The timed window of `steps` sweeps is placed so that it ends on a
    measurement sweep (it starts at a sweep index congruent to -steps modulo
    meas_every, after at least `warmup` sweeps), so it always holds the
    records of its share of the run.  With replay, the window is one replay
    of a HIP graph of `steps` sweeps captured (and run once) during the
    warm-up at the same phase; with direct, the same window is then timed
    again by direct launches at the same phase."""
    n_or = wl.n_or if n_or is None else n_or
    period = wl.meas_every if wl.meas_every > 0 else 1
    phase = (-steps) % period
    w0 = warmup + (phase - warmup) % period                    # >= warmup, congruent to phase
    n_total = w0 + 3 * steps + 2 * phase + period
    stream = torch.cuda.Stream()
    b = xy.Batch(graphs, wl.T, precision=precision, seeds=[s.seed for s in wl.samples],
                 max_records=n_total // max(wl.meas_every, 1) + 2, stream=stream)
    tune = None
    if precision == "fix16":
        if form is None:
            tune = b.autotune(n_or=n_or, use_cache=False, pt_every=wl.pt_every)
        else:
            b.set_fix16_form(trig=form[0], allow_unit=form[1])
        if phase_streams:
            b.set_phase_streams(phase_streams, phase_slices)
    kw = dict(n_or=n_or, pt_every=wl.pt_every, meas_every=wl.meas_every)
    _, acc0, tries0 = b.counters()                             # the tuner's trial swaps, left out of the rate
    b.sweep(w0, **kw)                                          # direct warm-up, ends at the window's phase

    def timed():
        b.synchronize()
        b.kernel_timing(True)
        with torch.cuda.stream(stream):
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0.record(stream)
            b.sweep(steps, **kw)
            t1.record(stream)
            torch.cuda.synchronize()
        k_ms, k_n = b.kernel_time()
        b.kernel_timing(False)
        return t0.elapsed_time(t1), k_ms / max(k_n, 1), k_n

    out = {}
    if replay:
        b.use_graph(steps)
        b.sweep(steps, **kw)                                   # capture at the window's phase, run once
        b.sweep(phase, **kw)                                   # direct, back to that phase
        ms, k_ms, k_n = timed()                                # one replay
        out.update(ms=ms, kernel_ms=k_ms, kernel_n=k_n, launch="HIP graph replay")
        b.use_graph(0)
        b.sweep(phase, **kw)
    if direct:
        ms_d, k_ms_d, k_n_d = timed()
        if not replay:
            out.update(ms=ms_d, kernel_ms=k_ms_d, kernel_n=k_n_d, launch="direct")
        out["direct_ms"] = ms_d
        out["direct_kernel_ms"] = k_ms_d
        if replay and ms_d < out["ms"]:
            # the faster launch mode of the same window is the run's: a replay
            # only saves host launch cost, and with many short launches on
            # several streams (small graphs) it is the slower one
            out.update(replay_ms=out["ms"], replay_kernel_ms=out["kernel_ms"], ms=ms_d, kernel_ms=k_ms_d,
                       kernel_n=k_n_d, launch="direct (faster than the HIP-graph replay of the same window)")
    nrec, acc, tries = b.counters()
    acc, tries = acc - acc0, tries - tries0
    n_groups = b.phase_streams() if precision == "fix16" else 1
    n_slices = b.phase_slices() if precision == "fix16" else 1
    b.close()
    out.update(window=[w0 + (steps + phase if replay else 0), steps], records=nrec, phase_streams=n_groups,
               phase_slices=n_slices,
               pt_rate=float(acc.sum()) / max(float(tries.sum()), 1.0), autotune=tune)
    return out


def time_walk(xy):
    """The random-walk workload of App. A: 20 graphs of L=196 (rho=3.5, z=4),
    4x10^4 walkers each starting on sites of degree > 2, 4096 steps.  Rate
    from the walk kernel's own duration (HIP events around it)."""
    from paper_1211_3991_amd import analysis
    G, W, T, L, rho = 20, 40000, 4096, 196, 3.5
    graphs = [xy.Graph.levy(L, 4, rho, 500 + k) for k in range(G)]
    seeds = np.arange(G, dtype=np.uint64) + 900
    xy.random_walk(graphs, W, 16, seeds=seeds, timing=True)          # first launch
    hist, ms = xy.random_walk(graphs, W, T, seeds=seeds, timing=True)
    steps = G * W * T
    d, err = analysis.spectral_dimension(hist.cpu().numpy().sum(axis=0), 32, 1024)
    # the 16-byte site record every step, and a 4-byte neighbour index on the
    # steps past the third neighbour: a fraction sum_i max(0, d_i - 3) / 2M
    # of them for a walker in its stationary law (0.312 on these graphs)
    bps = 16 + 4 * 0.312
    gbs = bps * steps / (ms * 1e6)
    return {"value": round(steps / (ms * 1e6), 2), "unit": "walker steps/ns", "kernel_ms": round(ms, 3),
            "workload": f"{G} graphs of L={L} (rho={rho}, z=4), {W} walkers each from sites of degree > 2, {T} steps",
            "dbar": round(d, 3), "dbar_err": round(err, 3), "dbar_formula": round(2 * 2 / (rho - 2), 3),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_step": bps,
                         "note": "one scattered record load per step, a second dependent one on about a third "
                                 "of the steps; the graphs (about 24 MB) stay in L2/MALL, "
                                 "so latency, not HBM bandwidth, binds"}}


def copy_bandwidth(torch, mib=1024, reps=10):
    """Achievable HBM rate of a plain device copy (bytes read + written per
    second), for context beside the published peak."""
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        dst.copy_(src)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2 * n * reps / (t0.elapsed_time(t1) * 1e6)
    del src, dst
    return round(gbs, 1)


def _pmc_rows(path):
    with open(path, newline="") as fh:
        rows = list(csv.DictReader(fh))
    return sorted(rows, key=lambda r: int(r["Dispatch_Id"]))


def write_traffic(wl, paths, argv, phase_streams, phase_slices=1):
    """HBM bytes per sweep of the dominant fix16 kernel from rocprofv3 counter
    CSVs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch, summed over a sweep's
    dispatches), each scaled by what the same counter reads for a plain 512 MiB
    device copy."""
    fetch, write, cal_f, cal_w = (_pmc_rows(p) for p in paths[:4])
    pat = "k_fix16_phase<" if uses_phase_form(wl) else "k_fix16_sweep<"

    def per_sweep(rows, counter, n_last=4):
        # counter summed over the dominant kernel's dispatches of each sweep
        # (a k_end_sweep after them ends one; with independent stream groups
        # every group ends its sweep with its own k_end_sweep, and the
        # dispatches are in enqueue order, so the later ones close nothing);
        # the mean of the last n_last sweeps, which all ran the tuned form.
        # With slices each slice runs the window's sweeps in turn, so a closed
        # run is one slice's sweep: the last n_last * phase_slices of them
        # make n_last sweeps of the whole batch
        sums, counts, cur, names, n_cur = [], [], 0.0, set(), 0
        for r in rows:
            if r["Counter_Name"] != counter:
                continue
            if pat in r["Kernel_Name"]:
                cur += float(r["Counter_Value"])
                names.add(r["Kernel_Name"])
                n_cur += 1
            elif "k_end_sweep" in r["Kernel_Name"] and n_cur:
                sums.append(cur)
                counts.append(n_cur)
                cur, n_cur = 0.0, 0
        k = n_last * phase_slices
        return sorted(names), sum(sums[-k:]) / n_last, sum(counts[-k:]) / n_last

    def copy_kib(rows, counter):
        v = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"] and r["Counter_Name"] == counter]
        return sum(v) / len(v)

    copy_bytes = 512 << 20
    f_scale = copy_bytes / (copy_kib(cal_f, "FETCH_SIZE") * 1024)
    w_scale = copy_bytes / (copy_kib(cal_w, "WRITE_SIZE") * 1024)
    names, f_kib, n_per_sweep = per_sweep(fetch, "FETCH_SIZE")
    _, w_kib, _ = per_sweep(write, "WRITE_SIZE")
    bytes_sweep = (f_kib * f_scale + w_kib * w_scale) * 1024
    upd = wl.updates_per_sweep()
    out = {"workload": wl.name, "kernels": names, "kernel_digest": kernel_source_digest(),
           "dispatches_per_sweep": round(n_per_sweep, 2), "fetch_kib_per_sweep": round(f_kib, 1),
           "write_kib_per_sweep": round(w_kib, 1), "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
           "bytes_per_sweep": int(bytes_sweep), "bytes_per_update": round(bytes_sweep / upd, 4),
           "updates_per_sweep": upd, "phase_streams": phase_streams,
           "phase_slices": phase_slices, "command": f"python bench.py {argv}"}
    # further counter CSVs (SQ_*, TCC_*, TCP_*): every counter they hold,
    # summed over a sweep's dispatches of the same kernels
    cnt = {}
    for path in paths[4:]:
        rows = _pmc_rows(path)
        for name in sorted({r["Counter_Name"] for r in rows}):
            cnt[name] = per_sweep(rows, name)[1]
    if cnt:
        out["counters_per_sweep"] = {k: round(v, 1) for k, v in cnt.items()}
    if "SQ_INSTS_VALU" in cnt:
        # VALU wave instructions of the same dispatches; x 64 lanes
        out["valu_lane_instr_per_sweep"] = int(cnt["SQ_INSTS_VALU"] * 64)
        out["valu_lane_instr_per_update"] = round(cnt["SQ_INSTS_VALU"] * 64 / upd, 2)
    if "SQ_INSTS_VMEM_RD" in cnt:
        out["vmem_rd_lane_instr_per_update"] = round(cnt["SQ_INSTS_VMEM_RD"] * 64 / upd, 2)
    if "SQ_WAIT_INST_ANY" in cnt and cnt.get("SQ_WAVE_CYCLES"):
        out["wave_cycles_waiting_frac"] = round(cnt["SQ_WAIT_INST_ANY"] / cnt["SQ_WAVE_CYCLES"], 4)
    if cnt.get("TCC_HIT_sum", 0) + cnt.get("TCC_MISS_sum", 0) > 0:
        out["l2_hit_rate"] = round(cnt["TCC_HIT_sum"] / (cnt["TCC_HIT_sum"] + cnt["TCC_MISS_sum"]), 4)
    if "TCC_READ_SECTORS_sum" in cnt:
        # 32-byte sectors read from the L2 by the kernels: the gathers' L2 traffic
        out["l2_read_bytes_per_sweep"] = int(cnt["TCC_READ_SECTORS_sum"] * 32)
        out["l2_read_bytes_per_update"] = round(cnt["TCC_READ_SECTORS_sum"] * 32 / upd, 3)
    if cnt.get("TCC_EA0_RDREQ_sum"):
        out["l2_miss_reads_to_dram_frac"] = round(cnt.get("TCC_EA0_RDREQ_DRAM_sum", 0.0) / cnt["TCC_EA0_RDREQ_sum"], 4)
    with open(traffic_file(wl.name), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def host_cpu():
    """The host's core count (this process's affinity) and CPU model."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "model": model}


def cpu_single_thread(wl_small, wl_large, large_sweeps=10):
    """The oracle on one core: the whole plain L=16 workload (one sample, 4 T,
    no tempering, measurement every sweep), and a slice of `large_sweeps`
    sweeps of one sample of the large workload with tempering."""
    import oracle
    out = {}
    for key, wl, n_sw in (("plain_l16", wl_small, wl_small.n_sweeps), ("slice", wl_large, large_sweeps)):
        s = wl.samples[0]
        e, _ = oracle.levy_graph(s.L, s.z, s.rho, s.seed)
        col, _ = oracle.slo_colour(s.L * s.L, e)
        sim = oracle.Sim(s.L * s.L, e, col, s.L, wl.T, s.seed)
        sim.init_random()
        t = time.perf_counter()
        sim.run(n_sw, n_or=wl.n_or, pt_every=wl.pt_every, meas_every=wl.meas_every if key == "plain_l16" else 0)
        dt = time.perf_counter() - t
        upd = s.L * s.L * wl.n_T * (1 + wl.n_or) * n_sw
        out[key] = {"value": round(upd / (dt * 1e9), 4), "unit": "spin updates/ns", "cores": 1,
                    "sample": f"{wl.name}: sample 0, {n_sw} sweeps, {upd} updates in {dt:.1f} s"}
    return out


def cpu_baseline(wl, seconds, workers):
    """The oracle (sequential FP64 C) on the host cores: `workers` threads,
    each sweeping its own sample of the workload (all temperatures, PT every
    sweep) for about `seconds`.  The oracle's C calls release the GIL, so the
    threads run in parallel; the rate is all updates over the wall time from a
    common start to the last thread's end."""
    import threading
    import oracle
    plans, done, errors = [None] * workers, [None] * workers, []
    ready = threading.Barrier(workers + 1)       # the workers and this thread

    def run(k):
        try:
            s = wl.samples[k % len(wl.samples)]
            e, _ = oracle.levy_graph(s.L, s.z, s.rho, s.seed)
            col, _ = oracle.slo_colour(s.L * s.L, e)
            sim = oracle.Sim(s.L * s.L, e, col, s.L, wl.T, s.seed)
            sim.init_random()
            t = time.perf_counter()
            sim.run(1, n_or=wl.n_or, pt_every=wl.pt_every, meas_every=0)
            n = max(1, int(seconds / max(time.perf_counter() - t, 1e-9)))
            plans[k] = (n, s.L * s.L * wl.n_T * (1 + wl.n_or) * n)
            ready.wait()
            sim.run(n, n_or=wl.n_or, pt_every=wl.pt_every, meas_every=0)
            done[k] = time.perf_counter()
        except BaseException as exc:             # noqa: BLE001 - reported by the caller
            errors.append(exc)
            ready.abort()

    threads = [threading.Thread(target=run, args=(k,)) for k in range(workers)]
    for th in threads:
        th.start()
    try:
        ready.wait()                             # the common start
    except threading.BrokenBarrierError:
        pass
    t0 = time.perf_counter()
    for th in threads:
        th.join()
    if errors:
        raise errors[0]
    wall = max(done) - t0
    upd = sum(u for _, u in plans)
    sweeps = sorted(set(n for n, _ in plans))
    return {"value": upd / (wall * 1e9), "unit": "spin updates/ns", "cores": workers, "kind": "oracle",
            "sample": f"samples 0-{workers - 1} of the workload (L={wl.samples[0].L}, {wl.n_T} T), one per thread, "
                      f"{sweeps[0]}-{sweeps[-1]} sweeps each with PT, {upd} updates in {wall:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="headline_l256", choices=sorted(workloads.ALL))
    ap.add_argument("--precision", default="fix16", choices=["fix16", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=32, help="sweeps of the FP64 plain comparison (0 = skip)")
    ap.add_argument("--parity-sweeps", type=int, default=1024,
                    help="sweeps of the fix16-vs-FP64 statistical comparison on the workload (0 = skip)")
    ap.add_argument("--direct", action="store_true", help="time direct launches instead of HIP-graph replay")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle time budget (0 = skip)")
    ap.add_argument("--cpu-workers", type=int, default=len(os.sched_getaffinity(0)),
                    help="oracle threads, one sample each (default: every host core this process may use)")
    ap.add_argument("--no-walk", action="store_true", help="skip the random-walk workload (App. A)")
    ap.add_argument("--split-steps", type=int, default=8,
                    help="sweeps of the Metropolis-only run that splits the rate into Met and OR (0 = skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (HBM counter calibration)")
    ap.add_argument("--phase-streams", type=int, default=0,
                    help="streams of the phase-form sample groups (default: the autotuner's choice); with "
                         "--traffic-from, the count the counters were taken with")
    ap.add_argument("--trig", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="fix the (cos, sin) form (0 two-level table, 1 2048-entry table, 2 hardware): nothing "
                         "is tuned then, and the sample groups are --phase-streams / --phase-slices or the "
                         "library's default (profiler runs, whose timing the counters distort)")
    ap.add_argument("--phase-slices", type=int, default=1,
                    help="with --phase-streams: slices of groups swept one after the other (default 1)")
    ap.add_argument("--traffic-from", nargs="+", metavar="CSV",
                    help="no GPU work: FETCH_CSV WRITE_CSV CAL_FETCH_CSV CAL_WRITE_CSV [COUNTER_CSV ...]: turn "
                         "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE counter CSVs of this workload and of "
                         "--calibrate-copy 512 (and optionally further counter CSVs: SQ_INSTS_VALU, SQ_WAIT_INST_ANY, "
                         "TCC_HIT_sum, TCC_READ_SECTORS_sum, ...) into profiles/traffic_<workload>.json")
    args = ap.parse_args()
    if args.traffic_from:
        if len(args.traffic_from) < 4:
            ap.error("--traffic-from takes at least 4 CSV paths")
        if not args.phase_streams:
            ap.error("--traffic-from needs --phase-streams: the group count the counters were taken with")
        write_traffic(workloads.ALL[args.workload](), args.traffic_from, " ".join(sys.argv[1:]), args.phase_streams,
                      args.phase_slices)
        return
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
    from paper_1211_3991_amd import parity as par
    graphs = par.build_graphs(wl.samples)
    setup_s = time.perf_counter() - t
    print(f"# graphs built in {setup_s:.1f} s; colours per sample: "
          f"{sorted(set(g.n_colours for g in graphs))}", file=sys.stderr, flush=True)

    upd_per_sweep = wl.updates_per_sweep()
    threshold = None
    if args.precision == "fix16" and len({s.L for s in wl.samples}) > 1 and "XY_FIX16_PHASE_MIN" not in os.environ:
        # uneven sizes: which samples take the phase form is tuned on trial batches
        from paper_1211_3991_amd import autotune
        threshold = autotune.tune_phase_threshold(graphs, wl.T, [s.seed for s in wl.samples], use_cache=False)
        if threshold.get("phase_min"):
            os.environ["XY_FIX16_PHASE_MIN"] = str(threshold["phase_min"])
        print(f"# phase-form threshold: {threshold}", file=sys.stderr, flush=True)
    main_run = time_gpu(wl, args.precision, args.steps, args.warmup, graphs, torch, xy,
                        form=(args.trig, 1) if args.trig >= 0 else None,
                        phase_streams=args.phase_streams, replay=not args.direct, phase_slices=args.phase_slices)
    value = upd_per_sweep * args.steps / (main_run["ms"] * 1e6)
    print(f"# {args.precision}: {main_run['ms'] / args.steps:.3f} ms/sweep ({main_run['launch']}), "
          f"{value:.1f} updates/ns; direct launches {main_run['direct_ms'] / args.steps:.3f} ms/sweep",
          file=sys.stderr, flush=True)

    z = wl.samples[0].z
    b_s = 2 if args.precision == "fix16" else 16
    bpu = alg_bytes_per_update(b_s, z, wl.n_T)
    k_ms = main_run["kernel_ms"]
    achieved = bpu * upd_per_sweep / (k_ms * 1e6)   # GB/s over the sweep's launches of the dominant kernel
    traffic, tr = None, {}
    if args.precision == "fix16" and os.path.exists(traffic_file(wl.name)):
        with open(traffic_file(wl.name)) as fh:
            tr = json.load(fh)
        # the counters hold for this kernel source and workload, in the
        # arrangement of sample groups they were taken with, which is named
        # beside them (the arrangement changes which blocks share the L2, so a
        # run in another one moves somewhat different bytes)
        if tr.get("kernel_digest") == kernel_source_digest() and tr.get("workload") == wl.name:
            traffic = tr["bytes_per_sweep"]
        else:
            tr = {}
    if args.precision == "fp64":
        kname = "k_fp64_phase (the 6·Q colour-phase launches of one sweep)"
    elif uses_phase_form(wl):
        kname = ("k_fix16_phase (the colour-phase launches of one sweep, 6·Q per sample group on its own stream, "
                 "each group also running its own energies, tempering and records; timed by HIP events on the "
                 "caller's stream around the timed window (its HIP-graph replay, or its direct launches when those "
                 "are faster: config.launch), per sweep)")
    else:
        kname = "k_fix16_sweep (one launch = one sweep of every (sample, slot))"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "achievable_copy_gbs": copy_bandwidth(torch),
                "kernel": kname,
                "kernel_ms": round(k_ms, 4), "alg_bytes_per_update": round(bpu, 3),
                "updates_per_sweep": upd_per_sweep}
    if traffic is not None:
        meas = traffic / (k_ms * 1e6)
        roofline.update(measured_gbs=round(meas, 1), measured_frac=round(meas / HBM_PEAK_GBS, 4),
                        measured_bytes_per_update=tr["bytes_per_update"],
                        traffic_sample_groups={"streams": tr.get("phase_streams"),
                                               "slices": tr.get("phase_slices", 1)})
        if tr.get("l2_read_bytes_per_sweep"):
            roofline["l2_read_gbs"] = round(tr["l2_read_bytes_per_sweep"] / (k_ms * 1e6), 1)
        if tr.get("l2_hit_rate") is not None:
            roofline["l2_hit_rate"] = tr["l2_hit_rate"]
        for k in ("l2_read_bytes_per_update", "l2_miss_reads_to_dram_frac", "wave_cycles_waiting_frac"):
            if tr.get(k) is not None:
                roofline[k] = tr[k]
    # VALU issue, from the counted VALU instructions of the same launches
    # (same digest rule as the traffic)
    alu = None
    if tr.get("valu_lane_instr_per_sweep"):
        lane = tr["valu_lane_instr_per_sweep"] / (k_ms * 1e-3) / 1e12
        alu = {"bound": "alu", "achieved": round(lane, 2), "peak": VALU_PEAK_TLANE, "unit": "T VALU lane-instr/s",
               "frac": round(lane / VALU_PEAK_TLANE, 4),
               "lane_instr_per_update": tr["valu_lane_instr_per_update"],
               "note": "peak: the published FP32 vector 157.3 TFLOP/s as FMA lane-instructions (2 flops each); "
                       "SQ_INSTS_VALU x 64 over the sweep's phase launches per second of kernel time"}
        if uses_phase_form(wl) and args.precision == "fix16":
            # issue slots: a transcendental occupies the SIMD TRANS_COST times as long as an FMA
            w = tr["valu_lane_instr_per_update"] + (TRANS_COST - 1.0) * TRANS_PER_UPDATE
            issue = lane * w / tr["valu_lane_instr_per_update"]
            alu.update(weighted_frac=round(issue / VALU_PEAK_TLANE, 4),
                       issue_frac_of_probe=round(issue / VALU_FMA_ISSUE_TLANE, 4),
                       trans_per_update=round(TRANS_PER_UPDATE, 2), trans_cost=round(TRANS_COST, 2),
                       probe_fma_issue=VALU_FMA_ISSUE_TLANE,
                       issue_note="FMA issue slots per second (transcendentals counted TRANS_COST times) over the "
                                  "rate a standalone v_fma_f32 probe reaches on this chip: the kernel is VALU-issue "
                                  "bound when this is near 1")
    # what binds: the larger of the measured HBM and VALU-issue utilisations
    if traffic is not None and alu is not None:
        u_hbm, u_alu = roofline["measured_frac"], alu.get("issue_frac_of_probe", alu["frac"])
        roofline["binding"] = {"resource": "alu" if u_alu > u_hbm else "hbm", "hbm_measured_frac": u_hbm,
                               "valu_issue_frac_of_probe": alu.get("issue_frac_of_probe"),
                               "valu_frac": alu["frac"], "valu_weighted_frac": alu.get("weighted_frac"),
                               "note": "HBM: measured bytes over the 8 TB/s peak; VALU: issue slots over the "
                                       "probe's FMA issue rate; the remainder is launch ramp and tail"}

    fp64 = None
    if args.precision == "fix16" and args.fp64_steps > 0:
        r = time_gpu(wl, "fp64", args.fp64_steps, 2, graphs, torch, xy, replay=False)
        v64 = upd_per_sweep * args.fp64_steps / (r["ms"] * 1e6)
        fp64 = {"value": round(v64, 2), "unit": "spin updates/ns", "ms_per_step": round(r["ms"] / args.fp64_steps, 3),
                "state": "FP64 unit vectors", "speedup_fix16_over_fp64": round(value / v64, 2),
                "window": r["window"], "launch": r["launch"]}
        print(f"# fp64 plain: {r['ms'] / args.fp64_steps:.3f} ms/sweep, {v64:.2f} updates/ns",
              file=sys.stderr, flush=True)

    parity = None
    if args.precision == "fix16" and args.parity_sweeps > 0:
        from paper_1211_3991_amd import parity as par
        pr, _, _ = par.fix16_vs_fp64(wl, args.parity_sweeps, meas_every=4, n_bins=20, graphs=graphs)
        parity = {k: pr[k] for k in ("sweeps", "meas_every", "keep", "records", "n_bins")}
        for k in ("per_sample", "disorder", "drift"):
            parity[k] = {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in pr[k].items()
                         if kk != "outliers"}
            parity[k]["outliers"] = pr[k]["outliers"][:8]
            if "mv" in pr[k]:
                parity[k]["mv"] = {kk: pr[k]["mv"][kk] for kk in ("min_p", "chi2_dof", "chi2_dof_bar", "nu", "n_T")}
        parity["max_rel_dev_disorder"] = {k: float(f"{v:.3g}") for k, v in pr["max_rel_dev_disorder"].items()}
        parity["rel_err_disorder"] = {k: float(f"{v:.3g}") for k, v in pr["rel_err_disorder"].items()}
        parity["r22_ok"] = par.r22_ok(pr, len(wl.samples))
        parity["note"] = ("fix16 against the FP64 sweep (bit-tied to the oracle), both from the ordered start with "
                          "independent keys: per (sample, T, observable) with jackknife errors over 20 time bins "
                          "(at most 1% beyond 3 sigma, chi2/dof <= 1.5), and disorder-paired per (T, observable) "
                          "(family-wise 1e-3 bar on each z, and Hotelling's test of the five observables of each T, "
                          "'mv'); the deviations are relative to the FP64 disorder average")
        print(f"# parity: per-sample frac>3 {parity['per_sample']['frac_gt']}, chi2 {parity['per_sample']['chi2_dof']}; "
              f"disorder frac>3 {parity['disorder']['frac_gt']}, chi2 {parity['disorder']['chi2_dof']}",
              file=sys.stderr, flush=True)

    split = None
    if args.split_steps > 0 and wl.n_or > 0:
        # Metropolis-only sweeps on the same batch shape and form; the OR rate
        # follows from the difference of the kernel times
        tuned = main_run["autotune"]
        form = (tuned["trig"], tuned["allow_unit"]) if tuned and "trig" in tuned else None
        if args.trig >= 0:
            form = (args.trig, 1)
        met = time_gpu(wl, args.precision, args.split_steps, 2, graphs, torch, xy, n_or=0, form=form,
                       phase_streams=main_run["phase_streams"], replay=not args.direct, direct=False,
                       phase_slices=main_run["phase_slices"])
        n_upd = upd_per_sweep // (1 + wl.n_or)
        or_ms = k_ms - met["kernel_ms"]
        split = {"met_only": round(n_upd / (met["kernel_ms"] * 1e6), 2),
                 "or_only": round(wl.n_or * n_upd / (or_ms * 1e6), 2) if or_ms > 0 else None,
                 "unit": "spin updates/ns (kernel time)", "met_kernel_ms": round(met["kernel_ms"], 4),
                 "note": "Metropolis-only sweeps (n_or=0, whose one sub-sweep also sums the energy for tempering) "
                         "timed the same way; OR from the difference"}
        print(f"# split: Met {split['met_only']} / OR {split['or_only']} updates/ns", file=sys.stderr, flush=True)

    walk = None
    if not args.no_walk:
        walk = time_walk(xy)
        print(f"# random walk: {walk['value']} walker steps/ns, dbar {walk['dbar']} (formula {walk['dbar_formula']})",
              file=sys.stderr, flush=True)

    cpu = None
    if args.cpu_seconds > 0:
        cpu = cpu_baseline(wl, args.cpu_seconds, args.cpu_workers)
        cpu["host"] = host_cpu()
        cpu["single_thread"] = cpu_single_thread(workloads.plain_fp64_l16(), wl)
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
                   else "FP64 unit vectors", "parallelism": "samples x temperatures on one GPU",
                   "launch": main_run["launch"], "timed_window": main_run["window"],
                   "sample_groups": {"streams": main_run["phase_streams"], "slices": main_run["phase_slices"]},
                   "records_in_window": -(-args.steps // wl.meas_every) if wl.meas_every else 0},
        "direct_launch": {"ms_per_step": round(main_run["direct_ms"] / args.steps, 4),
                          "value": round(upd_per_sweep * args.steps / (main_run["direct_ms"] * 1e6), 2)},
        "graph_replay": ({"ms_per_step": round(main_run["replay_ms"] / args.steps, 4),
                          "value": round(upd_per_sweep * args.steps / (main_run["replay_ms"] * 1e6), 2)}
                         if "replay_ms" in main_run else None),
        "roofline": roofline,
        "alu_roofline": alu,
        "fp64_plain": fp64,
        "fix16_vs_fp64": parity,
        "sub_sweep_rates": split,
        "random_walk": walk,
        "cpu_baseline": cpu,
        "pt_acceptance": round(main_run["pt_rate"], 4),
        "autotune": main_run["autotune"],
        "phase_threshold": threshold,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
