#!/usr/bin/env python3
"""Benchmark of the resampling hot path on one MI355X.

A step is one pass of the single-filter path over the N = 2^24 workload
(Gaussian-likelihood weights, y = 4, eps = 0.01, so B ~ 353), through the
HIP library's C ABI:
    mgp_compute_B                 reduction (fp32 max, fp64 sum), B, Megopolis offsets
    mgp_resample_gather_prepared  the accept loop (the dominant kernel) with
                                  x_bar_i = x_{k_i} (D = 8 fp32 states) as its epilogue
Each step uses a new seed. The weights and states are resident in HBM
before the timed region. Metropolis is timed the same way for comparison,
and the unfused step (accept loop, then mgp_gather) beside it.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "particles resampled/s at N=2^24 (Megopolis vs Metropolis) + % HBM peak; p99"
LOOP_SOURCES = ["paper_2109_13504_amd/csrc/mgp_device.h", "paper_2109_13504_amd/csrc/mgp_kernels.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_megopolis_fused_n2pow24_y4_d8.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for p in LOOP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--variant", default="megopolis", choices=["megopolis", "metropolis", "c1", "c2"])
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--y", type=float, default=4.0)
    ap.add_argument("--eps", type=float, default=0.01)
    ap.add_argument("--d", type=int, default=8)
    ap.add_argument("--metropolis-steps", type=int, default=3)
    ap.add_argument("--no-metropolis", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=16, help="oracle runs every k-th particle's chain")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-filters section")
    ap.add_argument("--batch-runs", type=int, default=20)
    ap.add_argument("--batch-shape", default=None,
                    help="fixed batched launch shape 'block_threads,particles_per_thread,schedule' (default: autotuned)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--no-sweep", action="store_true", help="skip the per-variant sweep at N=2^22")
    ap.add_argument("--no-prefix", action="store_true",
                    help="skip the prefix-sum methods (multinomial, systematic) against Megopolis")
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--no-sir", action="store_true", help="skip the SIR filter section")
    ap.add_argument("--no-segment64", action="store_true", help="skip the 64-wide-segment Megopolis step")
    ap.add_argument("--sir-table", action="store_true",
                    help="the SIR section for every (variant, B) row of Table 2 instead of Megopolis B=16 only")
    ap.add_argument("--sir-mc-runs", type=int, default=50)
    ap.add_argument("--sir-bsweep", action="store_true",
                    help="the SIR section for B in {5, 7, 10, 15, 20, 25, 30, 40} and every variant (Section 7's "
                         "B study)")
    ap.add_argument("--unfused-steps", type=int, default=10,
                    help="steps of the unfused comparison (accept loop, then mgp_gather)")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the streaming-read ceiling measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 256 MiB (counter calibration for profiling)")
    return ap.parse_args()


def timed_steps(torch, mgp, r, w, states, anc, out, variant, eps, steps, warmup, seed0, segment=32, fused=True):
    """Runs warmup + steps; returns wall ms per step and per-step event times.
    fused: mgp_compute_B, then mgp_resample_gather_prepared (the accept loop
    with the particle copy as its epilogue); otherwise mgp_compute_B,
    mgp_resample_prepared and mgp_gather."""
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]

    def one(s, e):
        seed = seed0 + s
        if e:
            e[0].record(stream)
        r.compute_B(w, variant, epsilon=eps, seed=seed, segment=segment)
        if e:
            e[1].record(stream)
        if fused:
            r.resample_gather_prepared(w, states, variant, epsilon=eps, seed=seed, out=out, anc=anc, segment=segment)
            if e:
                e[2].record(stream)
        else:
            r.resample_prepared(w, variant, epsilon=eps, seed=seed, out=anc, segment=segment)
            if e:
                e[2].record(stream)
            mgp.gather(states, anc, out=out)
        if e:
            e[3].record(stream)

    for s in range(warmup):
        one(1000 + s, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        one(s, ev[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = {"total": [], "reduce_B": [], "loop": [], "gather": []}
    for e in ev:
        per["reduce_B"].append(e[0].elapsed_time(e[1]))
        per["loop"].append(e[1].elapsed_time(e[2]))
        per["gather"].append(e[2].elapsed_time(e[3]))
        per["total"].append(e[0].elapsed_time(e[3]))
    return (t1 - t0) * 1000.0 / steps, per


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def median_call_ms(torch, fn, runs=10, warmup=3):
    """Median device time (HIP events on the current stream) of fn(k) for k =
    warmup .. warmup + runs - 1, after `warmup` untimed calls (fn(0) ..) that
    bring the weights into the caches and the launch path up to speed. Each
    timed call is synchronised alone."""
    import numpy as np
    stream = torch.cuda.current_stream()
    for k in range(warmup):
        fn(k)
    torch.cuda.synchronize()
    times = []
    for k in range(warmup, warmup + runs):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn(k)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def cpu_baseline(w_np, variant, eps, stride):
    """The oracle as it is, single-threaded, on a bounded sample: the full
    reduction and B, then the chains of every stride-th particle."""
    import numpy as np

    import oracle
    n = w_np.size
    idx = np.arange(0, n, stride, dtype=np.int32)
    t0 = time.perf_counter()
    B, _, _ = oracle.B_from_weights(w_np, eps)
    ref, accepts = oracle.resample_subset(w_np, variant, B, 12345, idx, return_accepts=True)
    dt = time.perf_counter() - t0
    out = {"value": idx.size / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
           "sample": f"single-threaded C oracle: fp64 reduction + B over all {n} weights, then the B-step chains "
                     f"of every {stride}th particle ({idx.size} particles, {variant}, B={B}); {dt:.1f} s",
           # the chains the GPU runs are the same (bit-identical ancestors),
           # so this is the acceptance rate of the timed accept loop too
           "acceptance_rate": accepts / (idx.size * B)}
    # the same sample with the chains split over the host's cores (the
    # oracle's calls release the GIL and share no state): identical output
    from concurrent.futures import ThreadPoolExecutor
    threads = min(16, len(os.sched_getaffinity(0)))
    if threads > 1:
        parts = np.array_split(idx, threads)
        t0 = time.perf_counter()
        B2, _, _ = oracle.B_from_weights(w_np, eps)
        with ThreadPoolExecutor(threads) as ex:
            got = list(ex.map(lambda part: oracle.resample_subset(w_np, variant, B2, 12345, part), parts))
        dt2 = time.perf_counter() - t0
        if B2 == B and np.array_equal(np.concatenate(got), ref):
            out["all_cores"] = {"value": idx.size / dt2, "cores": threads, "seconds": dt2}
    return out


def ceiling_section(torch, mgp):
    """The memory ceilings the accept loop is compared with, measured here:
    the streaming-read rate (mgp_probe_stream_read: float4 loads, four in
    flight per thread, each pass rotated so that the L2 cannot serve a block's
    next pass) over buffers of 64 MB to 2 GB, each launch reading its buffer
    as many times as makes about 4 GB; the best of 4096, 8192 and 16384 blocks
    of 256 threads, median of 3 launches after one warm-up. Up to 256 MB the
    buffer stays in the 256 MB Infinity Cache (the L2s hold 4 MB per XCD);
    from 1 GB it streams from HBM."""
    import numpy as np
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    buf = torch.ones((2 << 30) // 4, dtype=torch.float32, device=dev)
    sink = torch.empty(16384, dtype=torch.float32, device=dev)
    rows = {}
    for mb in (64, 128, 192, 256, 1024, 2048):
        nbytes = mb << 20
        passes = max(1, (4 << 30) // nbytes)
        best = None
        for blocks in (4096, 8192, 16384):
            times = []
            for k in range(4):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                mgp.mgp_probe_stream_read(buf.data_ptr(), nbytes, passes, blocks, sink.data_ptr(), stream.cuda_stream)
                b.record(stream)
                torch.cuda.synchronize()
                if k:
                    times.append(a.elapsed_time(b))
            ms = float(np.median(times))
            gbs = passes * nbytes / (ms * 1e-3) / 1e9
            if best is None or gbs > best["GBs"]:
                best = {"passes": passes, "blocks": blocks, "ms": ms, "GBs": gbs}
        rows[f"{mb}MB"] = best
    del buf, sink
    mall = max(rows[k]["GBs"] for k in ("64MB", "128MB", "192MB", "256MB"))
    hbm = max(rows[k]["GBs"] for k in ("1024MB", "2048MB"))
    log(f"[bench] streaming read: Infinity Cache {mall:.0f} GB/s, HBM {hbm:.0f} GB/s; "
        + ", ".join(f"{k} {v['GBs']:.0f}" for k, v in rows.items()))
    return {"workload": "streaming read (mgp_probe_stream_read), ~4 GB per launch, best of 4096/8192/16384 blocks "
                        "x 256 threads, median of 3", "rows": rows, "infinity_cache_read_GBs": mall,
            "hbm_read_GBs": hbm}


def pattern_ceiling(torch, mgp, n, steps):
    """The ceiling the Megopolis loop's own access pattern sets: its candidate
    reads over a mirrored array of 2n + 1024 floats (the 4n-byte weights
    twice) at `steps` shared offsets, without random draws or accept steps
    (mgp_probe_pattern_read); median of 5 launches after one warm-up. Rate =
    4 n steps bytes / time."""
    import numpy as np
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mirror = torch.rand(2 * n + 1024, dtype=torch.float32, device=dev)
    offs = torch.from_numpy(np.random.Generator(np.random.PCG64(2109)).integers(0, n, steps).astype(np.uint32)
                            .view(np.int32)).to(dev)
    sink = torch.empty(n // 1024, dtype=torch.float32, device=dev)
    times = []
    for k in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        mgp.mgp_probe_pattern_read(mirror.data_ptr(), mirror.numel() * 4, n, offs.data_ptr(), steps,
                                   sink.data_ptr(), stream.cuda_stream)
        b.record(stream)
        torch.cuda.synchronize()
        if k:
            times.append(a.elapsed_time(b))
    del mirror, offs, sink
    ms = float(np.median(times))
    gbs = 4.0 * n * steps / (ms * 1e-3) / 1e9
    log(f"[bench] Megopolis read pattern alone (n={n}, {steps} steps): {ms:.3f} ms, {gbs:.0f} GB/s")
    return {"workload": f"mgp_probe_pattern_read: the four-particle Megopolis loop's candidate reads, n={n}, "
                        f"{steps} steps, no draws or accept steps; median of 5 after one warm-up",
            "n": n, "steps": steps, "ms": ms, "GBs": gbs}


def batched_section(torch, mgp, inputs, runs, shape=None):
    """512 filters, N_f = round(2^U(10, 18)), y_f ~ U[0, 4], D = 4, Megopolis:
    one graph launch per run against the same filters as 512 per-filter
    launch sequences (reduce, finalize, loop, gather) issued from C. `shape`
    (block threads, particles per thread, schedule) skips the autotuner."""
    import tempfile

    import numpy as np
    dev = torch.device("cuda:0")
    sizes, ys = inputs.batch_filters()
    fl = []
    for f, (n, y) in enumerate(zip(sizes, ys)):
        w, st = inputs.gaussian_weights_and_states(int(n), float(y), 4, f)
        fl.append({"w": torch.from_numpy(w).to(dev), "anc": torch.empty(int(n), dtype=torch.int32, device=dev),
                   "states": torch.from_numpy(st).to(dev), "out": torch.empty((int(n), 4), device=dev),
                   "seed": 777000 + f, "stream_id": f, "epsilon": 0.01})
    cache = os.path.join(tempfile.gettempdir(), "mgp_batch_tune.txt")
    t0 = time.perf_counter()
    if shape:
        bt, ppt, sched = shape
        plan = mgp.BatchPlan(fl, "megopolis", d=4, block_threads=bt, particles_per_thread=ppt, schedule=sched)
    else:
        plan = mgp.BatchPlan(fl, "megopolis", d=4, tune_cache=cache)
    plan_s = time.perf_counter() - t0
    info = plan.info()
    stream = torch.cuda.current_stream()

    def timed(fn, k):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - w0) * 1000.0 / k
        per = [a.elapsed_time(b) for a, b in evs]
        return wall, per

    g_wall, g_per = timed(plan.run, runs)
    s_wall, s_per = timed(plan.run_separate, max(3, runs // 4))
    total_n = int(np.sum(sizes))
    steps = info["est_particle_steps"]
    plan.close()
    return {
        "workload": "512 filters, N_f=round(2^U(10,18)), y_f~U[0,4], eps=0.01, Megopolis, fused gather D=4",
        "particles": total_n,
        "particle_steps": steps,
        "graph_ms": g_wall,
        "graph_p50_ms": pct(g_per, 50),
        "graph_p99_ms": pct(g_per, 99),
        "separate_ms": s_wall,
        "separate_p50_ms": pct(s_per, 50),
        "separate_p99_ms": pct(s_per, 99),
        "speedup_vs_separate": s_wall / g_wall,
        "particles_per_s": total_n / (g_wall * 1e-3),
        "effective_weight_GBs": 4.0 * steps / (g_wall * 1e-3) / 1e9,
        "tuned_shape": {"block_threads": info["block_threads"], "particles_per_thread": info["particles_per_thread"],
                        "schedule": "grid" if info["schedule"] == 1 else "persistent",
                        "from_cache": bool(info["from_cache"])},
        "plan_create_s": plan_s,
    }


def sweep_section(torch, mgp, inputs):
    """The paper's timing experiment on this GPU: resample time (reduction, B,
    accept loop; no gather) at N = 2^22 for Megopolis, Metropolis, C1 and C2
    at 128 and 2048 bytes, y = 0..4, eps = 0.01; median of 10 calls after 3
    warm-up calls. Then the
    partition-size study: C1 and C2 at 128..2048 bytes at y = 4."""
    import numpy as np
    dev = torch.device("cuda:0")
    n = 1 << 22
    r = mgp.Resampler(n)
    anc = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    rows = [("megopolis", 128), ("metropolis", 128), ("c1", 128), ("c1", 2048), ("c2", 128), ("c2", 2048)]
    out = {}
    for y in range(5):
        w = torch.from_numpy(inputs.gaussian_weights(n, float(y), 0)).to(dev)
        for v, ps in rows:
            key = f"{v}-ps{ps}" if v in ("c1", "c2") else v
            ms = median_call_ms(torch, lambda k: r.resample(w, v, epsilon=0.01, seed=k, partition_bytes=ps, out=anc))
            out.setdefault(key, {})[f"y{y}"] = {"ms": ms, "B": r.last_stats()["B"]}
    # the partition-size study: C1 and C2 at every partition size, y = 4
    w = torch.from_numpy(inputs.gaussian_weights(n, 4.0, 0)).to(dev)
    parts = {}
    for v in ("c1", "c2"):
        for ps in (128, 256, 512, 1024, 2048):
            parts[f"{v}-ps{ps}"] = median_call_ms(
                torch, lambda k: r.resample(w, v, epsilon=0.01, seed=k, partition_bytes=ps, out=anc))
    return {"workload": "N=2^22, Gaussian-likelihood weights, eps=0.01; resample = reduction + B + accept loop "
                        "(no gather); median of 10 calls after 3 warm-up calls", "ms": out,
            "partition_sizes_y4_ms": parts}


def configs_section(torch, mgp, inputs):
    """The two smaller workloads, timed like the paper's experiment (median of
    the calls after 3 warm-up calls, HIP events on the launch stream):
      - one filter, N = 4096, y = 2, eps = 0.01: Metropolis and Megopolis,
        resample only (reduction + B + accept loop);
      - one filter, N = 2^20, y = 0..4, eps = 0.01: the four variants (C1/C2
        with 128-byte partitions), resample alone and resample + gather of D = 4
        fp32 states."""
    import numpy as np
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def med(fn, runs):
        return median_call_ms(torch, fn, runs=runs)

    small = {}
    n = 4096
    r = mgp.Resampler(n)
    anc = torch.empty(n, dtype=torch.int32, device=dev)
    w = torch.from_numpy(inputs.gaussian_weights(n, 2.0, 0)).to(dev)
    for v in ("metropolis", "megopolis"):
        ms = med(lambda k: r.resample(w, v, epsilon=0.01, seed=k, out=anc), 20)
        small[v] = {"ms": ms, "B": r.last_stats()["B"]}
    mid = {}
    n = 1 << 20
    r = mgp.Resampler(n)
    anc = torch.empty(n, dtype=torch.int32, device=dev)
    out = torch.empty((n, 4), device=dev)
    for y in range(5):
        wn, st = inputs.gaussian_weights_and_states(n, float(y), 4, 0)
        w, states = torch.from_numpy(wn).to(dev), torch.from_numpy(st).to(dev)
        for v in ("megopolis", "metropolis", "c1", "c2"):
            ms_r = med(lambda k: r.resample(w, v, epsilon=0.01, seed=k, out=anc), 10)
            B = r.last_stats()["B"]

            def step(k):
                r.resample(w, v, epsilon=0.01, seed=k, out=anc)
                mgp.gather(states, anc, out=out)
            mid.setdefault(v, {})[f"y{y}"] = {"resample_ms": ms_r, "with_gather_ms": med(step, 10), "B": B}
    return {"n4096_y2": {"workload": "single filter, N=4096, y=2, eps=0.01; resample = reduction + B + accept loop; "
                                     "median of 20 calls after 3 warm-up calls", "ms": small},
            "n2pow20": {"workload": "single filter, N=2^20, y=0..4, eps=0.01, C1/C2 at 128-byte partitions; "
                                    "resample, and resample + gather of D=4 fp32 states; median of 10 calls after 3 "
                                    "warm-up calls",
                        "ms": mid}}


def table2():
    """Table 2 of the paper (K40m): {(variant, B): (resample ratio, RMSE)}."""
    with open(os.path.join(ROOT, "tests", "golden", "sir_table2.json")) as f:
        g = json.load(f)
    return {(r["variant"], r["B"]): (r["resample_ratio"], r["rmse"]) for r in g["rows"]}


def sir_rmse(est, truth, trajectories, mc_runs):
    """Mean over trajectories of the RMSE of Section 7: per step, the root
    mean square error over the Monte Carlo runs; then the mean over steps."""
    import numpy as np
    T = est.shape[1]
    e = est.reshape(trajectories, mc_runs, T) - truth[:, None, 1:]
    per_traj = np.sqrt(np.mean(e * e, axis=1)).mean(axis=1)
    return float(per_traj.mean()), per_traj


def sir_section(torch, mgp, inputs, rows, trajectories=16, mc_runs=50, log2n=20, T=100):
    """Section 7's experiment: the SIR filter of Algorithm 6 on the model of
    eqs. (predict-end2end)/(update-end2end), 16 ground-truth trajectories x
    50 Monte Carlo runs, 2^20 particles, 100 steps, all 800 runs advanced
    together. Per (variant, B): stage by stage with HIP events around each stage for the resample ratio
    tau_2 / (tau_1 + tau_2 + tau_3), then the whole experiment as one graph
    launch (timed; its estimates must equal the stage-by-stage ones), and the
    RMSE."""
    import numpy as np
    n = 1 << log2n
    R = trajectories * mc_runs
    dev = torch.device("cuda:0")
    truth, z = inputs.sir_truth(T, trajectories)
    zr = np.repeat(z, mc_runs, axis=0)  # run r follows trajectory r // mc_runs
    x0 = inputs.sir_initial_particles_torch(R, n, dev)
    stream = torch.cuda.current_stream()
    out = {}
    unbiased = {r["method"]: (r["resample_ratio"], r["rmse"])
                for r in json.load(open(os.path.join(ROOT, "tests", "golden", "sir_table2.json")))["unbiased"]}
    for variant, B in rows:
        if variant in unbiased:
            key = variant
        else:
            key = f"{variant}-B{B}" if variant not in ("c1", "c2") else f"{variant}-ps128-B{B}"
        t0 = time.perf_counter()
        f = mgp.SirFilter(R, n, T, variant=variant, B=B, epsilon=0.1, seed=2021, use_graph=True)
        create_s = time.perf_counter() - t0
        f.set_measurements(zr)
        # stage by stage, events around each stage (this pass also warms up)
        f.reset(x0)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(T)]
        for t in range(1, T + 1):
            e = ev[t - 1]
            e[0].record(stream)
            f.predict_update(t)
            e[1].record(stream)
            f.resample(t)
            e[2].record(stream)
            f.estimate(t)
            e[3].record(stream)
        torch.cuda.synchronize()
        tau = [sum(e[k].elapsed_time(e[k + 1]) for e in ev) for k in range(3)]
        est2 = f.results()[0]
        # the whole experiment as one graph launch
        f.reset(x0)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        f.run()
        b.record(stream)
        torch.cuda.synchronize()
        graph_ms = [a.elapsed_time(b)]
        est, bs, st = f.results()
        f.close()
        rmse, per_traj = sir_rmse(est, truth, trajectories, mc_runs)
        ratio = tau[1] / sum(tau)
        paper = unbiased.get(variant) if variant in unbiased else table2().get((variant, B))
        steps = R * n * T
        out[key] = {
            "B": B, "rmse": rmse, "rmse_per_trajectory_min": float(per_traj.min()),
            "rmse_per_trajectory_max": float(per_traj.max()),
            "resample_ratio": ratio, "stage_ms_per_step": [x / T for x in tau],
            "graph_ms_per_step": graph_ms[-1] / T, "particle_steps_per_s": steps / (graph_ms[-1] * 1e-3),
            "stage_by_stage_equals_graph": bool(np.array_equal(est, est2)),
            "degenerate_steps": int((st != 0).sum()), "create_s": create_s,
            "mean_B": float(bs[st == 0].mean()) if (st == 0).any() else 0.0,
            "paper_k40m": {"resample_ratio": paper[0], "rmse": paper[1]} if paper else None,
        }
        log(f"[bench] sir {key}: RMSE {rmse:.3f} (paper {paper[1] if paper else '-'}), ratio {ratio:.3f} "
            f"(paper {paper[0] if paper else '-'}), stages {[round(x / T, 3) for x in tau]} ms/step, "
            f"graph {graph_ms[-1] / T:.3f} ms/step")
    del x0
    return {"workload": f"SIR filter (Algorithm 6), {trajectories} trajectories x {mc_runs} Monte Carlo runs, "
                        f"N=2^{log2n}, T={T}; stage 1 fp64, x/w fp32; C1/C2 partitions of 128 bytes",
            "runs": R, "n": n, "steps": T, "rows": out}


# Table 3 (Megopolis), y = 4 column, seconds on the Tesla K40m, by N
K40M_MEGOPOLIS_Y4 = {1 << 15: 5.170e-4, 1 << 16: 8.173e-4, 1 << 17: 0.0014, 1 << 18: 0.0027, 1 << 19: 0.0055,
                     1 << 20: 0.0113, 1 << 21: 0.0233, 1 << 22: 0.0478}


def n_sweep_section(torch, mgp, inputs):
    """Megopolis resample time (reduction, B, offsets, accept loop; no
    gather) against N = 2^12 .. 2^26, Gaussian-likelihood weights y = 4,
    eps = 0.01, median of 10 calls after 3 warm-up calls; the paper's Table 3
    y = 4 column (from 2^15) as
    context."""
    import numpy as np
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    rows = {}
    for ln in range(12, 27):
        n = 1 << ln
        w = torch.from_numpy(inputs.gaussian_weights(n, 4.0, 0)).to(dev)
        anc = torch.empty(n, dtype=torch.int32, device=dev)
        r = mgp.Resampler(n)
        ms = median_call_ms(torch, lambda k: r.resample(w, "megopolis", epsilon=0.01, seed=k, out=anc))
        B = r.last_stats()["B"]
        k40 = K40M_MEGOPOLIS_Y4.get(n)
        rows[f"2^{ln}"] = {"ms": ms, "B": B, "particles_per_s": n / (ms * 1e-3),
                           "effective_GBs": 4.0 * n * (B + 2) / (ms * 1e-3) / 1e9,
                           "k40m_ms": k40 * 1e3 if k40 else None}
        del w, anc, r
    return {"workload": "Megopolis, Gaussian-likelihood weights y=4, eps=0.01; resample = reduction + B + accept loop "
                        "(no gather); median of 10 after 3 warm-up calls; k40m_ms from Table 3", "rows": rows}


def prefix_section(torch, mgp, inputs):
    """Section 6.5's comparison with the unbiased prefix-sum methods on this
    GPU: multinomial (Algorithm 7) and systematic (Algorithm 8) resampling
    through mgp_resample_prefix against Megopolis (mgp_resample), N = 2^16 ..
    2^24, y = 0, 2, 4, eps = 0.01; each a whole call (reduction and validation,
    the fixed-point prefix sum, the search), median of 10 calls after 3
    warm-up calls."""
    import numpy as np
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}

    def med(fn):
        return median_call_ms(torch, fn)

    for ln in (16, 20, 24):
        n = 1 << ln
        rp = mgp.PrefixResampler(n)
        rm = mgp.Resampler(n)
        anc = torch.empty(n, dtype=torch.int32, device=dev)
        for y in (0, 2, 4):
            w = torch.from_numpy(inputs.gaussian_weights(n, float(y), 0)).to(dev)
            row = {}
            for method in ("multinomial", "systematic"):
                row[method + "_ms"] = med(lambda k: rp.resample(w, method, seed=k, out=anc))
            row["megopolis_ms"] = med(lambda k: rm.resample(w, "megopolis", epsilon=0.01, seed=k, out=anc))
            row["megopolis_B"] = rm.last_stats()["B"]
            row["speedup_vs_multinomial"] = row["multinomial_ms"] / row["megopolis_ms"]
            row["speedup_vs_systematic"] = row["systematic_ms"] / row["megopolis_ms"]
            out[f"2^{ln}_y{y}"] = row
            del w
        del rp, rm, anc
    log("[bench] prefix-sum methods: " + "; ".join(
        f"{k} mult {v['multinomial_ms']:.3f} syst {v['systematic_ms']:.3f} mego {v['megopolis_ms']:.3f} ms"
        for k, v in out.items()))
    return {"workload": "Gaussian-likelihood weights, eps=0.01 for Megopolis; whole resample calls, ancestors only, "
                        "median of 10 after 3 warm-up calls", "rows": out}


def m_neq_n_section(torch, mgp, inputs):
    """M != N resampling (Section 8's D-PMC remark): Megopolis, B from
    eps = 0.01 on Gaussian-likelihood weights with y = 4, N inputs -> M
    outputs for (2^24 -> 2^22) and (2^22 -> 2^24); whole mgp_resample_m call
    (reduction, B, offsets, accept loop), median of 10 after 3 warm-up calls."""
    import numpy as np
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = {}
    for ln, lm in ((24, 22), (22, 24)):
        n, m = 1 << ln, 1 << lm
        w = torch.from_numpy(inputs.gaussian_weights(n, 4.0, 0)).to(dev)
        anc = torch.empty(m, dtype=torch.int32, device=dev)
        r = mgp.Resampler(n)
        ms = median_call_ms(torch, lambda k: r.resample_m(w, m, "megopolis", epsilon=0.01, seed=k, out=anc))
        B = r.last_stats()["B"]
        out[f"n2^{ln}_m2^{lm}"] = {"ms": ms, "B": B, "outputs_per_s": m / (ms * 1e-3),
                                   "kernel": "mirrored" if m <= n else "generic",
                                   "effective_GBs": 4.0 * m * (B + 2) / (ms * 1e-3) / 1e9}
        del w, anc, r
    return {"workload": "Megopolis, Gaussian-likelihood weights y=4, eps=0.01; N inputs -> M outputs", "runs": out}


def serving_section(torch, mgp, inputs, n_requests, streams=4, max_batch=8, max_particles=1 << 22):
    """Poisson stream of requests, N = round(2^U(12, 22)), y ~ U[0, 4], D = 16
    states resident on the device, Megopolis, admitted by HBM budget. The
    arrival rate is 70% of the capacity measured with all requests queued at
    once; a second run with a 2 GB budget forces queueing; a third at 10% of
    capacity gives the latency with little queueing."""
    import threading

    import numpy as np
    dev = torch.device("cuda:0")
    switch = sys.getswitchinterval()
    sys.setswitchinterval(5e-5)  # the collector must not wait 5 ms for the GIL
    sets = 48
    g = np.random.Generator(np.random.PCG64(inputs.SERVE_SEED))
    sizes = np.rint(2.0 ** g.uniform(12.0, 22.0, sets)).astype(int)
    ys = g.uniform(0.0, 4.0, sets)
    pool = []
    for k, (n, y) in enumerate(zip(sizes, ys)):
        w, st = inputs.gaussian_weights_and_states(int(n), float(y), 16, 3000 + k)
        pool.append((torch.from_numpy(w).to(dev), torch.from_numpy(st).to(dev)))
    torch.cuda.synchronize()

    def run(budget, rate, count, open_loop=True):
        srv = mgp.Server("megopolis", d=16, hbm_budget=budget, streams=streams, max_batch=max_batch,
                         max_batch_particles=max_particles)
        arrivals = np.cumsum(np.random.Generator(np.random.PCG64(7)).exponential(1.0 / rate, count)) if open_loop \
            else np.zeros(count)
        tickets = [None] * count
        ready = threading.Semaphore(0)

        def submitter():
            # pace arrivals by sleeping (which releases the GIL for the
            # collector) and spin only the last ~30 us of each gap
            t0 = time.perf_counter()
            for k in range(count):
                gap = arrivals[k] - (time.perf_counter() - t0)
                if gap > 50e-6:
                    time.sleep(gap - 30e-6)
                while time.perf_counter() - t0 < arrivals[k]:
                    pass
                w, st = pool[k % sets]
                tickets[k] = srv.submit(w, seed=10_000 + k, stream_id=k, states=st)
                ready.release()

        th = threading.Thread(target=submitter)
        w0 = time.perf_counter()
        th.start()
        lat, parts = [], 0
        for k in range(count):
            ready.acquire()
            r = srv.wait(tickets[k], 120000.0)
            assert r["state"] == 2
            lat.append((r["t_done"] - r["t_submit"]) * 1000.0)
            parts += r["n"]
            srv.release(tickets[k])
        th.join()
        wall = time.perf_counter() - w0
        st = srv.stats()
        srv.close()
        return {"requests": count, "wall_s": wall, "particles_per_s": parts / wall,
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(np.mean(lat)),
                "micro_batches": st["micro_batches"], "pool_peak_bytes": st["pool_peak"],
                "max_concurrent_batches": st["max_concurrent_batches"]}

    cap = run(16 << 30, 1.0, 400, open_loop=False)
    mean_n = float(np.mean(sizes))
    capacity_rps = cap["particles_per_s"] / mean_n
    rate = 0.7 * capacity_rps
    main_run = run(16 << 30, rate, n_requests)
    tight = run(2 << 30, rate, max(500, n_requests // 4))
    # at 10% of capacity requests rarely wait for one another: the latency
    # is close to the service time of a request alone
    light = run(16 << 30, 0.1 * capacity_rps, 500)
    sys.setswitchinterval(switch)
    return {"workload": "Poisson requests, N=round(2^U(12,22)), y~U[0,4], D=16 states resident, Megopolis, "
                        f"{streams} streams, micro-batches <= {max_batch} requests / {max_particles} particles",
            "capacity_particles_per_s": cap["particles_per_s"], "capacity_requests_per_s": capacity_rps,
            "arrival_rate_per_s": rate, "budget_16GB": main_run, "budget_2GB": tight, "load_10pct": light}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library resamples on one GPU (the multi-GPU design is not built)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2109_13504_amd import inputs, mgp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mgp.lib()
    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    log(f"[bench] generating inputs N=2^{args.log2n} y={args.y} D={args.d}")
    w_np, st_np = inputs.gaussian_weights_and_states(n, args.y, args.d, 0)
    w = torch.from_numpy(w_np).to(dev)
    states = torch.from_numpy(st_np).to(dev)
    del st_np
    anc = torch.empty(n, dtype=torch.int32, device=dev)
    out = torch.empty((n, args.d), dtype=torch.float32, device=dev)
    r = mgp.Resampler(n)
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    log(f"[bench] {args.variant}: warmup {args.warmup}, steps {args.steps}")
    ms, per = timed_steps(torch, mgp, r, w, states, anc, out, args.variant, args.eps, args.steps, args.warmup, 0)
    st = r.last_stats()
    B = st["B"]
    assert st["status"] == 0
    d = args.d
    fused_ms = float(np.mean(per["loop"]))
    # what the fused kernel must move per launch: B candidate weights, the
    # particle's own weight, the ancestor write, and the state row read and
    # written (the gather's ancestor re-read is gone)
    fused_bytes = 4.0 * n * B + 4.0 * n + 4.0 * n + 8.0 * n * d
    achieved = fused_bytes / (fused_ms * 1e-3) / 1e9
    step_bytes = 4.0 * n + fused_bytes
    log(f"[bench] {args.variant}: {ms:.3f} ms/step, loop + copy {fused_ms:.3f} ms, B={B}, {achieved:.0f} GB/s")

    # the same step unfused (accept loop, then mgp_gather), for the loop-only
    # rate of 4 N B weight bytes and the saving of the fusion
    ms_u, per_u = timed_steps(torch, mgp, r, w, states, anc, out, args.variant, args.eps, max(1, args.unfused_steps),
                              1, 500, fused=False)
    loop_ms = float(np.mean(per_u["loop"]))
    loop_bytes = 4.0 * n * B
    log(f"[bench] unfused: {ms_u:.3f} ms/step, loop {loop_ms:.3f} ms, gather {float(np.mean(per_u['gather'])):.3f} ms")

    ceil = None if args.no_ceiling else ceiling_section(torch, mgp)
    mall = ceil["infinity_cache_read_GBs"] if ceil else float("nan")
    hbm = ceil["hbm_read_GBs"] if ceil else float("nan")
    pat = float("nan")
    if ceil and n % 1024 == 0 and B >= 5:
        ceil["megopolis_pattern_read"] = pattern_ceiling(torch, mgp, n, 5 * (B // 5))
        pat = ceil["megopolis_pattern_read"]["GBs"]
    kernel = {"megopolis": f"k_megopolis_mirror<4, {d // 4 if d % 4 == 0 and d <= 16 else -1}>",
              }.get(args.variant, f"k_resample<{args.variant}>")

    result = {
        "metric": METRIC,
        "value": n / (ms * 1e-3),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"single filter, N=2^{args.log2n}, Gaussian-likelihood weights y={args.y:g}, "
                               f"eps={args.eps:g} (B={B}), {args.variant}, with the particle copy of D={d} fp32 "
                               f"states fused into the accept loop",
                   "n": n, "y": args.y, "eps": args.eps, "B": B, "d": d, "variant": args.variant,
                   "step": "mgp_compute_B + mgp_resample_gather_prepared"},
        "p50_ms": pct(per["total"], 50),
        "p99_ms": pct(per["total"], 99),
        "phase_ms": {"reduce_B": float(np.mean(per["reduce_B"])), "loop_and_copy": fused_ms,
                     "total": float(np.mean(per["total"]))},
        "hbm_frac_effective": (step_bytes / (ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
        "roofline": {
            "kernel": f"{kernel} (accept loop with the particle copy as its epilogue)",
            "bound": "hbm",
            "level": "memory side of the fabric: the 128 MB weight mirror streams from the 256 MB Infinity Cache "
                     "in front of HBM; the state rows come from and go to HBM",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "bytes_formula": "4NB candidate weights + 4N own weight + 4N ancestor + 8ND state row in and out",
            "algorithmic_bytes_per_launch": fused_bytes,
            "avg_launch_ms": fused_ms,
            "ceiling": {"infinity_cache_read_GBs": mall, "frac_of_infinity_cache_read": achieved / mall,
                        "hbm_read_GBs": hbm,
                        "megopolis_pattern_read_GBs": pat, "frac_of_pattern_read": achieved / pat,
                        "what": "mgp_probe_stream_read in this run: the best streaming-read rate over buffers of "
                                "64-256 MB (Infinity Cache resident) and at 1-2 GB (HBM); mgp_probe_pattern_read: "
                                "the loop's candidate reads alone at this n and B rounded down to whole rounds "
                                "of five steps"},
            "traffic": None,
            "traffic_what": "bytes past the L2 (TCC to fabric: Infinity Cache or HBM), calibrated FETCH_SIZE + "
                            "WRITE_SIZE per launch",
        },
        "loop_only": {"kernel": "k_megopolis_mirror<4, 0> (accept loop, unfused step)" if args.variant == "megopolis"
                      else f"k_resample<{args.variant}>",
                      "ms": loop_ms, "bytes_formula": "4NB candidate weights", "bytes": loop_bytes,
                      "GBs": loop_bytes / (loop_ms * 1e-3) / 1e9,
                      "frac_of_hbm_peak": loop_bytes / (loop_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "frac_of_infinity_cache_read": loop_bytes / (loop_ms * 1e-3) / 1e9 / mall,
                      "frac_of_pattern_read": loop_bytes / (loop_ms * 1e-3) / 1e9 / pat},
        "unfused": {"ms_per_step": ms_u, "loop_ms": loop_ms, "gather_ms": float(np.mean(per_u["gather"])),
                    "gather_GBs": 4.0 * n * (2 * d + 1) / (float(np.mean(per_u["gather"])) * 1e-3) / 1e9,
                    "fused_saving_ms": ms_u - ms},
        "memory_ceilings": ceil,
    }

    if os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("source_hash") == source_hash() and t.get("n") == n and t.get("B") == B and t.get("d") == d:
            result["roofline"]["traffic"] = t["bytes_per_launch"]

    if not args.no_metropolis and args.variant != "metropolis":
        log(f"[bench] metropolis: {args.metropolis_steps} steps")
        ms_m, per_m = timed_steps(torch, mgp, r, w, states, anc, out, "metropolis", args.eps,
                                  args.metropolis_steps, 1, 0)
        lm = float(np.mean(per_m["loop"]))
        result["metropolis"] = {"value": n / (ms_m * 1e-3), "unit": "particles/s", "ms_per_step": ms_m,
                                "loop_and_copy_ms": lm,
                                "effective_GBs": fused_bytes / (lm * 1e-3) / 1e9,
                                "p99_ms": pct(per_m["total"], 99),
                                "step": "mgp_compute_B + mgp_resample_gather_prepared, as for Megopolis"}
        result["speedup_vs_metropolis"] = ms_m / ms
        log(f"[bench] metropolis: {ms_m:.3f} ms/step, loop + copy {lm:.3f} ms -> speedup {ms_m / ms:.2f}x")

    if args.variant == "megopolis" and not args.no_segment64:
        ms_s, per_s = timed_steps(torch, mgp, r, w, states, anc, out, "megopolis", args.eps, 5, 1, 0, segment=64)
        ls = float(np.mean(per_s["loop"]))
        result["megopolis_segment64"] = {"ms_per_step": ms_s, "loop_and_copy_ms": ls,
                                         "effective_GBs": fused_bytes / (ls * 1e-3) / 1e9,
                                         "workload": "the same step with 64-wide Megopolis segments"}
        log(f"[bench] megopolis, 64-wide segments: {ms_s:.3f} ms/step, loop {ls:.3f} ms")

    if not args.no_batched:
        log("[bench] batched: 512 filters")
        shape = tuple(int(v) for v in args.batch_shape.split(",")) if args.batch_shape else None
        result["batched"] = batched_section(torch, mgp, inputs, args.batch_runs, shape)
        bt = result["batched"]
        log(f"[bench] batched: graph {bt['graph_ms']:.3f} ms/run, separate {bt['separate_ms']:.3f} ms/run "
            f"-> {bt['speedup_vs_separate']:.2f}x, shape {bt['tuned_shape']}")

    if not args.no_sweep:
        log("[bench] per-variant sweep at N=2^22")
        result["paper_sweep"] = sweep_section(torch, mgp, inputs)
        log("[bench] configurations N=4096 and N=2^20")
        result["configs"] = configs_section(torch, mgp, inputs)
        c2 = result["configs"]["n2pow20"]["ms"]
        log("[bench] N=2^20 resample ms, y=0..4: " + "; ".join(
            f"{v} " + "/".join(f"{c2[v][f'y{y}']['resample_ms']:.3f}" for y in range(5)) for v in c2))
        log("[bench] N sweep")
        result["n_sweep"] = n_sweep_section(torch, mgp, inputs)
        log("[bench] " + ", ".join(f"{k}: {v['ms']:.3f} ms" for k, v in result["n_sweep"]["rows"].items()))
        log("[bench] M != N")
        result["m_neq_n"] = m_neq_n_section(torch, mgp, inputs)

        log(f"[bench] M != N: {result['m_neq_n']['runs']}")

    if not args.no_prefix:
        log("[bench] prefix-sum methods")
        result["prefix_sum_methods"] = prefix_section(torch, mgp, inputs)

    if not args.no_serving:
        log("[bench] serving")
        result["serving"] = serving_section(torch, mgp, inputs, args.serve_requests)
        sv = result["serving"]["budget_16GB"]
        log(f"[bench] serving: p50 {sv['p50_ms']:.3f} ms, p99 {sv['p99_ms']:.3f} ms, "
            f"{sv['particles_per_s']:.3e} particles/s; at 10% load p50 "
            f"{result['serving']['load_10pct']['p50_ms']:.3f} ms, p99 {result['serving']['load_10pct']['p99_ms']:.3f} ms")

    if not args.no_sir:
        rows = [("megopolis", 16)]
        if args.sir_table:
            rows = [(v, b) for b in (16, 32, 64) for v in ("megopolis", "metropolis", "c1", "c2")]
            rows += [("multinomial", 0), ("systematic", 0)]  # Table 2's unbiased rows (Algorithms 7 and 8)
        if args.sir_bsweep:
            rows = [(v, b) for b in (5, 7, 10, 15, 20, 25, 30, 40) for v in ("megopolis", "metropolis", "c1", "c2")]
            rows.append(("megopolis", 0))  # B from eq. (bcalc) with epsilon = 0.1 at every step
        log(f"[bench] SIR filter: {len(rows)} configuration(s)")
        result["sir"] = sir_section(torch, mgp, inputs, rows, mc_runs=args.sir_mc_runs)

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(w_np, args.variant, args.eps, args.cpu_stride)
        log(f"[bench] cpu baseline: {result['cpu_baseline']['value']:.3e} particles/s")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
