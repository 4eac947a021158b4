#!/usr/bin/env python3
"""Benchmark of the PVFinder hot path on one MI355X, through the C ABI.

A step is one pvf_execute over one batch: FC stage + histogram, the UNet, and
peak finding, with the inputs already resident in HBM.  Default workload: the
production slice of 1000 events (Poisson(180) tracks, Poisson(5.6) vertices,
seed 0) in FP32.  Prints ONE JSON line on stdout; per-launch detail goes to
stderr.

Roofline: the dominant kernel is the kernel instance with the largest total
time; its algorithmic FLOPs per launch (2 x MACs of the layers it runs, per
event, times the events of one launch) over its average launch duration,
measured with HIP events recorded by the library on the stream the kernels
run on, against the MI355X dense FP32 matrix peak (157.3 TFLOP/s).

CPU baseline: the FP64 oracle (plain C, threads over events; rebuilt for
this host's CPU when gcc is there) on a bounded sample of the same batch, on
the host cores this process may use (its affinity set, capped by
OMP_NUM_THREADS when that names the process's CPU share).

The same line also carries, measured in the same run: the BF16, FP16 and FP8
paths on the same batch (other_dtypes), the heavy-tailed 4096-event BF16
batch run as one captured HIP graph with autotuned tiles (heavy_tailed), and
a short continuous-batching serving pass in FP32 and BF16 (serving).
"""

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "events/sec on 1 MI355X (FP32 vs BF16/FP8 at stated tol); p99 µs/event"
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "fp8_e4m3": 5000.0}
DTYPE_TAG = {"fp32": "f32", "bf16": "bf16", "fp16": "f16", "fp8_e4m3": "fp8_e4m3"}
HBM_PEAK_GBS = 8000.0
# error bounds against the FP64 oracle that the GPU tests enforce for each
# reduced-precision path (max |p - p_ref|; vertices matched within 0.05 mm)
STATED_TOL = {"bf16": {"max_abs_dp": 2e-2, "vertices_matched_min": 0.995, "extra_vertices_max": 0.005},
              "fp16": {"max_abs_dp": 5e-3, "vertices_matched_min": 0.999, "extra_vertices_max": 0.001},
              "fp8_e4m3": {"max_abs_dp": 0.3, "vertices_matched_min": 0.95, "extra_vertices_max": 0.05}}
# the heavy-tailed batch (log-normal track counts up to 1500) in BF16
STATED_TOL_HEAVY = {"bf16": {"max_abs_dp": 0.22, "vertices_matched_min": 0.95, "extra_vertices_max": 0.005}}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {"conv_mfma_f32": "conv_kernel.hip", "conv_mfma_lp": "conv_lp_kernel.hip",
                  "track_stage": "track_kernel.hip", "peak_finder": "peaks_kernel.hip",
                  "conv_mfma_fp8": "conv_fp8_kernel.hip", "first_conv": "aux_kernels.hip"}


def kernel_source_sha(kernel_name):
    """sha256 of the source file that defines `kernel_name` (counters taken on
    an older version of a kernel are not reported for the current one)."""
    import hashlib
    for prefix, f in KERNEL_SOURCES.items():
        if kernel_name.startswith(prefix):
            path = os.path.join(ROOT, "paper_2602_19959_amd", "csrc", f)
            return hashlib.sha256(open(path, "rb").read()).hexdigest()
    return None


def units(spec):
    """UNet sequences per event: 1, or the interval count (interval layout)."""
    return spec.n_bins // spec.bins_per_interval if spec.unet_layout == 1 else 1


def layer_macs(spec, n_hidden=6, hidden=20, n_feat=9):
    """Algorithmic multiply-adds per event of each launch, in launch order
    (the track stage's figure is per network evaluation of one track)."""
    n, c0, U = spec.n_levels, spec.base_channels, units(spec)
    L0 = spec.n_bins // U
    out = {"track": n_feat * hidden + (n_hidden - 1) * hidden * hidden + hidden * spec.bins_per_interval}
    for l in range(n):
        L, C = L0 >> l, c0 << l
        cin = 1 if l == 0 else (c0 << (l - 1))
        out[f"enc{l}.c1"] = L * C * cin * 5
        out[f"enc{l}.c2"] = L * C * C * 5
    for l in range(n - 2, -1, -1):
        L, C = L0 >> l, c0 << l
        out[f"up{l}"] = L * C * (2 * C)
        out[f"dec{l}.c1"] = L * C * 2 * C * 5
        key = "dec0.c2+head" if l == 0 else f"dec{l}.c2"
        out[key] = L * C * C * 5 + (L * C if l == 0 else 0)
    out["peaks"] = 0
    return {k: (v * U if k != "track" else v) for k, v in out.items()}


def layer_bytes(spec, eb):
    """Algorithmic HBM bytes per event of each launch: every input activation
    read once, every output written once (eb bytes per element, the compute
    dtype; the histogram and the probability are FP32).  The track stage's
    figure is per track for its input (36 B) plus the histogram write."""
    n, c0, U = spec.n_levels, spec.base_channels, units(spec)
    L0 = spec.n_bins // U
    out = {"track": None, "enc0.c1": L0 * 4 + L0 * c0 * eb}
    for l in range(n):
        L, C = L0 >> l, c0 << l
        if l > 0:
            out[f"enc{l}.c1"] = L * (c0 << (l - 1)) * eb + L * C * eb
        out[f"enc{l}.c2"] = L * C * eb + L * C * eb + ((L // 2) * C * eb if l < n - 1 else 0)
    for l in range(n - 2, -1, -1):
        L, C = L0 >> l, c0 << l
        out[f"up{l}"] = (L // 2) * (2 * C) * eb + L * C * eb
        out[f"dec{l}.c1"] = L * 2 * C * eb + L * C * eb
        out["dec0.c2+head" if l == 0 else f"dec{l}.c2"] = L * C * eb + (L * 4 if l == 0 else L * C * eb)
    out["peaks"] = L0 * 4
    return {k: (v * U if v is not None else v) for k, v in out.items()}


def layer_bytes_between(spec, eb, first):
    """Bytes per event of the tensor that launch `first` stores for the
    launch after it (the one a fusion keeps out of HBM)."""
    n, c0, U = spec.n_levels, spec.base_channels, units(spec)
    L0 = spec.n_bins // U
    if first == "enc0.c1":
        return L0 * c0 * eb * U
    l = int(first[3])                      # "decL.c2"
    return (L0 >> l) * (c0 << l) * eb * U


def cpu_threads():
    """(threads to use, affinity size, OMP_NUM_THREADS or None): every core
    of this process's affinity set, unless OMP_NUM_THREADS names a smaller
    CPU share for the process."""
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    share = int(omp) if omp and omp.isdigit() and int(omp) > 0 else None
    return max(1, min(aff, share) if share else aff), aff, share


def native_oracle():
    """Build the oracle for this host's CPU (-march=native, same source and
    otherwise the same flags: no fast-math, no contraction, so the same
    results) into a temporary directory and point the oracle module at it.
    Returns the flags used; the shipped build stays in use if gcc fails."""
    import subprocess
    import tempfile
    from oracle import build as ob
    d = tempfile.mkdtemp(prefix="pvf_oracle_native_")
    lib = os.path.join(d, "libpvf_oracle_native.so")
    cmd = ["gcc", "-std=c11", "-O2", "-march=native", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-o", lib, ob.SRC, "-lm"]
    try:
        subprocess.run(cmd, check=True, capture_output=True, timeout=120)
    except (OSError, subprocess.SubprocessError):
        return "shipped build (-O2)"
    os.environ["PVF_ORACLE_LIB"] = lib
    return "-O2 -march=native -ffp-contract=off"


def cpu_baseline(batch, w, target_s):
    flags = native_oracle()
    import oracle
    threads, aff, share = cpu_threads()
    t0 = time.perf_counter()
    oracle.run_batch(batch.subset([0]), w, threads=1)
    t_one = time.perf_counter() - t0
    n = int(max(threads, min(batch.n_events, round(target_s * threads / max(t_one, 1e-3)))))
    n = min(n, batch.n_events)
    sub = batch.subset(range(n))
    t0 = time.perf_counter()
    oracle.run_batch(sub, w, threads=threads)
    dt = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu, "cpu_count": os.cpu_count(), "affinity_cores": aff, "omp_num_threads": share,
            "build": flags,
            "sample": f"first {n} events of the same batch, FP64 C oracle ({flags}), {threads} threads "
                      f"(affinity {aff} cores, OMP_NUM_THREADS {share}), {dt:.1f} s wall on {cpu}"}


def fp8_calibration_table(pv, blob, n_events, seed, mix, variant=None):
    """Set-up, outside every timed region: per-channel scales for an FP8
    engine from an FP32 run over other events."""
    import numpy as np
    from synth import make_events
    cb = make_events(n_events, seed=seed, mix=mix)
    CT = np.diff(cb.offsets)
    cspec = pv.default_spec(max_events=cb.n_events, max_tracks_total=int(max(CT.sum(), 1)),
                            max_tracks_per_event=max(1500, int(CT.max())), **(variant or {}))
    ceng = pv.Engine(blob, cspec)
    cf, co = pv.upload_events(cb)
    amax = ceng.calibrate(cf, co)
    ceng.close()
    return amax


def serve_pass(dtype, blob, pool_events, n_requests, loads, seed, pool_gb=8.0, lanes=2, results="host",
               warm=False, amax=None):
    """Continuous-batching serving of one dtype: capacity with every request
    queued at once, then Poisson arrivals at the given fractions of that
    capacity.  Requests arrive with their features in page-locked host
    memory; the consumer callback takes each request's results where the
    server leaves them (results="host": page-locked host blocks; "device":
    HBM) and drops them."""
    import numpy as np
    from paper_2602_19959_amd.serve import Server, poisson_requests

    srv = Server(blob, pool_bytes=int(pool_gb * (1 << 30)), lanes=lanes, compute_dtype=dtype, fp8_amax=amax,
                 results=results)
    print(f"[serve] {dtype} pool {pool_gb} GB, {lanes} lanes x {srv.lane_events} events, results on {results}",
          file=sys.stderr, flush=True)
    consume = lambda r: None
    if warm:
        # steady state of a long-running server (allocator caches filled)
        srv.run(poisson_requests(1e9, n_requests, seed + 7, pool_events, pinned=True), realtime=False,
                on_complete=consume)
    reqs = poisson_requests(1e9, n_requests, seed + 8, pool_events, pinned=True)
    cap = srv.run(reqs, realtime=False, on_complete=consume).summary()
    print(f"[serve] {dtype} capacity {cap['events_per_s']:.0f} events/s", file=sys.stderr, flush=True)
    mean_size = float(np.mean([r.n_events for r in reqs]))
    out = {"capacity": cap, "lane_events": srv.lane_events, "results_on": results, "loads": {}}
    for f in loads:
        rate = f * cap["events_per_s"] / mean_size
        rq = poisson_requests(rate, n_requests, seed + 9, pool_events, pinned=True)
        out["loads"][f"{f:.2f}"] = dict(srv.run(rq, realtime=True, on_complete=consume).summary(),
                                        offered_requests_per_s=rate)
        print(f"[serve] {dtype} load {f:.2f}: {out['loads'][f'{f:.2f}']}", file=sys.stderr, flush=True)
    srv.close()
    return out


def serve_bench(args):
    """Continuous-batching serving: capacity with every request queued at
    once, then Poisson arrivals at fractions of that capacity."""
    import paper_2602_19959_amd as pv
    from synth import make_events, make_weights, weights_to_blob

    blob = weights_to_blob(make_weights(args.seed))
    pool_events = make_events(8000, seed=args.seed + 1, mix="lognormal")
    amax = (fp8_calibration_table(pv, blob, args.calib_events, args.seed + 5, "lognormal")
            if args.dtype == "fp8_e4m3" else None)
    res = serve_pass(args.dtype, blob, pool_events, args.serve_requests,
                     [float(x) for x in args.serve_loads.split(",")], args.seed, args.pool_gb, args.lanes,
                     args.results, warm=args.serve_warm, amax=amax)
    cap = res["capacity"]
    print(json.dumps({
        "metric": METRIC, "value": cap["events_per_s"], "unit": "events/s", "n_gpus": 1,
        "higher_is_better": True, "dtype": DTYPE_TAG[args.dtype], "data": "synthetic",
        "config": {"workload": f"serving: slices of U{{100..2000}} events (log-normal track counts), "
                               f"Poisson arrivals, {args.pool_gb} GB HBM pool, {args.lanes} lanes of "
                               f"{res['lane_events']} events, continuous batching, results on {args.results}",
                   "requests": args.serve_requests, "warm_pass": bool(args.serve_warm)},
        "capacity": cap, "loads": res["loads"],
        "budget_us_per_event": 400.0,
    }), flush=True)


def heavy_tailed_pass(args, blob):
    """The heavy-tailed batch in BF16 as a batching configuration: 4096 events
    with log-normal track counts (median 180, clipped to [5, 1500]), the
    work-queue track stage, tile variants picked by the autotuner on this
    batch, the whole path captured as one HIP graph; K graph replays timed
    with HIP events on the engine's stream."""
    import numpy as np
    import torch
    import paper_2602_19959_amd as pv
    from synth import make_events

    E = 4096
    batch = make_events(E, seed=args.seed, mix="lognormal")
    T = np.diff(batch.offsets)
    spec = pv.default_spec(max_events=E, max_tracks_total=int(T.sum()), compute_dtype="bf16",
                           max_tracks_per_event=max(1500, int(T.max())))
    eng = pv.Engine(blob, spec)
    eng.set_track_schedule(True)
    feat, off = pv.upload_events(batch)
    out = eng.alloc_outputs(E, with_prob=False)
    t_tune = time.perf_counter()
    eng.autotune(feat, off, out, reps=1)
    t_tune = time.perf_counter() - t_tune
    eng.graph_capture(feat, off, out)
    s = eng.stream
    for _ in range(3):
        eng.graph_launch()
    s.synchronize()
    steps = max(5, args.steps // 5)
    ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        eng.graph_launch()
        e1.record(s)
        s.synchronize()
        ms.append(e0.elapsed_time(e1))
    wall = time.perf_counter() - t0
    eng.profile(True)
    eng.execute(feat, off, out)
    s.synchronize()
    split = eng.profile_read()
    eng.profile(False)
    host = out.to_host()
    eng.close()
    if np.any(host["status"] & (pv.EV_TOO_MANY_TRACKS | pv.EV_BAD_INPUT)):
        print("[bench] unexpected bypassed events in the heavy-tailed batch", file=sys.stderr)
        sys.exit(1)
    us = sorted(m * 1e3 / E for m in ms)
    res = {"value": E * steps / wall, "unit": "events/s", "dtype": "bf16", "steps": steps,
           "ms_per_step": wall / steps * 1e3,
           "p50_us_per_event": statistics.median(us), "p99_us_per_event": us[min(len(us) - 1, int(round(0.99 * (len(us) - 1))))],
           "config": {"workload": f"{E} events, log-normal track counts (median 180, clipped to [5, 1500]; "
                                  f"mean {T.mean():.1f}, max {int(T.max())}), work-queue track stage, autotuned "
                                  f"tiles ({t_tune:.1f} s set-up), one HIP graph per step"},
           "stages_ms_eager": {"track": split[0], "unet": sum(split[1:-1]), "peaks": split[-1]},
           "stated_tolerance": STATED_TOL_HEAVY["bf16"]}
    print(f"[bench] heavy-tailed bf16 graph: {res['value']:.0f} events/s", file=sys.stderr, flush=True)
    return res


def gemm_yardstick(args):
    """Per 5-tap conv layer: this library's launch time (HIP events on the
    engine's stream) beside the vendor GEMM (torch.mm, i.e. hipBLASLt) on
    the same layer's plain GEMM, M = positions x events, N = Cout,
    K = 5 Cin, with A already unfolded in HBM (so the vendor side skips the
    halo handling a convolution needs).  A yardstick, not part of a step."""
    import numpy as np
    import torch

    import paper_2602_19959_amd as pv
    from synth import make_events, make_weights, weights_to_blob

    if args.dtype == "fp8_e4m3":
        print("--gemm-yardstick covers fp32, bf16 and fp16", file=sys.stderr)
        sys.exit(2)
    E = args.events
    batch = make_events(E, seed=args.seed, mix=args.mix)
    T = np.diff(batch.offsets)
    spec = pv.default_spec(max_events=E, max_tracks_total=int(max(T.sum(), 1)), compute_dtype=args.dtype,
                           max_tracks_per_event=max(1500, int(T.max())))
    eng = pv.Engine(weights_to_blob(make_weights(args.seed)), spec)
    feat, off = pv.upload_events(batch)
    out = eng.alloc_outputs(E, with_prob=False)
    eng.profile(True)
    names, kernels = eng.launch_names(), eng.launch_kernels()
    runs = []
    for r in range(args.warmup + args.steps):
        eng.execute(feat, off, out)
        eng.synchronize()
        if r >= args.warmup:
            runs.append(eng.profile_read())
    ours = np.median(np.array(runs), axis=0)
    eng.close()
    macs = layer_macs(spec)
    tdt = {"fp32": torch.float32, "bf16": torch.bfloat16, "fp16": torch.float16}[args.dtype]
    torch.backends.cuda.matmul.allow_tf32 = False
    c0 = spec.base_channels
    rows = []
    for i, nm in enumerate(names):
        if not (nm.startswith("enc") or nm.startswith("dec")) or nm == "enc0.c1" or nm not in macs:
            continue
        lvl = int(nm[3])
        L, C = spec.n_bins >> lvl, c0 << lvl
        if nm.startswith("enc"):
            cin = (c0 << (lvl - 1)) if nm.endswith("c1") else C
        else:
            cin = 2 * C if nm.endswith("c1") else C
        M, N, K = L * E, C, 5 * cin
        g = torch.Generator(device="cuda").manual_seed(1)
        a = torch.randn(M, K, device="cuda", dtype=tdt, generator=g)
        b = torch.randn(K, N, device="cuda", dtype=tdt, generator=g)
        c = torch.empty(M, N, device="cuda", dtype=tdt)
        for _ in range(3):
            torch.mm(a, b, out=c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            torch.mm(a, b, out=c)
        e1.record()
        torch.cuda.synchronize()
        vend = e0.elapsed_time(e1) / args.steps
        del a, b, c
        fl = 2.0 * M * N * K
        # a layer fused into another launch has no time of its own: its work
        # is inside the host launch's figure, so it counts zero here
        fused = kernels[i].startswith("conv (in")
        t_ours = 0.0 if fused else float(ours[i]) * 1e3
        rows.append({"layer": nm, "M": M, "N": N, "K": K, "kernel": kernels[i],
                     "ours_us": round(t_ours, 1), "vendor_gemm_us": round(vend * 1e3, 1),
                     "ours_tflops": None if fused else round(fl / (t_ours * 1e6), 1),
                     "vendor_gemm_tflops": round(fl / (vend * 1e9), 1)})
        print(f"[yardstick] {rows[-1]}", file=sys.stderr, flush=True)
    tot_o = sum(r["ours_us"] for r in rows)
    tot_v = sum(r["vendor_gemm_us"] for r in rows)
    print(json.dumps({"yardstick": "vendor GEMM (torch.mm -> hipBLASLt) on each 5-tap conv layer's GEMM shape",
                      "dtype": DTYPE_TAG[args.dtype], "events": E, "layers": rows,
                      "sum_ours_us": round(tot_o, 1), "sum_vendor_gemm_us": round(tot_v, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--events", type=int, default=1000)
    ap.add_argument("--mix", default="poisson", choices=["poisson", "lognormal"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--dtype", default="fp32", choices=["fp32", "bf16", "fp16", "fp8_e4m3"])
    ap.add_argument("--width", type=int, default=32, choices=[32, 64],
                    help="UNet base channels (64 = the paper's deployed width)")
    ap.add_argument("--levels", type=int, default=None, help="UNet levels (default 4; 3 with --layout interval)")
    ap.add_argument("--layout", default="event", choices=["event", "interval"],
                    help="one UNet sequence per event, or per 100-bin interval")
    ap.add_argument("--boundary-mm", type=float, default=0.0,
                    help="boundary tracks closer than this to a shared interval edge also feed the neighbour")
    ap.add_argument("--calib-events", type=int, default=256,
                    help="FP8: events (seed + 5) of the FP32 calibration run that sets the channel scales")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", default="queue", choices=["queue", "block"],
                    help="track stage: persistent work queue (default) or one block per event")
    ap.add_argument("--graph", action="store_true",
                    help="time replays of one captured HIP graph (per-launch times then come from an "
                         "eager pass after the timed region)")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: Poisson arrivals of event slices into a fixed HBM pool "
                         "with continuous batching; prints one JSON line with latency percentiles per load")
    ap.add_argument("--serve-requests", type=int, default=60)
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95")
    ap.add_argument("--pool-gb", type=float, default=8.0)
    ap.add_argument("--lanes", type=int, default=2)
    ap.add_argument("--results", default="host", choices=["host", "device"],
                    help="serving: results back to page-locked host memory, or left in HBM for device consumers")
    ap.add_argument("--serve-warm", action="store_true",
                    help="serving: a first, untimed pass of the same size before the measured ones")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="default run: skip the heavy-tailed graph pass and the short serving pass")
    ap.add_argument("--autotune", action="store_true",
                    help="time every tile variant per launch first and keep the fastest (the built-in "
                         "defaults are the picks of such sweeps on this workload)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-compare-dtypes", dest="compare_dtypes", action="store_false",
                    help="FP32 runs only: skip the BF16 and FP8 passes on the same batch")
    ap.add_argument("--gemm-yardstick", action="store_true",
                    help="instead: per 5-tap conv layer, this library's launch time beside the vendor GEMM "
                         "(torch.mm) of the same GEMM shape; one JSON line")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size kernel "
                         "for scaling hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the path shards by event with no collective, so a "
              "multi-GPU figure is the one-GPU value times N; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2602_19959_amd as pv
    from synth import make_events, make_weights, weights_to_blob

    if not torch.cuda.is_available():
        print("bench.py needs an MI355X", file=sys.stderr)
        sys.exit(1)
    if args.serve:
        serve_bench(args)
        return
    if args.gemm_yardstick:
        gemm_yardstick(args)
        return
    E = args.events
    from synth import NetShape
    levels = args.levels or (3 if args.layout == "interval" else 4)
    shape = NetShape(n_levels=levels, base_channels=args.width)
    batch = make_events(E, seed=args.seed, mix=args.mix)
    w = make_weights(args.seed, shape=shape)
    T = np.diff(batch.offsets)
    variant = dict(n_levels=levels, base_channels=args.width, unet_layout=args.layout,
                   boundary_mm=args.boundary_mm)
    def measure(dtype, copy_mib):
        """One dtype on this batch: build (and for FP8 calibrate) an engine,
        warm up, time the steps, and return (result dict, engine)."""
        spec = pv.default_spec(max_events=E, max_tracks_total=int(max(T.sum(), 1)), compute_dtype=dtype,
                               max_tracks_per_event=max(1500, int(T.max())), **variant)
        amax = None
        if dtype == "fp8_e4m3":
            # set-up, before and outside the timed region: channel scales from an
            # FP32 run over other events
            amax = fp8_calibration_table(pv, weights_to_blob(w), args.calib_events, args.seed + 5, args.mix,
                                         variant)
            print(f"[bench] FP8 calibration over {args.calib_events} events: {amax.size} channel scales",
                  file=sys.stderr, flush=True)
        eng = pv.Engine(weights_to_blob(w), spec, fp8_amax=amax)
        eng.set_track_schedule(args.schedule == "queue")
        feat, off = pv.upload_events(batch)
        out = eng.alloc_outputs(E, with_prob=False)
        names = eng.launch_names()
        if args.autotune:
            t_tune = time.perf_counter()
            picked = eng.autotune(feat, off, eng.alloc_outputs(E, with_prob=False), reps=2)
            print(f"[bench] autotuned in {time.perf_counter() - t_tune:.1f} s: "
                  + ", ".join(f"{n}={v}" for n, v in zip(names, picked) if v >= 0), file=sys.stderr, flush=True)
        kernels = eng.launch_kernels()
        print(f"[bench] E={E} mix={args.mix} tracks={int(T.sum())} arena={eng.arena_bytes / 1e9:.2f} GB "
              f"launches={len(names)}", file=sys.stderr, flush=True)

        if copy_mib > 0:
            n = copy_mib * (1 << 20) // 4
            src = torch.ones(n, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
            print(f"[bench] calibration copy of {copy_mib} MiB done", file=sys.stderr, flush=True)

        for _ in range(args.warmup):
            eng.execute(feat, off, out)
        eng.synchronize()
        torch.cuda.synchronize()

        per_launch = [[] for _ in names]
        step_ms = []
        s = eng.stream
        if args.graph:
            eng.graph_capture(feat, off, out)
            eng.graph_launch()
            eng.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(s)
                eng.graph_launch()
                ev1.record(s)
                s.synchronize()
                step_ms.append(ev0.elapsed_time(ev1))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            eng.profile(True)                       # per-launch split from eager passes
            for _ in range(3):
                eng.execute(feat, off, out)
                s.synchronize()
                for i, ms in enumerate(eng.profile_read()):
                    per_launch[i].append(ms)
            eng.profile(False)
        else:
            eng.profile(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(s)
                eng.execute(feat, off, out)
                ev1.record(s)
                s.synchronize()
                step_ms.append(ev0.elapsed_time(ev1))
                for i, ms in enumerate(eng.profile_read()):
                    per_launch[i].append(ms)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            eng.profile(False)

        host = out.to_host()
        if np.any(host["status"] & (pv.EV_TOO_MANY_TRACKS | pv.EV_BAD_INPUT)):
            print("[bench] unexpected bypassed events", file=sys.stderr)
            sys.exit(1)

        macs = layer_macs(spec)
        valid_tracks = float(T.sum())
        mean_ms = [statistics.mean(v) for v in per_launch]
        flops_launch = [2.0 * (macs[n] * valid_tracks if n == "track" else macs[n] * E) for n in names]
        eb = {"fp32": 4, "fp8_e4m3": 1}.get(dtype, 2)
        lbytes = layer_bytes(spec, eb)
        lbytes["track"] = (36.0 * valid_tracks + E * spec.n_bins * 4) / E
        # a launch that ran inside another ("first_conv (in enc0.c2)",
        # "transposed conv (in dec1.c2)"): its work is the host launch's; the
        # tensor between the two never goes through HBM
        for j, k in enumerate(kernels):
            if " (in " in k:
                i = names.index(k.split(" (in ")[1].rstrip(")"))
                flops_launch[i] += flops_launch[j]
                flops_launch[j] = 0.0
                inner = layer_bytes_between(spec, eb, names[min(i, j)])
                lbytes[names[i]] = lbytes[names[i]] + lbytes[names[j]] - 2 * inner
                lbytes[names[j]] = 0.0
        print(f"[bench] {'launch':14s} {'kernel':36s} {'ms':>8s} {'TFLOP/s':>8s}", file=sys.stderr)
        for n, k, ms, fl in zip(names, kernels, mean_ms, flops_launch):
            print(f"[bench] {n:14s} {k:36s} {ms:8.3f} {fl / ms / 1e9:8.2f}", file=sys.stderr)

        # dominant kernel instance: largest total time per step
        by_kernel = {}
        for n, k, ms, fl in zip(names, kernels, mean_ms, flops_launch):
            d = by_kernel.setdefault(k, {"ms": 0.0, "flops": 0.0, "launches": 0, "layers": []})
            d["ms"] += ms
            d["flops"] += fl
            d["launches"] += 1
            d["layers"].append(n)
        dom_name, dom = max(by_kernel.items(), key=lambda kv: kv[1]["ms"])
        avg_dur_s = dom["ms"] / dom["launches"] / 1e3
        flops_per_launch = dom["flops"] / dom["launches"]
        bytes_per_launch = sum(lbytes[n] * E for n in dom["layers"]) / dom["launches"]
        peak = PEAK_TFLOPS[dtype]
        ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)          # flop per byte
        intensity = flops_per_launch / bytes_per_launch
        if intensity >= ridge:
            bound, achieved, peak_v, unit = "mfma", flops_per_launch / avg_dur_s / 1e12, peak, "TFLOP/s"
        else:
            bound, achieved, peak_v, unit = "hbm", bytes_per_launch / avg_dur_s / 1e9, HBM_PEAK_GBS, "GB/s"
        def measured_traffic(kernel):
            """HBM bytes per launch from the committed counter passes, if they
            were taken on this kernel's current source at this batch size."""
            if not os.path.exists(TRAFFIC_FILE):
                return None
            tr = json.load(open(TRAFFIC_FILE)).get(f"{kernel}|E={E}")
            if tr and tr.get("source_sha256") == kernel_source_sha(kernel):
                return tr.get("bytes_per_launch")
            return None

        default_shape = (args.width == 32 and args.layout == "event" and levels == 4 and args.boundary_mm == 0
                         and args.mix == "poisson" and args.seed == 0)
        traffic = measured_traffic(dom_name) if default_shape else None

        stage = {"track": mean_ms[0], "unet": sum(mean_ms[1:-1]), "peaks": mean_ms[-1]}
        ms_per_step = wall / args.steps * 1e3
        us_ev = sorted(m * 1e3 / E for m in step_ms)
        p50 = statistics.median(us_ev)
        p99 = us_ev[min(len(us_ev) - 1, int(round(0.99 * (len(us_ev) - 1))))]
        unet_flops = sum(f for n, f in zip(names, flops_launch) if n not in ("track", "peaks"))
        # track stage: network evaluations of every kept track (a boundary track
        # counts once here), input bytes 36 per track plus the histogram rows
        track_ms = mean_ms[0]
        track_bytes = 36.0 * valid_tracks + E * spec.n_bins * 4
        track_traffic = measured_traffic(kernels[0]) if default_shape else None

        result = {
            "metric": METRIC,
            "value": E * args.steps / wall,
            "unit": "events/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": ms_per_step,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": DTYPE_TAG[dtype],
            "data": "synthetic: seeded events (Poisson(5.6) PVs, Poisson(180) tracks) and seeded He-init weights",
            "config": {"workload": f"{E} events per batch, {args.mix} track counts (mean {T.mean():.1f}), "
                                   f"UNet {'/'.join(str(args.width << l) for l in range(levels))} over "
                                   + ("4000 bins" if args.layout == "event" else "each 100-bin interval")
                                   + (f", boundary tracks within {args.boundary_mm} mm feed two intervals"
                                      if args.boundary_mm > 0 else "")
                                   + f", {dtype.upper()} convolutions (FP32 accumulate)"
                                   + (f", FP8 scales from {args.calib_events} calibration events" if amax is not None else "")
                                   + f", seed {args.seed}",
                       "events_per_batch": E, "tracks_total": int(T.sum()), "max_tracks": int(T.max()),
                       "track_schedule": args.schedule, "hip_graph": bool(args.graph)},
            "p50_us_per_event": p50,
            "p99_us_per_event": p99,
            "stages_ms": stage,
            "unet_tflops": unet_flops / (stage["unet"] / 1e3) / 1e12,
            "variants": dict((n, v) for n, v in zip(names, eng.variants()) if v >= 0),
            "events_per_s_median_step": E / (statistics.median(step_ms) / 1e3),
            "track_stage": {"ms": track_ms, "gflops": flops_launch[0] / track_ms / 1e6,
                            "algorithmic_gbs": track_bytes / track_ms / 1e6,
                            "measured_gbs": (track_traffic / track_ms / 1e6) if track_traffic else None},
            "roofline": {"bound": bound, "kernel": dom_name, "layers": dom["layers"],
                         "achieved": achieved, "peak": peak_v, "unit": unit, "frac": achieved / peak_v,
                         "traffic": traffic,
                         "hbm_frac": (traffic / avg_dur_s / (HBM_PEAK_GBS * 1e9)) if traffic else None,
                         "flops_per_launch": flops_per_launch,
                         "algorithmic_bytes_per_launch": bytes_per_launch, "intensity_flop_per_byte": intensity,
                         "ridge_flop_per_byte": ridge, "avg_launch_ms": avg_dur_s * 1e3},
        }
        return result, eng

    result, eng = measure(args.dtype, args.copy_calibration_mib)
    eng.close()
    if args.compare_dtypes and args.dtype == "fp32":
        # the same batch and timing in the reduced-precision paths, each with
        # the error bound the GPU tests hold it to against the FP64 oracle
        result["other_dtypes"] = {}
        for dt in ("bf16", "fp16", "fp8_e4m3"):
            r, e2 = measure(dt, 0)
            e2.close()
            result["other_dtypes"][dt] = {
                "value": r["value"], "unit": "events/s", "ms_per_step": r["ms_per_step"],
                "p50_us_per_event": r["p50_us_per_event"], "p99_us_per_event": r["p99_us_per_event"],
                "stages_ms": r["stages_ms"], "dtype": r["dtype"],
                "roofline": {k: r["roofline"][k] for k in ("bound", "kernel", "achieved", "peak", "unit", "frac",
                                                           "traffic")},
                "stated_tolerance": STATED_TOL[dt]}
            print(f"[bench] {dt}: {r['value']:.0f} events/s", file=sys.stderr, flush=True)
    default_run = (args.dtype == "fp32" and args.width == 32 and args.layout == "event" and levels == 4
                   and args.boundary_mm == 0 and args.mix == "poisson" and E == 1000)
    if args.extras and default_run:
        blob = weights_to_blob(w)
        result["heavy_tailed"] = heavy_tailed_pass(args, blob)
        pool_events = make_events(4000, seed=args.seed + 1, mix="lognormal")
        result["serving"] = {
            "workload": "slices of U{100..2000} events (log-normal track counts), 40 requests per pass, "
                        "8 GB HBM pool, 2 lanes, continuous batching, features arriving in page-locked host "
                        "memory, no warm-up pass; capacity with all requests queued, then Poisson arrivals "
                        "at 0.8 of it; latency from arrival to results in host memory",
            "budget_us_per_event": 400.0}
        for dt in ("fp32", "bf16"):
            result["serving"][dt] = serve_pass(dt, blob, pool_events, 40, [0.8], args.seed)
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (FP64 oracle)...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(batch, w, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
