"""Throughput of the structure-function path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload c2|c3|c4|c5] [--spec f32|bf16|f16] [--accum plain|kahan]
                    [--ingest device|host] [--capacity C]

Default workload (c2): 1000 uint16 frames of 1024x1024 (12-bit camera model,
Poisson noise), 50 log-spaced lags 1..500, 512 |q| rings, FP32 spectra and
plain FP32 sums. c3 is the precision workload: 4000 frames of the same model
with every lag 1..400. c5 is the differentiation workload: 256 float32
frames of 512x512 under a Hann window, lags 1, 2, 4, ..., 64, 256 rings; its
step also runs the gradient of a loss of D with respect to the frames and
the window (nfs_backward). c4 is the batching workload: 16 uint16 sequences of
frame size 256..2048 and 200..2000 frames run together (nfs_batch_*). The
frames are drawn on the GPU and are resident in
HBM before timing. One step is the whole path on that stack: reset the sums,
push the frames (normalise + 2D transform + store), accumulate the lag pairs,
bin into D(q, tau). Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frame-pairs/sec and HBM GB/s for D(q,tau), 1024^2 x 1000 frames, 1 GPU"
# MI355X published peaks: HBM3E 8 TB/s, FP32 vector 157.3 TFLOP/s (packed
# FP32 FMAs). The library's device code is built without packed FP32
# instructions, so the rate it can reach is the non-packed one derived from
# the unit counts: 256 CUs x 64 lanes x 2.4 GHz lane-instructions per
# second, 78.6 TFLOP/s counting an FMA as 2 FLOP.
HBM_PEAK_GBPS = 8000.0
FP32_PEAK_TFLOPS = 157.3
VALU_LANE_OPS = 256 * 64 * 2.4e9
FP32_NONPACKED_TFLOPS = VALU_LANE_OPS * 2 / 1e12  # 78.6


METRIC_C3 = "frame-pairs/sec for D(q,tau), 1024^2 x 4000 frames, lags 1..400, 1 GPU"
METRIC_C5 = ("frame-pairs/sec for D(q,tau) and its gradient with respect to frames and window, "
             "512^2 x 256 frames, 1 GPU")
WORKLOADS = {
    "c2": "1000 uint16 frames 1024x1024, 50 log-spaced lags 1..500, 512 |q| rings",
    "c3": "4000 uint16 frames 1024x1024, lags 1..400, 512 |q| rings",
    "c5": "256 float32 frames 512x512, Hann window, lags 1,2,4,...,64, 256 |q| rings",
    "c4": ("16 uint16 sequences, n in {256, 512, 1024, 2048}, N in [200, 2000], 32 log-spaced "
           "lags up to N/2, n/2 |q| rings, master seed 4"),
}
METRIC_C4 = ("frame-pairs/sec for D(q,tau) over 16 sequences of uneven frame size and length "
             "(batching form), 1 GPU")

# Counter summaries (profiles/): each names the sources that shape its
# kernel's memory traffic and their sha256; a figure is reported only while
# those sources are unchanged.
PAIR_COUNTERS = os.path.join(ROOT, "profiles", "pair_kernel_1000x1024_counters.md")
TRANSFORM_COUNTERS = os.path.join(ROOT, "profiles", "transform_1000x1024_counters.md")


def source_digest(rels):
    import hashlib
    h = hashlib.sha256()
    for rel in rels:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_figure(path, key):
    """Field `key` of a counter summary, or None when the summary is missing
    or the sources it lists changed since the counters were taken."""
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    fields[k.strip()] = v.strip().strip("`")
        rels = [r.strip() for r in fields["sources"].split(",")]
        if fields.get("source_sha256") != source_digest(rels):
            return None
        return float(fields[key])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=160)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer 5 times (known bytes), to scale "
                         "memory counters of the same profiler run")
    ap.add_argument("--bandwidth-probe", action="store_true",
                    help="only measure copy/read/write rates of cache-resident and "
                         "HBM-sized buffers with the library's probe kernel")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--batch-streams", type=int, default=0,
                    help="c4: time only an eager run on this many streams (for profiling)")
    ap.add_argument("--budget-gb", type=float, default=200.0,
                    help="c4: memory budget of all sequences' workspaces (rings become time "
                         "windows when the whole stacks do not fit)")
    ap.add_argument("--spec", default="f32", choices=["f32", "bf16", "f16"],
                    help="storage type of the resident spectra")
    ap.add_argument("--accum", default="plain", choices=["plain", "kahan"],
                    help="per-mode pair accumulation")
    ap.add_argument("--ingest", default="device", choices=["device", "host"],
                    help="device: frames resident in HBM before timing (the metric); host: "
                         "frames in pinned host memory, uploaded inside the timed step "
                         "through the plan's staging buffers (streaming ingest)")
    ap.add_argument("--tune", action="store_true",
                    help="tune the pair kernel's launch shape on the stack before timing")
    ap.add_argument("--capacity", type=int, default=0,
                    help="ring slots (0 = the number of frames)")
    ap.add_argument("--frames-cache", default=None,
                    help="load the stack from this .npy if it exists, else draw it and "
                         "save it there (lets profiler runs skip the generator)")
    return ap.parse_args()


def frame_pairs(N, lags):
    return sum(max(0, N - t) for t in lags)


def host_cores():
    """Host threads for the CPU baseline: the cores this process may run on,
    at most 16 (the CPU share of one GPU on the benchmark machines)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frames_gpu, cfg, n_frames):
    """Time the FP64 oracle on the first `n_frames` frames and the lags below
    n_frames, on every host core this process gets: the oracle's own
    functions, unchanged, called from a thread pool over frames (O1-O3:
    normalise, full-plane transform) and over blocks of k-rows (O4: pair
    loop), then its binning (O5-O6). NumPy releases the interpreter lock in
    its transforms and array arithmetic, so the threads run in parallel."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    lags = [t for t in cfg["lags"] if t < n_frames]
    n, nb = cfg["n"], cfg["n_bins"]
    sample = frames_gpu[:n_frames].cpu().numpy()
    cores = host_cores()
    t0 = time.perf_counter()
    spec = np.empty((n_frames, n, n), dtype=np.complex128)

    def transform(t):
        spec[t] = oracle.spectra(oracle.normalise(sample[t:t + 1])[0])[0]

    P = np.empty((len(lags), n, n), dtype=np.float64)
    rows = max(1, n // (4 * cores))

    def pairs(r0):
        P[:, r0:r0 + rows] = oracle.pair_power(spec[:, r0:r0 + rows], lags)[0]

    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(transform, range(n_frames)))
        list(ex.map(pairs, range(0, n, rows)))
    bidx = oracle.bin_index(n, nb)
    D = oracle.azimuthal_average(P, bidx, nb)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(D))
    fp = frame_pairs(n_frames, lags)
    return {"value": fp / dt, "unit": "frame-pairs/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": (f"first {n_frames} frames of the timed stack, the {len(lags)} of its "
                       f"lags below {n_frames} ({fp} frame-pairs), {nb} rings: FP64 NumPy "
                       f"full-plane oracle (its functions unchanged) on {cores} threads over "
                       f"frames and k-row blocks, {dt:.1f} s")}


def copy_calibration():
    """Five device-to-device copies of 1 GiB: 1 GiB read and 1 GiB written each."""
    import torch
    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": n, "copy_bytes_written_per_launch": n,
                      "launches": 5}))


def bandwidth_probe(args):
    """Copy, read and write rates of the library's probe kernel over buffers
    that fit the 256 MB Infinity Cache (16..128 MiB) and over ones that do
    not (1 and 4 GiB): separates the cache-resident rate from the HBM rate.
    Each size and mode: 5 warm-up passes, then the median of 20 event-timed
    passes."""
    import statistics
    import torch
    import paper_1209_3362_amd as nfs
    out = {}
    for mib in (16, 32, 64, 128, 1024, 4096):
        nbytes = mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for mode, name in ((0, "copy"), (1, "read"), (2, "write")):
            for _ in range(5):
                nfs.probe_bandwidth(mode, src, dst, nbytes)
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(20)]
            for a, b in evs:
                a.record()
                nfs.probe_bandwidth(mode, src, dst, nbytes)
                b.record()
            torch.cuda.synchronize()
            ms = statistics.median(a.elapsed_time(b) for a, b in evs)
            moved = 2 * nbytes if mode == 0 else nbytes
            out[f"{name}_{mib}MiB_gbps"] = moved / (ms * 1e-3) / 1e9
        del src, dst
        torch.cuda.empty_cache()
    print(json.dumps({"bandwidth_probe": out}))


def host_ingest(args, cfg, frames):
    """Streaming ingest: every step uploads the stack from pinned host memory
    (nfs_push_host_frames) and finishes D; the upload alone is timed beside
    it with a plain pinned-to-device copy of the same bytes."""
    import torch
    import paper_1209_3362_amd as nfs
    n, N, lags, nb = cfg["n"], cfg["N"], cfg["lags"], cfg["n_bins"]
    host = torch.empty(frames.shape, dtype=frames.dtype, pin_memory=True)
    host.copy_(frames)
    dev_copy = torch.empty_like(frames)
    torch.cuda.synchronize()
    cap = args.capacity or N
    plan = nfs.Plan(n, lags, nb, in_dtype="u16", capacity=cap, spec=args.spec,
                    accum=args.accum, host_staging=True)
    out = plan.empty_outputs()
    pairs = frame_pairs(N, lags)

    def step():
        plan.reset()
        plan.push(host)
        plan.structure_function(sync=False, out=out)

    for _ in range(args.warmup):
        step()
    plan.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    plan.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    st = int(out[3].item())
    assert bool(torch.isfinite(out[0]).all()), "non-finite D"
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dev_copy.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    ms_copy = (time.perf_counter() - t0) * 1e3 / args.steps
    nbytes = host.numel() * host.element_size()
    plan.close()
    print(json.dumps({
        "metric": "frame-pairs/sec for D(q,tau) with the frames uploaded from pinned host "
                  "memory inside the step, 1024^2 x 1000 frames, 1 GPU",
        "value": pairs / (ms_step * 1e-3), "unit": "frame-pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + ", seed %d" % args.seed,
                   "frames": N, "capacity": cap, "spectra": args.spec,
                   "accumulation": args.accum, "ingest": "pinned host memory",
                   "parallelism": "single GPU"},
        "frames_per_s": N / (ms_step * 1e-3),
        "upload_only_ms": ms_copy,
        "upload_only_gbps": nbytes / (ms_copy * 1e-3) / 1e9,
        "status": st,
    }))


def batching(args):
    """c4: the 16 sequences analysed one after another on one stream, on
    four streams, and as a replayed graph of the four-stream run."""
    import torch
    import gen
    import paper_1209_3362_amd as nfs
    cfgs = gen.batch_workload(master_seed=4)
    frames = [gen.make_stack(c, c["seed"], device="cuda") for c in cfgs]
    torch.cuda.synchronize()
    seqs = [(c["n"], c["lags"], c["n_bins"], "u16", c["N"], "f32") for c in cfgs]
    caps = nfs.batch_capacities(seqs, int(args.budget_gb * (1 << 30)))
    specs = [dict(n=c["n"], lags=c["lags"], n_bins=c["n_bins"], in_dtype="u16", capacity=cap)
             for c, cap in zip(cfgs, caps)]
    pairs = sum(frame_pairs(c["N"], c["lags"]) for c in cfgs)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    res = {}
    tuned = None
    if args.batch_streams:
        b = nfs.Batch(specs, streams=args.batch_streams)
        ms = timed(lambda: b.run(frames, sync=False), args.steps, args.warmup)
        b.close()
        print(json.dumps({"metric": METRIC_C4, "value": pairs / (ms * 1e-3),
                          "unit": "frame-pairs/s", "ms_per_step": ms, "steps": args.steps,
                          "warmup": args.warmup, "streams": args.batch_streams}))
        return
    b = nfs.Batch(specs, streams=1)
    res["one_stream"] = timed(lambda: b.run(frames, sync=False), args.steps, args.warmup)
    b.close()
    del b
    b = nfs.Batch(specs, streams=4)
    if args.tune:
        tuned = b.tune(frames)
        torch.cuda.synchronize()
    res["four_streams"] = timed(lambda: b.run(frames, sync=False), args.steps, args.warmup)
    outs = b.capture(frames)
    res["four_streams_graph"] = timed(lambda: b.replay(sync=False), args.steps, args.warmup)
    st = [int(o[3].item()) for o in outs]
    assert all(bool(torch.isfinite(o[0]).all()) for o in outs)
    ws = b.workspace.numel()
    b.close()
    best = min(res.values())
    # Serial-stage floor of each sequence (as for the 1000-frame workload:
    # frames read and stored modes written at the HBM peak, 4 VALU
    # lane-instructions per pair-k at the issue rate, sums read at the HBM
    # peak), summed over the sequences; and the pair work's FP32 rate over
    # the whole run against the published FP32 peak.
    import math
    floor_ms, pair_k = 0.0, 0
    for c in cfgs:
        h = c["n"] // 2
        M = sum(math.isqrt(h * h - 1 - ky * ky) + 1 for ky in range(-h + 1, h))
        pk = frame_pairs(c["N"], c["lags"]) * M
        pair_k += pk
        floor_ms += ((c["N"] * c["n"] * c["n"] * 2 + c["N"] * M * 8 + len(c["lags"]) * M * 4)
                     / (HBM_PEAK_GBPS * 1e9) + 4.0 * pk / VALU_LANE_OPS) * 1e3
    achieved = 6.0 * pair_k / (best * 1e-3) / 1e12
    print(json.dumps({
        "metric": METRIC_C4, "value": pairs / (best * 1e-3), "unit": "frame-pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": best,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c4"], "sequences": len(cfgs),
                   "frames": [c["N"] for c in cfgs], "n": [c["n"] for c in cfgs],
                   "capacities": caps, "frame_pairs": pairs, "workspace_gb": ws / 1e9,
                   "parallelism": "single GPU",
                   "pair_shapes": "four-stream runs tuned %s" % tuned if tuned else "planned"},
        "ms_per_step_by_mode": res, "status": st,
        "serial_floor_ms": floor_ms, "frac_of_serial_floor": floor_ms / best,
        "roofline": {"kernel": "pair kernels of all 16 sequences (6 FLOP per pair-k), timed "
                               "over the whole batch run", "bound": "alu",
                     "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "peak_nonpacked": FP32_NONPACKED_TFLOPS,
                     "frac_nonpacked": achieved / FP32_NONPACKED_TFLOPS,
                     "flop_per_step": 6.0 * pair_k, "traffic": None},
    }))


def differentiation(args):
    """c5: forward (push + D) and backward (nfs_backward: gradients of
    sum(G * D) for a fixed random G with respect to frames and window)."""
    import numpy as np
    import torch
    import gen
    import paper_1209_3362_amd as nfs
    cfg = gen.config("c5")
    n, N, lags, nb = cfg["n"], cfg["N"], cfg["lags"], cfg["n_bins"]
    frames = gen.make_stack(cfg, args.seed, device="cuda")
    w = torch.from_numpy(np.outer(np.hanning(n), np.hanning(n)).astype(np.float32)).cuda()
    G = torch.from_numpy(np.random.default_rng(args.seed).standard_normal((len(lags), nb))).cuda()
    # --capacity below N: the ring holds fewer spectra than frames and the
    # backward recomputes them from the frames (needs capacity > 2 x 64).
    capacity = args.capacity or N
    recompute = capacity < N
    plan = nfs.Plan(n, lags, nb, in_dtype="f32", capacity=capacity, window=w, backward=True,
                    spec=args.spec, accum=args.accum)
    stream = plan.stream
    out = plan.empty_outputs()
    gf = torch.empty(frames.shape, dtype=torch.float32, device="cuda")
    gw = torch.empty((n, n), dtype=torch.float32, device="cuda")
    import ctypes

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        plan.reset()
        plan.push(frames)
        plan.structure_function(sync=False, out=out)
        if ev:
            ev[1].record(stream)
        plan._check(plan.lib.nfs_backward(plan.handle, ctypes.c_void_p(G.data_ptr()),
                                          ctypes.c_void_p(frames.data_ptr()),
                                          ctypes.c_void_p(gf.data_ptr()),
                                          ctypes.c_void_p(gw.data_ptr())))
        if ev:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    ms_wall = (time.perf_counter() - t0) * 1e3 / args.steps
    import statistics
    ms_step = statistics.median(e[0].elapsed_time(e[2]) for e in evs)
    ms_fwd = statistics.median(e[0].elapsed_time(e[1]) for e in evs)
    ms_bwd = statistics.median(e[1].elapsed_time(e[2]) for e in evs)
    assert bool(torch.isfinite(gf).all()) and bool(torch.isfinite(gw).all())
    pairs = frame_pairs(N, lags)
    M = plan.modes
    # Backward algorithmic traffic: the stored spectra read once, the frames
    # read once, the frame gradient written once; recomputing adds one more
    # read of the frames and one write of the spectra.
    spec_bytes = N * M * (8 if args.spec == "f32" else 4)
    bwd_bytes = spec_bytes + 2 * N * n * n * 4
    if recompute:
        bwd_bytes += spec_bytes + N * n * n * 4
    plan.close()
    print(json.dumps({
        "metric": METRIC_C5, "value": pairs / (ms_step * 1e-3), "unit": "frame-pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "ms_per_step_stat": "median of per-step HIP-event times", "ms_per_step_mean_wall": ms_wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c5"] + ", seed %d" % args.seed, "frames": N, "n": n,
                   "lags": len(lags), "n_bins": nb, "frame_pairs": pairs, "stored_modes": M,
                   "spectra": args.spec, "accumulation": args.accum, "capacity": capacity,
                   "backward_spectra": "recomputed" if recompute else "resident",
                   "parallelism": "single GPU"},
        "stage_ms": {"forward": ms_fwd, "backward": ms_bwd},
        "backward_gbps_algorithmic": bwd_bytes / (ms_bwd * 1e-3) / 1e9,
        "roofline": {"kernel": "nfs_backward (k-space gradient, inverse transforms, "
                               "normalisation adjoint" + (", spectra recomputed" if recompute
                                                          else "") + ")",
                     "bound": "hbm", "achieved": bwd_bytes / (ms_bwd * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": bwd_bytes / (ms_bwd * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "algorithmic_bytes_per_step": bwd_bytes, "traffic": None},
    }))


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.bandwidth_probe:
        bandwidth_probe(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU per process; --gpus must be 1 (multi-GPU sharding is a design only)"}))
        sys.exit(2)

    import torch
    import gen
    import paper_1209_3362_amd as nfs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    if args.workload in ("c4", "c5"):
        torch.cuda.set_device(0)
        (batching if args.workload == "c4" else differentiation)(args)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = gen.config(args.workload)
    n, N, lags, nb = cfg["n"], cfg["N"], cfg["lags"], cfg["n_bins"]
    frames = None
    if args.frames_cache and os.path.exists(args.frames_cache):
        import numpy as np
        arr = np.load(args.frames_cache)
        frames = torch.from_numpy(arr.view(np.int16)).to(dev).view(torch.uint16)
    if frames is None:
        frames = gen.make_stack(cfg, args.seed, device="cuda")
        if args.frames_cache:
            import numpy as np
            np.save(args.frames_cache, frames.view(torch.int16).cpu().numpy().view(np.uint16))
    torch.cuda.synchronize()
    if args.ingest == "host":
        host_ingest(args, cfg, frames)
        return

    plan = nfs.Plan(n, lags, nb, in_dtype="u16", capacity=args.capacity or N, device=dev,
                    spec=args.spec, accum=args.accum)
    stream = plan.stream
    out = plan.empty_outputs()
    M = plan.modes
    tuned = None
    if args.tune:
        plan.push(frames)
        tuned = plan.tune_pairs()
        plan.reset()
    pairs = frame_pairs(N, lags)

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        plan.reset()
        plan.push(frames)
        if ev:
            ev[1].record(stream)
        plan.accumulate()
        if ev:
            ev[2].record(stream)
        plan.structure_function(sync=False, out=out)
        if ev:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    import statistics
    med = statistics.median
    # Per step, HIP events on the plan's stream: the whole step and its
    # stages; the step time is the median over the timed steps.
    ms_steps = [e[0].elapsed_time(e[3]) for e in evs]
    ms_fft = med([e[0].elapsed_time(e[1]) for e in evs])
    ms_pair = med([e[1].elapsed_time(e[2]) for e in evs])
    ms_bin = med([e[2].elapsed_time(e[3]) for e in evs])
    ms_step = med(ms_steps)
    ms_wall = wall * 1e3 / args.steps

    D = out[0].cpu()
    assert bool(torch.isfinite(D).all()), "non-finite D"
    st = int(out[3].item())

    # Algorithmic traffic of one step: frames read once, each stored mode
    # (half disc, the modes any ring uses) written once and read once, per-lag
    # sums written and read once.
    bytes_frames = N * n * n * 2
    bytes_spec = N * M * (8 if args.spec == "f32" else 4)
    bytes_sums = len(lags) * M * 4
    alg_bytes = bytes_frames + 2 * bytes_spec + 2 * bytes_sums
    # Serial-stage floor of this design: the transform's HBM bytes (frames
    # read, spectra written) at the HBM peak, 4 VALU lane-instructions per
    # pair-k at the issue rate, the binning's sums read at the HBM peak.
    floor_ms = ((bytes_frames + bytes_spec) / (HBM_PEAK_GBPS * 1e9)
                + 4.0 * pairs * M / VALU_LANE_OPS + bytes_sums / (HBM_PEAK_GBPS * 1e9)) * 1e3
    # Achievable copy bandwidth on this GPU now: 1 GiB device-to-device.
    src = torch.ones((1 << 28,), dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * (1 << 30) / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    pair_k = pairs * M
    # Pair kernel: per pair and mode 2 subtractions + 2 FMAs = 6 FLOP
    # (4 VALU lane-instructions; the Kahan form adds a few per chunk).
    pair_tflops = 6.0 * pair_k / (ms_pair * 1e-3) / 1e12
    base = (args.workload, args.spec, args.accum, args.capacity or N) == ("c2", "f32", "plain", N)
    # Transform stage (A1-A3): algorithmic bytes are the frames read once and
    # the stored modes written once; the row-to-column intermediate is not
    # algorithmic. Its counter traffic (all row and column passes of one
    # step) comes from the committed summary.
    tr_bytes = bytes_frames + bytes_spec
    tr_gbps = tr_bytes / (ms_fft * 1e-3) / 1e9

    rec = {
        "metric": METRIC if args.workload == "c2" else METRIC_C3,
        "value": pairs / (ms_step * 1e-3),
        "unit": "frame-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_stat": "median of per-step HIP-event times",
        "ms_per_step_mean_wall": ms_wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + ", seed %d" % args.seed,
                   "frames": N, "n": n, "lags": len(lags), "n_bins": nb,
                   "frame_pairs": pairs, "stored_modes": M, "spectra": args.spec,
                   "accumulation": args.accum, "parallelism": "single GPU",
                   "pair_shapes": "tuned %s" % tuned if tuned else "planned"},
        "hbm_gbps_algorithmic": alg_bytes / (ms_step * 1e-3) / 1e9,
        "hbm_frac_algorithmic": alg_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "copy_gbps_measured": copy_gbps,
        "serial_floor_ms": floor_ms,
        "frac_of_serial_floor": floor_ms / ms_step,
        "stage_ms": {"normalise_fft_store": ms_fft, "lag_pairs": ms_pair, "bin": ms_bin},
        "status": st,
        "roofline": {
            "kernel": "pair_kernel (lag-pair accumulator)",
            "bound": "alu",
            "achieved": pair_tflops,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": pair_tflops / FP32_PEAK_TFLOPS,
            "traffic": counter_figure(PAIR_COUNTERS, "traffic_bytes_per_launch") if base
                       else None,
            "flop_per_launch": 6.0 * pair_k,
            "peak_nonpacked": FP32_NONPACKED_TFLOPS,
            "frac_nonpacked": pair_tflops / FP32_NONPACKED_TFLOPS,
            "valu_issue_frac": 4.0 * pair_k / (ms_pair * 1e-3) / VALU_LANE_OPS,
        },
        "transform_roofline": {
            "kernel": "row_pass_kernel + col_pass_kernel (normalise, 2D transform, store)",
            "bound": "hbm",
            "achieved": tr_gbps,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": tr_gbps / HBM_PEAK_GBPS,
            "algorithmic_bytes_per_step": tr_bytes,
            "traffic": counter_figure(TRANSFORM_COUNTERS, "traffic_bytes_per_step") if base
                       else None,
        },
    }
    if not args.no_cpu_baseline and args.workload == "c2":
        rec["cpu_baseline"] = cpu_baseline(frames, cfg, args.cpu_frames)
    plan.close()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
