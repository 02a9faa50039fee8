"""Throughput benchmark of the gfx950 FT surface reconstruction.

One step = one frame through the whole path (splat -> 3x forward FFT ->
spectral solve -> inverse FFT -> iso-level -> marching cubes), inputs already
resident in HBM.  Default workload: the 6-view human proxy (700k points)
on a 256^3 grid over a 2.0 m box.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--config proxy256] [--pool P]
                  [--poses Q] [--latency-frames L] [--no-cpu-baseline]

The pool holds P distinct frames resident in HBM (64 by default: 1.25 GB at
256^3, well beyond the 256 MB last-level cache): Q of them ray-cast, the
others those captures with the rig turned by a seeded yaw and shifted
(synth.repose), since ray-casting a frame takes seconds on the host.
Throughput is the K timed steps; p50/p99 come from a separate sample of
max(L, K) frames, each a synchronous call timed on the host clock.

Per-kernel durations come from HIP events the library records on its stream
around every launch, in an untimed pass after the warmup; that pass names the
dominant kernel.  Inside the timed region events surround that kernel only,
and its roofline uses its average duration there and its algorithmic bytes
(defined inputs read once, outputs written once).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/s at 256^3 grid (splat->FFT->solve->iFFT->MC); p99 frame latency"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "proxy256": "human proxy, 6 depth views, 700k points, 256^3 grid, 2.0 m box",
    "proxy128": "human proxy, 4 depth views, 400k points, 128^3 grid, 2.0 m box",
    "sphere64": "sphere r=0.8, 50k points, 64^3 grid, [-1,1]^3 box",
}


def kernel_alg_bytes(dims, m, nv, nt):
    """Algorithmic bytes per launch of each kernel: its defined inputs read
    once and outputs written once (F = one float32 field, S = one complex64
    half spectrum, m points of 28 bytes: position, normal, weight)."""
    nx, ny, nz = dims
    n = nx * ny * nz
    F = 4 * n
    S = 8 * nz * ny * (nx // 2 + 1)
    return {
        "prep": 0,
        "bin_count": 28 * m + 8 * m,
        "tile_list": 0,
        "bin_scatter": 36 * m + 32 * m,
        "splat_fft_x": 28 * m + 3 * S,
        "fft_y_fwd": 3 * S + 2 * S,
        "fft_z_solve": 2 * S + S,
        "fft_y_inv": 2 * S,
        "fft_x_c2r": S + F,
        "fft_yx_inv": S + F,
        "level": 12 * m,
        "mc_classify": 0,
        "mc_count": F,
        "mc_generate": F + 12 * nv,
        "mc_triangles": 12 * nt,
    }


# Source files each kernel is compiled from (plus the shared headers and the
# build flags): a stored counter reading is used only while these are unchanged.
_CSRC = os.path.join(ROOT, "paper_1712_03084_amd", "csrc")
KERNEL_SOURCES = {
    "prep": "fvr_mc.hip", "bin_count": "fvr_splat.hip", "tile_list": "fvr_splat.hip",
    "tile_order": "fvr_splat.hip", "bin_scatter": "fvr_splat.hip", "splat_fft_x": "fvr_splat.hip",
    "fft_y_fwd": "fvr_fft.hip", "fft_z_solve": "fvr_fft.hip", "fft_y_inv": "fvr_fft.hip",
    "fft_x_c2r": "fvr_fft.hip", "fft_yx_inv": "fvr_fft.hip", "level": "fvr_mc.hip", "mc_classify": "fvr_mc.hip", "mc_count": "fvr_mc.hip",
    "mc_scan": "fvr_mc.hip", "mc_generate": "fvr_mc.hip", "mc_triangles": "fvr_mc.hip",
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_proxy256.txt")


def kernel_source_digest(name):
    """sha256 over the kernel's source file, the shared device headers and the
    build script (first 16 hex digits)."""
    import hashlib
    h = hashlib.sha256()
    for f in (os.path.join(_CSRC, KERNEL_SOURCES[name]), os.path.join(_CSRC, "fvr_common.h"),
              os.path.join(_CSRC, "fvr_fft_engine.h"), os.path.join(_CSRC, "fvr_scan.h"),
              os.path.join(ROOT, "paper_1712_03084_amd", "build.py")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(name, config):
    """HBM bytes per launch of `name` from the stored rocprofv3 FETCH_SIZE and
    WRITE_SIZE readings (scaled by the plain-copy calibration), or None when
    there is no reading for this kernel and workload or its sources changed
    since the reading was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    digest = kernel_source_digest(name)
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            # kernel workload fetch_bytes write_bytes traffic_bytes digest
            if len(f) == 6 and f[0] == name and f[1] == config and f[5] == digest:
                return int(f[4])
    return None


def kernel_touched_bytes(dims, m, stats):
    """Bytes the sparse passes actually move on this frame (the dense figures
    of kernel_alg_bytes priced on the parts of the grid they touch): the
    splat writes the spectrum rows of busy tiles only, the y pass reads those
    rows and writes the non-zero z planes, the z pass reads those planes."""
    nx, ny, nz = dims
    S = 8 * nz * ny * (nx // 2 + 1)
    tf = stats["busy_tiles"] / max(1, stats["tiles"])
    pf = stats["nonzero_planes"] / max(1, stats["planes"])
    return {
        "splat_fft_x": round(28 * m + 3 * S * tf),
        "fft_y_fwd": round(3 * S * tf + 2 * S * pf),
        "fft_z_solve": round(2 * S * pf + S),
    }


def frame_alg_bytes(dims, m, nv, nt):
    """Whole-frame algorithmic bytes: each stage of the method reads its
    defined input once and writes its output once (8F + 8S + 40m + mesh)."""
    nx, ny, nz = dims
    F = 4 * nx * ny * nz
    S = 8 * nz * ny * (nx // 2 + 1)
    return 8 * F + 8 * S + 40 * m + 12 * nv + 12 * nt


def _load_frame(synth, config, seed, cache):
    """Generate a seeded frame, or reuse a copy saved by an earlier run."""
    import numpy as np
    path = os.path.join(cache, f"{config}_{seed}.npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path)
        return synth.Frame(z["points"], z["normals"], z["weights"], tuple(int(x) for x in z["dims"]),
                           tuple(float(x) for x in z["bbox"]), name=f"{config}_{seed}")
    f = synth.config_frame(config, seed=seed)
    if path:
        os.makedirs(cache, exist_ok=True)
        np.savez(path, points=f.points, normals=f.normals, weights=f.weights,
                 dims=np.asarray(f.dims), bbox=np.asarray(f.bbox))
    return f


def bench_batch(args, fvr, synth, torch, np, dev):
    """Batched workload: the same uneven frames through the plain
    single-frame call (one synchronisation per frame) and through a batch
    (one captured graph per launch, one synchronisation per batch)."""
    print(f"[bench] batched workload: {args.batch} frames", file=sys.stderr, flush=True)
    frames, _ = synth.batch_frames(args.batch, seed=4000)
    devs = [tuple(torch.from_numpy(a).to(dev) for a in (f.points, f.normals, f.weights)) + (f.dims, f.bbox)
            for f in frames]
    vcap = 400_000
    outs = [(torch.empty((vcap, 3), dtype=torch.float32, device=dev),
             torch.empty((2 * vcap, 3), dtype=torch.int32, device=dev)) for _ in frames]
    n = len(frames)
    reps = max(1, args.steps // n)
    ctx = fvr.Context(0)
    tuned = {}
    if args.autotune:
        # the project's autotuner picks radix orders and splat tiles per grid
        # shape on the first frame of each shape; every later call (plain and
        # batched) uses them
        from paper_1712_03084_amd import autotune
        for i, f in enumerate(frames):
            if f.dims in tuned:
                continue
            d = devs[i]
            r = autotune.tune(ctx, d[0], d[1], d[2], f.dims, f.bbox, reps=10)
            tuned[f.dims] = r
            if args.tune_cache:
                autotune.save_entry(f.dims, r, path=args.tune_cache)
            print(f"[bench] autotune {f.dims}: {r['default_us']:.1f} -> {r['us']:.1f} us per frame "
                  f"({r['tried']} tried) {r['params']}", file=sys.stderr, flush=True)
    plain = [ctx.prepare(d[0], d[1], d[2], grid_dim=d[3], bbox=d[4], out=o) for d, o in zip(devs, outs)]
    for p in plain:
        p.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for p in plain:
            p.run()
    torch.cuda.synchronize()
    plain_fps = reps * n / (time.perf_counter() - t0)
    sweep = {}
    best = None
    for slots in [int(x) for x in args.batch_slots.split(",") if x]:
        b = fvr.Batch(slots=slots, graph=True)
        pb = b.prepare(devs, outs)
        for _ in range(2):
            pb.run()  # capture, then a replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pb.run()
        fps = reps * n / (time.perf_counter() - t0)
        sweep[slots] = round(fps, 2)
        if best is None or fps > best[1]:
            best = (slots, fps, b, pb)
        else:
            b.close()
    slots, fps, b, pb = best
    lat = []
    for _ in range(max(args.latency_frames, args.steps)):
        ts = time.perf_counter()
        pb.run()
        lat.append(time.perf_counter() - ts)
    lat = np.asarray(lat) * 1e3
    # the graph-free form of the same batch
    b.use_graph(False)
    pb2 = b.prepare(devs, outs)
    pb2.run()
    t0 = time.perf_counter()
    for _ in range(reps):
        pb2.run()
    nograph_fps = reps * n / (time.perf_counter() - t0)
    b.close()
    grids = [f.dims[0] for f in frames]
    pts = [f.n_points for f in frames]
    return {"workload": f"{n} human-proxy frames of 2-6 views, grids from {{96,128,160,192}}^3 "
                        f"({grids}), {min(pts)}-{max(pts)} points",
            "frames": n, "unit": "frames/s",
            "plain_value": round(plain_fps, 2),
            "batched_value": round(fps, 2), "slots": slots, "slots_sweep": sweep,
            "batched_no_graph_value": round(nograph_fps, 2),
            "batch_p50_ms": round(float(np.percentile(lat, 50)), 4),
            "batch_p99_ms": round(float(np.percentile(lat, 99)), 4),
            "batch_latency_samples": len(lat),
            "alg_bytes_per_batch": sum(frame_alg_bytes(f.dims, f.n_points, 0, 0) for f in frames),
            "autotuned": {"x".join(map(str, k)): {"params": v["params"], "default_us": v["default_us"],
                                                  "tuned_us": v["us"]} for k, v in tuned.items()}}


def bench_batch_headline(args, fvr, torch, np, dev, pool, dims, bbox):
    """The headline workload's frames through the batch: n frames of the pool
    per call, spread over S slots (frames of different slots overlap on the
    device), one captured graph and one synchronisation per call."""
    n = min(args.headline_batch, len(pool))
    print(f"[bench] headline frames batched: {n} per call", file=sys.stderr, flush=True)
    vcap = 200_000
    outs = [(torch.empty((vcap, 3), dtype=torch.float32, device=dev),
             torch.empty((2 * vcap, 3), dtype=torch.int32, device=dev)) for _ in range(n)]
    devs = [tuple(pool[i]) + (dims, bbox) for i in range(n)]
    reps = max(2, args.steps // n)
    sweep, best = {}, None
    for slots in [int(x) for x in args.headline_slots.split(",") if x]:
        b = fvr.Batch(slots=slots, graph=True)
        pb = b.prepare(devs, outs)
        for _ in range(2):
            pb.run()  # capture, then a replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pb.run()
        fps = reps * n / (time.perf_counter() - t0)
        sweep[slots] = round(fps, 2)
        if best is None or fps > best[1]:
            if best is not None:
                best[2].close()
            best = (slots, fps, b, pb)
        else:
            b.close()
    slots, fps, b, pb = best
    lat = []
    for _ in range(max(20, args.latency_frames // n)):
        ts = time.perf_counter()
        pb.run()
        lat.append(time.perf_counter() - ts)
    b.close()
    lat = np.asarray(lat) * 1e3
    return {"workload": f"{n} frames of the headline pool per call", "frames": n, "unit": "frames/s",
            "batched_value": round(fps, 2), "slots": slots, "slots_sweep": sweep,
            "batch_p50_ms": round(float(np.percentile(lat, 50)), 4),
            "batch_p99_ms": round(float(np.percentile(lat, 99)), 4),
            "batch_latency_samples": len(lat)}


def bench_serve(args, fvr, synth, np, captures):
    """Serving (config 5): three capture stations (128^3 with 4 views, 192^3
    and 256^3 with 6) emit frames at 30 Hz each with exponential
    inter-arrival times; the server admits them by device memory as slots
    free up.  Frames come from per-station pools (reposed copies of one
    capture each, inputs in pinned host memory, uploaded per request);
    latency runs from arrival to the mesh in host memory."""
    import torch
    stations = [("128^3, 4 views", captures["proxy128"], (128, 128, 128), None),
                ("192^3, 6 views", captures["proxy256b"], (192, 192, 192), 550_000),
                ("256^3, 6 views", captures["proxy256"], (256, 256, 256), None)]
    pools = []
    for si, (name, cap, dims, m) in enumerate(stations):
        base = synth.subsample(cap, m, seed=500 + si) if m else cap
        pool = []
        for j in range(args.serve_pool):
            f = base if j == 0 else synth.repose(base, seed=9000 + 100 * si + j)
            pool.append(tuple(torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
                              for a in (f.points, f.normals, f.weights)))
        pools.append((name, dims, base.bbox, pool, base.n_points))
    rng = np.random.default_rng(5000)
    arrivals = []
    for si in range(len(pools)):
        t = 0.0
        while True:
            t += rng.exponential(1.0 / args.serve_rate)
            if t > args.serve_seconds:
                break
            arrivals.append((t, si, int(rng.integers(0, args.serve_pool))))
    arrivals.sort()
    storages = [x for x in args.serve_storages.split(",") if x]
    out = None
    for storage in storages:
        r = _serve_stream(args, fvr, np, pools, arrivals, storage)
        if out is None:
            out = r
            out["storage"] = storage
            out["other_storages"] = {}
        else:
            out["other_storages"][storage] = {k: r[k] for k in ("completed", "value", "p50_ms", "p99_ms",
                                                                 "stations", "max_in_flight", "device_bytes")}
    return out


def _serve_stream(args, fvr, np, pools, arrivals, storage):
    """One pass of the arrival stream through a fresh server, every request
    with the given spectrum storage."""
    srv = fvr.Server(slots=args.serve_slots, hbm_budget=int(args.serve_budget_gib * (1 << 30)))
    # warm the slots up: every station's shape once per slot, so the
    # measured stream runs on grown scratch
    for _ in range(args.serve_slots):
        for name, dims, bbox, pool, _m in pools:
            srv.submit(*pool[0], dims, bbox, storage=storage)
    srv.drain()
    print(f"[bench] serving ({storage} spectra): {len(arrivals)} requests over {args.serve_seconds} s",
          file=sys.stderr, flush=True)
    results = []
    t0 = time.perf_counter()
    for t, si, j in arrivals:
        while time.perf_counter() - t0 < t:
            results += srv.poll()
        name, dims, bbox, pool, _m = pools[si]
        srv.submit(*pool[j], dims, bbox, user=si, storage=storage)
    results += srv.drain()
    elapsed = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    ok = [r for r in results if r["status"] == 0]
    lat = np.array([r["latency_ms"] for r in ok])
    per = {}
    for si, (name, dims, bbox, pool, m) in enumerate(pools):
        ls = np.array([r["latency_ms"] for r in ok if r["user"] == si])
        per[name] = {"frames": int(len(ls)), "points": m,
                     "p50_ms": round(float(np.percentile(ls, 50)), 3) if len(ls) else None,
                     "p99_ms": round(float(np.percentile(ls, 99)), 3) if len(ls) else None}
    return {"workload": "3 stations x 30 Hz Poisson (128^3 4 views, 192^3 6 views, 256^3 6 views), "
                        f"{args.serve_seconds} s stream, pools of {args.serve_pool} frames per station",
            "requests": len(arrivals), "completed": len(ok), "unit": "frames/s",
            "value": round(len(ok) / elapsed, 2),
            "offered_rate": round(len(arrivals) / args.serve_seconds, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "stations": per, "slots": args.serve_slots, "max_in_flight": info["max_in_flight"],
            "device_bytes": info["device_bytes"], "budget_bytes": info["budget"],
            "latency": "arrival -> mesh in host memory (upload, all stages, download)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="proxy256", choices=sorted(WORKLOADS))
    ap.add_argument("--pool", type=int, default=64, help="distinct frames resident in HBM, cycled through")
    ap.add_argument("--poses", type=int, default=2,
                    help="ray-cast captures in the pool; the rest are reposed copies of them")
    ap.add_argument("--latency-frames", type=int, default=200,
                    help="frames in the separate latency sample (at least --steps)")
    ap.add_argument("--secondary", default="proxy128",
                    help="comma-separated workloads measured after the headline one and reported "
                         "under 'secondary' (empty: none)")
    ap.add_argument("--storages", default="bf16,fp16",
                    help="16-bit spectrum storages measured on the headline workload after it and "
                         "reported under 'storage' (empty: none)")
    ap.add_argument("--headline-batch", type=int, default=16,
                    help="frames of the headline pool per batched call, measured after the plain "
                         "form and reported under 'batched_headline' (0: skip)")
    ap.add_argument("--headline-slots", default="2,4,8",
                    help="slot counts of the batched headline measurement; the fastest is reported")
    ap.add_argument("--batch", type=int, default=16,
                    help="frames of the batched workload (16 uneven frames on {96..192}^3 grids) "
                         "measured after the headline one, batched and plain (0: skip)")
    ap.add_argument("--batch-slots", default="1,2,4,8,16",
                    help="slot counts of the batched measurement; the fastest is reported")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the simulated serving stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=30.0, help="frames/s per station")
    ap.add_argument("--serve-pool", type=int, default=16, help="frames per station pool")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--serve-storages", default="f32,bf16",
                    help="spectrum storages of the serving passes (the same arrival stream each); the "
                         "first is reported under 'serving', the others under its 'other_storages'")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="measure the batched workload on the default plans")
    ap.add_argument("--tune-cache", default=None, help="JSON file the autotuner's choices are added to")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the all-cores CPU baseline (0: the host's CPUs, at most 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--breakdown", type=int, default=20,
                    help="untimed frames with events around every kernel, for the per-kernel table")
    ap.add_argument("--calib-copy", action="store_true",
                    help="before the timed region, copy a 256 MiB float32 buffer once (a plain copy "
                         "kernel of known size, for scaling profiler byte counters)")
    ap.add_argument("--cache", default=None,
                    help="directory to keep generated frames in (.npz), reused on later runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the frame-parallel "
              "multi-GPU path is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1712_03084_amd as fvr
    import synth

    npose = max(1, min(args.poses, args.pool))
    print(f"[bench] generating {npose} capture(s) of {args.config}, pool of {args.pool}",
          file=sys.stderr, flush=True)
    base_seed = synth.CONFIGS[args.config]["seed"]
    caps_pool = [_load_frame(synth, args.config, base_seed + i, args.cache) for i in range(npose)]
    frames = list(caps_pool) + [synth.repose(caps_pool[i % npose], seed=base_seed + 100 + i)
                                for i in range(args.pool - npose)]
    dev = torch.device("cuda:0")
    pool = [tuple(torch.from_numpy(a).to(dev) for a in (f.points, f.normals, f.weights))
            for f in frames]
    dims, bbox = frames[0].dims, frames[0].bbox
    m = frames[0].n_points
    ctx = fvr.Context(0)
    vcap = 2_000_000
    out = (torch.empty((vcap, 3), dtype=torch.float32, device=dev),
           torch.empty((2 * vcap, 3), dtype=torch.int32, device=dev))

    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # Each pool frame's call is marshalled once (Context.prepare), as a serving
    # loop with fixed staging buffers would; every step still runs the whole
    # fvr_reconstruct call: validation, all kernels, the status readback.
    prepared = [ctx.prepare(*fr, grid_dim=dims, bbox=bbox, out=out) for fr in pool]

    print("[bench] warmup", file=sys.stderr, flush=True)
    for k in range(args.warmup):
        prepared[k % len(pool)].run()
    torch.cuda.synchronize()

    # Per-kernel breakdown from an untimed pass with events around every
    # launch; it names the dominant kernel.
    kernels = {}
    dom = None
    if not args.no_kernel_timing:
        ctx.timing(True)
        ctx.timing_reset()
        for k in range(args.breakdown):
            prepared[k % len(pool)].run()
        torch.cuda.synchronize()
        for name, (ms, cnt) in ctx.timings().items():
            if cnt:
                kernels[name] = {"avg_us": round(ms / cnt * 1e3, 2), "launches": cnt}
        dom = max(kernels, key=lambda n: kernels[n]["avg_us"])
        # inside the timed region only the dominant kernel carries events
        ctx.timing_select([dom])
        ctx.timing_reset()

    lat = []
    nv_tot = nt_tot = 0
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        nv, nt = prepared[k % len(pool)].run()
        lat.append(time.perf_counter() - ts)
        nv_tot += nv
        nt_tot += nt
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.timing(False)
    elapsed = t1 - t0
    fps = args.steps / elapsed

    stats = ctx.last_stats()

    # latency sample: each frame a synchronous call, timed on the host clock
    nlat = max(args.latency_frames, args.steps)
    print(f"[bench] latency sample of {nlat} frames", file=sys.stderr, flush=True)
    lat = []
    for k in range(nlat):
        ts = time.perf_counter()
        prepared[k % len(pool)].run()
        lat.append(time.perf_counter() - ts)

    # the same frames through Context.reconstruct, which checks and marshals
    # its tensors on every call (reported beside the headline figure)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for k in range(args.steps):
        ctx.reconstruct(*pool[k % len(pool)], grid_dim=dims, bbox=bbox, out=out)
    torch.cuda.synchronize()
    fps_call = args.steps / (time.perf_counter() - c0)
    lat_ms = np.sort(np.asarray(lat) * 1e3)
    nv_avg = nv_tot / args.steps
    nt_avg = nt_tot / args.steps

    roof = None
    if dom is not None:
        ms, cnt = ctx.timings()[dom]
        alg = kernel_alg_bytes(dims, m, nv_avg, nt_avg)
        avg_s = ms / cnt * 1e-3
        ach = alg.get(dom, 0) / avg_s / 1e9 if avg_s > 0 else 0.0
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(dom, args.config),
                "alg_bytes_per_launch": alg.get(dom, 0),
                "avg_us_timed_region": round(ms / cnt * 1e3, 2), "launches": cnt}

    fb = frame_alg_bytes(dims, m, nv_avg, nt_avg)
    result = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "grid": list(dims), "points": m,
                   "frames_in_pool": args.pool, "captures_in_pool": npose,
                   "binding": "Context.prepare(...).run()"},
        "value_reconstruct_call": round(fps_call, 2),
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
        "latency_frames": nlat,
        "mesh": {"vertices": round(nv_avg), "triangles": round(nt_avg)},
        "frame_roofline": {"alg_bytes": fb, "achieved_GBs": round(fb * fps / 1e9, 1),
                           "frac": round(fb * fps / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roof,
        "kernels": kernels,
        "work": stats,
    }
    touched = kernel_touched_bytes(dims, m, stats)
    algb = kernel_alg_bytes(dims, m, nv_avg, nt_avg)
    for name, kv in kernels.items():
        kv["alg_bytes"] = algb.get(name)
        if name in touched:
            kv["touched_bytes"] = touched[name]

    # secondary workloads: throughput and latency of the same call on other
    # grids (their own pools of one capture and reposed copies)
    sec = {}
    sec_caps = {}
    for name in [x for x in args.secondary.split(",") if x and x != args.config]:
        print(f"[bench] secondary workload {name}", file=sys.stderr, flush=True)
        cap = _load_frame(synth, name, synth.CONFIGS[name]["seed"], args.cache)
        sec_caps[name] = cap
        sframes = [cap] + [synth.repose(cap, seed=7000 + i) for i in range(15)]
        sdims, sbbox = cap.dims, cap.bbox
        sprep = [ctx.prepare(*(torch.from_numpy(a).to(dev) for a in (f.points, f.normals, f.weights)),
                             grid_dim=sdims, bbox=sbbox, out=out) for f in sframes]
        for k in range(args.warmup):
            sprep[k % len(sprep)].run()
        torch.cuda.synchronize()
        q0 = time.perf_counter()
        for k in range(args.steps):
            sprep[k % len(sprep)].run()
        torch.cuda.synchronize()
        sfps = args.steps / (time.perf_counter() - q0)
        slat = []
        for k in range(max(args.latency_frames, args.steps)):
            ts = time.perf_counter()
            sprep[k % len(sprep)].run()
            slat.append(time.perf_counter() - ts)
        slat = np.asarray(slat) * 1e3
        sfb = frame_alg_bytes(sdims, cap.n_points, 0, 0)
        sec[name] = {"workload": WORKLOADS[name], "value": round(sfps, 2), "unit": "frames/s",
                     "ms_per_step": round(1e3 / sfps, 4),
                     "p50_ms": round(float(np.percentile(slat, 50)), 4),
                     "p99_ms": round(float(np.percentile(slat, 99)), 4),
                     "frames_in_pool": len(sframes),
                     "frame_alg_bytes": sfb,
                     "effective_GBs": round(sfb * sfps / 1e9, 1)}
        del sprep
    if sec:
        result["secondary"] = sec

    # 16-bit spectrum storage on the headline workload: throughput of the same
    # prepared calls, the per-kernel times, and the indicator's deviation from
    # the float32-storage result on the first pool frame (the error against
    # the FP64 oracle is what the precision tests bound)
    storages = [x for x in args.storages.split(",") if x]
    if storages:
        stor = {}
        A32, _ = ctx.indicator(*pool[0], grid_dim=dims, bbox=bbox)
        arange = float(A32.max() - A32.min())
        all_kernels = [ctx.lib.fvr_timing_name(i).decode() for i in range(ctx.lib.fvr_timing_count())]
        for sname in storages:
            print(f"[bench] storage {sname}", file=sys.stderr, flush=True)
            sp = [ctx.prepare(*fr, grid_dim=dims, bbox=bbox, out=out, storage=sname) for fr in pool[:16]]
            for k in range(args.warmup):
                sp[k % len(sp)].run()
            skern = {}
            if not args.no_kernel_timing:
                ctx.timing_select(all_kernels)
                ctx.timing(True)
                ctx.timing_reset()
                for k in range(args.breakdown):
                    sp[k % len(sp)].run()
                torch.cuda.synchronize()
                ctx.timing(False)
                skern = {n: round(ms / cnt * 1e3, 2) for n, (ms, cnt) in ctx.timings().items() if cnt}
            torch.cuda.synchronize()
            q0 = time.perf_counter()
            for k in range(args.steps):
                sp[k % len(sp)].run()
            torch.cuda.synchronize()
            sfps = args.steps / (time.perf_counter() - q0)
            A16, _ = ctx.indicator(*pool[0], grid_dim=dims, bbox=bbox, storage=sname)
            dev_max = float((A16 - A32).abs().max()) / arange
            dev_rms = float(((A16 - A32) ** 2).mean().sqrt()) / arange
            stor[sname] = {"value": round(sfps, 2), "unit": "frames/s", "ms_per_step": round(1e3 / sfps, 4),
                           "kernels_avg_us": skern,
                           "indicator_dev_vs_f32_storage": {"max": float(f"{dev_max:.3g}"),
                                                            "rms": float(f"{dev_rms:.3g}"),
                                                            "of": "the indicator's range"}}
            del sp, A16
        del A32
        result["storage"] = stor

    if args.headline_batch > 0:
        result["batched_headline"] = bench_batch_headline(args, fvr, torch, np, dev, pool, dims, bbox)

    if args.batch > 0:
        result["batched"] = bench_batch(args, fvr, synth, torch, np, dev)

    if args.serve_seconds > 0:
        caps = {"proxy256": caps_pool[0],
                "proxy256b": caps_pool[1] if len(caps_pool) > 1 else synth.repose(caps_pool[0], seed=77),
                "proxy128": sec_caps.get("proxy128") or _load_frame(synth, "proxy128",
                                                                   synth.CONFIGS["proxy128"]["seed"], args.cache)}
        result["serving"] = bench_serve(args, fvr, synth, np, caps)

    if not args.no_cpu_baseline:
        # the oracle as it stands (FP64), on whole frames of the same workload:
        # single-threaded, then on the host's cores (OpenMP over voxel and
        # marching-cubes planes, FFT lines over workers: the same sums)
        import oracle
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        nthr = args.cpu_threads or max(1, min(16, avail))
        print(f"[bench] cpu baseline: host has {os.cpu_count()} CPUs ({avail} available); "
              f"oracle at 1 and {nthr} threads", file=sys.stderr, flush=True)

        def leg(threads, budget_s):
            tc = time.perf_counter()
            nf = 0
            while nf < len(frames) and (nf == 0 or time.perf_counter() - tc < budget_s):
                f = frames[nf % len(frames)]
                oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox, threads=threads)
                nf += 1
                print(f"[bench] cpu baseline ({threads} thread(s)): {nf} frame(s), "
                      f"{time.perf_counter() - tc:.1f} s", file=sys.stderr, flush=True)
            return nf, time.perf_counter() - tc

        nf1, t1c = leg(1, 10.0)
        nfa, tac = leg(nthr, 10.0)
        result["cpu_baseline"] = {
            "value": round(nfa / tac, 5), "unit": "frames/s", "cores": nthr, "kind": "oracle",
            "sample": f"{nfa} full frame(s) of the same workload ({m} points, "
                      f"{dims[0]}x{dims[1]}x{dims[2]}), {tac:.2f} s FP64 on {nthr} threads",
            "host_cpus": os.cpu_count(), "host_cpus_available": avail,
            "single_core": {"value": round(nf1 / t1c, 5), "unit": "frames/s", "cores": 1,
                            "sample": f"{nf1} full frame(s), {t1c:.2f} s single-threaded FP64"},
        }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
