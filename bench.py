"""Throughput benchmark of the gfx950 FT surface reconstruction.

One step = one frame through the whole path (splat -> 3x forward FFT ->
spectral solve -> inverse FFT -> iso-level -> marching cubes), inputs already
resident in HBM.  Default workload: the 6-view human proxy (700k points)
on a 256^3 grid over a 2.0 m box.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--config proxy256] [--pool P]
                  [--no-cpu-baseline]

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="proxy256", choices=sorted(WORKLOADS))
    ap.add_argument("--pool", type=int, default=2, help="distinct seeded frames cycled through")
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

    print(f"[bench] generating {args.pool} frame(s) of {args.config}", file=sys.stderr, flush=True)
    base_seed = synth.CONFIGS[args.config]["seed"]
    frames = [_load_frame(synth, args.config, base_seed + i, args.cache) for i in range(args.pool)]
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
                   "frames_in_pool": args.pool, "binding": "Context.prepare(...).run()"},
        "value_reconstruct_call": round(fps_call, 2),
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
        "mesh": {"vertices": round(nv_avg), "triangles": round(nt_avg)},
        "frame_roofline": {"alg_bytes": fb, "achieved_GBs": round(fb * fps / 1e9, 1),
                           "frac": round(fb * fps / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline": roof,
        "kernels": kernels,
    }

    if not args.no_cpu_baseline:
        # the oracle as it stands, single-threaded FP64, on whole frames of the
        # same workload until about 10 s of CPU time have passed
        import oracle
        print("[bench] cpu baseline: oracle on full frames", file=sys.stderr, flush=True)
        tc = time.perf_counter()
        nf = 0
        while nf < len(frames) * 4 and (nf == 0 or time.perf_counter() - tc < 10.0):
            f = frames[nf % len(frames)]
            oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
            nf += 1
            print(f"[bench] cpu baseline: {nf} frame(s), {time.perf_counter() - tc:.1f} s",
                  file=sys.stderr, flush=True)
        tcpu = time.perf_counter() - tc
        result["cpu_baseline"] = {"value": round(nf / tcpu, 5), "unit": "frames/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"{nf} full frame(s) of the same workload "
                                            f"({m} points, {dims[0]}x{dims[1]}x{dims[2]}), "
                                            f"{tcpu:.2f} s single-threaded FP64"}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
