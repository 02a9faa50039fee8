"""Autotuner of the plan parameters of a grid shape: the radix order of each
axis's mixed-radix passes and the splat tile (``fvr_set_tuning``).

For one representative frame of the shape, ``tune`` times whole
reconstructions (synchronous calls, median of ``reps``) under candidate
parameters, one axis or knob at a time starting from the library's
defaults (coordinate descent), keeps the fastest, and records it in a JSON
cache keyed by the device (name, architecture, compute units) and the grid
shape.  ``load`` applies a cache's entries for the current device to the
library, for every context and batch of the process.

Candidates:
  * radix order of an axis: the distinct orders of its default radices, and
    of the same length with each 8 split into 4 x 2 (the Stockham passes run
    them in the given order; lengths 16..256 that are powers of two use
    fixed register pencils along y and z, but the splat's x transform is a
    Stockham pass at every length);
  * splat tile ty x tz: an even number of rows R = ty tz in {4, 8, 16, 32,
    64} with R Nx <= 2048 and (ty + 3)(tz + 3) <= 128, each split of R into
    ty, tz with both at most 16.
"""
from __future__ import annotations

import ctypes
import itertools
import json
import os
import time

from . import FvrError, _Frame, load_library  # noqa: F401

__all__ = ["device_key", "default_cache_path", "get_tuning", "set_tuning", "candidates", "tune",
           "load", "save_entry"]


class _Tuning(ctypes.Structure):
    _fields_ = [("nstages", ctypes.c_int32 * 3), ("radices", (ctypes.c_int32 * 8) * 3),
                ("splat_ty", ctypes.c_int32), ("splat_tz", ctypes.c_int32)]


def _lib():
    lib = load_library()
    if not getattr(lib, "_tuning_bound", False):
        lib.fvr_set_tuning.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_Tuning)]
        lib.fvr_set_tuning.restype = ctypes.c_int
        lib.fvr_get_tuning.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_Tuning)]
        lib.fvr_get_tuning.restype = ctypes.c_int
        lib._tuning_bound = True
    return lib


def _dims(dims):
    return (ctypes.c_int32 * 3)(*[int(x) for x in dims])


def device_key(device: int = 0) -> str:
    import torch
    p = torch.cuda.get_device_properties(device)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}cu"


def default_cache_path() -> str:
    return os.environ.get("FVR_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "fvr", "autotune.json")


def get_tuning(dims) -> dict:
    """The parameters plans of this shape use now (tuned or default)."""
    lib = _lib()
    t = _Tuning()
    st = lib.fvr_get_tuning(_dims(dims), ctypes.byref(t))
    if st:
        raise FvrError(st, "fvr_get_tuning")
    return {"radices": [[int(t.radices[a][k]) for k in range(t.nstages[a])] for a in range(3)],
            "splat_tile": [int(t.splat_ty), int(t.splat_tz)]}


def set_tuning(dims, params: dict | None) -> None:
    """Apply ``params`` ({"radices": [[...]x3], "splat_tile": [ty, tz]}) to
    shape ``dims`` for the whole process, or clear its tuning (None)."""
    lib = _lib()
    if params is None:
        st = lib.fvr_set_tuning(_dims(dims), None)
    else:
        t = _Tuning()
        for a, rad in enumerate(params.get("radices", [[], [], []])):
            t.nstages[a] = len(rad)
            for k, r in enumerate(rad):
                t.radices[a][k] = int(r)
        ty, tz = params.get("splat_tile", [0, 0])
        t.splat_ty, t.splat_tz = int(ty), int(tz)
        st = lib.fvr_set_tuning(_dims(dims), ctypes.byref(t))
    if st:
        msg = lib.fvr_last_error(None)
        raise FvrError(st, msg.decode() if msg else "fvr_set_tuning")


def _orders(rad):
    """Distinct orders of a radix list and of its variants with 8 -> 4 x 2."""
    out = []
    variants = [list(rad)]
    if 8 in rad:
        v = []
        for r in rad:
            v += [4, 2] if r == 8 else [r]
        if len(v) <= 8:
            variants.append(v)
    for v in variants:
        for p in sorted(set(itertools.permutations(v))):
            if list(p) not in out:
                out.append(list(p))
    return out[:12]


def candidates(dims) -> dict:
    """Candidate values of each knob for shape ``dims``."""
    base = get_tuning(dims)
    nx = int(dims[0])
    tiles = []
    for R in (4, 8, 16, 32, 64):
        if R * nx > 2048:
            continue
        for ty in range(1, 17):
            if R % ty:
                continue
            tz = R // ty
            if tz <= 16 and (ty + 3) * (tz + 3) <= 128:
                tiles.append([ty, tz])
    # y and z lengths 16..256 that are powers of two run fixed register pencils
    pencil = lambda n: n in (16, 32, 64, 128, 256)  # noqa: E731
    rad = [_orders(r) if (a == 0 or not pencil(int(dims[a]))) else [list(r)]
           for a, r in enumerate(base["radices"])]
    return {"radices": rad, "splat_tile": tiles}


def _time_frame(prepared, reps: int) -> float:
    prepared.run()  # plan (re)built
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        prepared.run()
        ts.append(time.perf_counter() - t0)
    ts.sort()
    return ts[len(ts) // 2] * 1e6


def tune(ctx, points, normals, weights, grid_dim, bbox, reps: int = 15, verbose: bool = False) -> dict:
    """Coordinate-descent search over ``candidates`` on one frame (device
    tensors).  Leaves the best parameters applied and returns
    {"params", "us", "default_us", "tried"}."""
    import torch
    dims = tuple(int(x) for x in grid_dim)
    set_tuning(dims, None)
    nx, ny, nz = dims
    vcap = max(4096, 6 * (nx * ny + ny * nz + nx * nz))
    out = (torch.empty((vcap, 3), dtype=torch.float32, device=f"cuda:{ctx.device}"),
           torch.empty((2 * vcap, 3), dtype=torch.int32, device=f"cuda:{ctx.device}"))
    prep = ctx.prepare(points, normals, weights, grid_dim=dims, bbox=bbox, out=out)
    best = get_tuning(dims)
    best_us = default_us = _time_frame(prep, reps)
    tried = 1
    cand = candidates(dims)
    for a in range(3):
        for order in cand["radices"][a]:
            if order == best["radices"][a]:
                continue
            trial = {"radices": [list(r) for r in best["radices"]], "splat_tile": list(best["splat_tile"])}
            trial["radices"][a] = order
            set_tuning(dims, trial)
            us = _time_frame(prep, reps)
            tried += 1
            if verbose:
                print(f"[autotune] {dims} axis {a} radices {order}: {us:.1f} us", flush=True)
            if us < best_us:
                best, best_us = trial, us
    for tile in cand["splat_tile"]:
        if tile == best["splat_tile"]:
            continue
        trial = {"radices": [list(r) for r in best["radices"]], "splat_tile": tile}
        set_tuning(dims, trial)
        us = _time_frame(prep, reps)
        tried += 1
        if verbose:
            print(f"[autotune] {dims} splat tile {tile}: {us:.1f} us", flush=True)
        if us < best_us:
            best, best_us = trial, us
    set_tuning(dims, best)
    return {"params": best, "us": round(best_us, 2), "default_us": round(default_us, 2), "tried": tried}


def _shape_key(dims) -> str:
    return "x".join(str(int(x)) for x in dims)


def save_entry(dims, result: dict, path: str | None = None, device: int = 0) -> str:
    """Record a ``tune`` result in the JSON cache (merged with what is there)."""
    path = path or default_cache_path()
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data.setdefault(device_key(device), {})[_shape_key(dims)] = result
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def load(path: str | None = None, device: int = 0) -> int:
    """Apply the cache's entries for this device; returns how many."""
    path = path or default_cache_path()
    if not os.path.exists(path):
        return 0
    with open(path) as fh:
        data = json.load(fh)
    n = 0
    for shape, res in data.get(device_key(device), {}).items():
        dims = tuple(int(x) for x in shape.split("x"))
        set_tuning(dims, res["params"])
        n += 1
    return n
