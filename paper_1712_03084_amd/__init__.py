"""MI355X (gfx950) volumetric Fourier-transform surface reconstruction.

Python binding over the C ABI in ``include/fvr.h`` (``libfvr.so``).  The
binding only marshals arguments: every step of the reconstruction runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream: inputs
are CUDA (HIP) float32 tensors on the context's device and work is enqueued
on ``torch.cuda.current_stream()``.

The method is Sec. III-B of Alexiadis et al. (IEEE TCSVT 2017): weighted
Gaussian splat of oriented points (eqs. (1)-(2)), forward 3D FFT of the three
components, integration filter j w / |w|^2, inverse FFT and component sum,
iso-level at the input points, marching cubes.

There is no CPU fallback: if the library is missing, importing works but every
call raises ``FvrUnavailable``.
"""
from __future__ import annotations

import ctypes
import os
from collections import namedtuple

__all__ = [
    "FvrError", "FvrUnavailable", "Context", "PreparedFrame", "Batch", "PreparedBatch", "Server", "Mesh",
    "reconstruct", "indicator",
    "extract", "debug_splat", "mc_table", "check_grid", "check_frame", "library_path", "load_library",
    "STATUS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfvr.so")

STATUS = {0: "FVR_OK", -1: "FVR_E_INVALID", -2: "FVR_E_UNSUPPORTED", -3: "FVR_E_NOMEM",
          -4: "FVR_E_CAPACITY", -5: "FVR_E_DEVICE", -6: "FVR_E_RANGE"}
FVR_FLAG_OPEN_SURFACE = 1


class FvrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class FvrUnavailable(RuntimeError):
    pass


class _Frame(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("normals", ctypes.c_void_p),
                ("weights", ctypes.c_void_p), ("n_points", ctypes.c_int64),
                ("dims", ctypes.c_int32 * 3), ("bbox", ctypes.c_float * 6),
                ("options", ctypes.c_uint32)]


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "busy_tiles", "tiles", "nonzero_planes", "planes", "mc_blocks_listed", "mc_blocks",
        "points_used", "points_rejected")]


class _DepthViews(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("cameras", ctypes.c_void_p), ("views", ctypes.c_int32),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("step_threshold", ctypes.c_float),
                ("box_radius", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("normals", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("n_points", ctypes.c_int64), ("dims", ctypes.c_int32 * 3), ("bbox", ctypes.c_float * 6),
                ("options", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("vertices", ctypes.c_void_p),
                ("triangles", ctypes.c_void_p), ("normals_out", ctypes.c_void_p),
                ("vertex_capacity", ctypes.c_int64), ("triangle_capacity", ctypes.c_int64),
                ("user", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int), ("n_vertices", ctypes.c_int64),
                ("n_triangles", ctypes.c_int64), ("n_rejected", ctypes.c_int64), ("level", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("user", ctypes.c_void_p), ("submit_ms", ctypes.c_double),
                ("admit_ms", ctypes.c_double), ("done_ms", ctypes.c_double), ("error", ctypes.c_char * 96)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "pending", "in_flight", "results_waiting", "admitted", "completed", "refused", "max_in_flight",
        "device_bytes", "budget")]


class _Mesh(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("triangles", ctypes.c_void_p),
                ("vertex_capacity", ctypes.c_int64), ("triangle_capacity", ctypes.c_int64),
                ("n_vertices", ctypes.c_int64), ("n_triangles", ctypes.c_int64),
                ("level", ctypes.c_double), ("n_rejected", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("normals", ctypes.c_void_p)]


FVR_SPLAT_NEAREST = 1
# splat variants of Sec. III-B: the weighted Gaussian splat of eqs. (1)-(2),
# and the non-weighted one (each normal to its nearest voxel, mean per voxel)
SPLATS = {"gaussian": 0, "nearest": FVR_SPLAT_NEAREST}
# spectrum storage between the transform passes (computation is float32)
STORAGES = {"f32": 0, "bf16": 2, "fp16": 4}

Mesh = namedtuple("Mesh", "vertices triangles level n_rejected open_surface normals", defaults=(None,))


def _fill_mesh(m, out):
    """Point a _Mesh at output buffers (vertices, triangles[, normals])."""
    verts, tris = out[0], out[1]
    nrm = out[2] if len(out) > 2 else None
    m.vertices = verts.data_ptr()
    m.triangles = tris.data_ptr()
    m.normals = nrm.data_ptr() if nrm is not None else None
    m.vertex_capacity = verts.shape[0] if nrm is None else min(verts.shape[0], nrm.shape[0])
    m.triangle_capacity = tris.shape[0]


def _result(m, out):
    """Mesh of a finished call as views of its output buffers."""
    nrm = out[2][:m.n_vertices] if len(out) > 2 and out[2] is not None else None
    return Mesh(out[0][:m.n_vertices], out[1][:m.n_triangles], m.level, int(m.n_rejected),
                bool(m.flags & FVR_FLAG_OPEN_SURFACE), nrm)

_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libfvr.so (raises FvrUnavailable if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise FvrUnavailable(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.fvr_create.argtypes = [I, P, ctypes.POINTER(P)]
    lib.fvr_destroy.argtypes = [P]
    lib.fvr_destroy.restype = None
    lib.fvr_set_stream.argtypes = [P, P]
    lib.fvr_reconstruct.argtypes = [P, ctypes.POINTER(_Frame), ctypes.POINTER(_Mesh)]
    lib.fvr_reconstruct_noalloc.argtypes = [P, ctypes.POINTER(_Frame), ctypes.POINTER(_Mesh)]
    lib.fvr_indicator.argtypes = [P, ctypes.POINTER(_Frame), P, ctypes.POINTER(ctypes.c_double)]
    lib.fvr_extract.argtypes = [P, P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                                ctypes.c_float, ctypes.POINTER(_Mesh), P]
    lib.fvr_debug_splat.argtypes = [P, ctypes.POINTER(_Frame), P]
    lib.fvr_check_grid.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
    lib.fvr_check_frame.argtypes = [ctypes.POINTER(_Frame)]
    lib.fvr_last_stats.argtypes = [P, ctypes.POINTER(_Stats)]
    lib.fvr_depth_to_points.argtypes = [P, ctypes.POINTER(_DepthViews), P, P, P, i64,
                                        ctypes.POINTER(i64)]
    lib.fvr_server_create.argtypes = [I, I, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.fvr_server_destroy.argtypes = [P]
    lib.fvr_server_destroy.restype = None
    lib.fvr_server_submit.argtypes = [P, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.fvr_server_poll.argtypes = [P, ctypes.POINTER(_Result), I, ctypes.POINTER(I)]
    lib.fvr_server_info.argtypes = [P, ctypes.POINTER(_ServerStats)]
    lib.fvr_server_last_error.argtypes = [P]
    lib.fvr_server_last_error.restype = ctypes.c_char_p
    lib.fvr_batch_create.argtypes = [I, P, I, ctypes.POINTER(P)]
    lib.fvr_batch_destroy.argtypes = [P]
    lib.fvr_batch_destroy.restype = None
    lib.fvr_batch_set_stream.argtypes = [P, P]
    lib.fvr_batch_use_graph.argtypes = [P, I]
    lib.fvr_batch_reconstruct.argtypes = [P, ctypes.POINTER(_Frame), ctypes.POINTER(_Mesh), I]
    lib.fvr_batch_last_error.argtypes = [P]
    lib.fvr_batch_last_error.restype = ctypes.c_char_p
    lib.fvr_mc_table.argtypes = [P, P]
    lib.fvr_timing_enable.argtypes = [P, I]
    lib.fvr_timing_select.argtypes = [P, ctypes.c_uint32]
    lib.fvr_timing_reset.argtypes = [P]
    lib.fvr_timing_count.argtypes = []
    lib.fvr_timing_name.argtypes = [I]
    lib.fvr_timing_name.restype = ctypes.c_char_p
    lib.fvr_timing_get.argtypes = [P, I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.fvr_status_string.argtypes = [I]
    lib.fvr_status_string.restype = ctypes.c_char_p
    lib.fvr_last_error.argtypes = [P]
    lib.fvr_last_error.restype = ctypes.c_char_p
    for fn in ("fvr_create", "fvr_set_stream", "fvr_reconstruct", "fvr_reconstruct_noalloc",
               "fvr_indicator", "fvr_extract",
               "fvr_debug_splat", "fvr_check_grid", "fvr_check_frame", "fvr_last_stats", "fvr_mc_table",
               "fvr_timing_enable", "fvr_depth_to_points", "fvr_server_create", "fvr_server_submit",
               "fvr_server_poll", "fvr_server_info", "fvr_batch_create", "fvr_batch_set_stream", "fvr_batch_use_graph",
               "fvr_batch_reconstruct",
               "fvr_timing_select", "fvr_timing_reset", "fvr_timing_get"):
        getattr(lib, fn).restype = I
    _lib = lib
    return lib


def _check(lib, status, ctx=None):
    if status != 0:
        msg = lib.fvr_last_error(ctx)
        raise FvrError(status, msg.decode() if msg else "")


def check_grid(dims, bbox) -> int:
    """Host-only validation of dims/bbox; returns the fvr_status code."""
    lib = load_library()
    d = (ctypes.c_int32 * 3)(*[int(x) for x in dims])
    b = (ctypes.c_float * 6)(*[float(x) for x in bbox])
    return int(lib.fvr_check_grid(d, b))


def check_frame(n_points, grid_dim, bbox, points_ptr=1, normals_ptr=1, weights_ptr=0, options=0) -> int:
    """Host-only validation of a frame's host-side fields (point count,
    required pointers, grid, bbox, option bits) as ``fvr_reconstruct`` does
    before any launch; the pointers are not dereferenced.  Returns the
    fvr_status code."""
    lib = load_library()
    f = _Frame()
    f.points, f.normals, f.weights = points_ptr or None, normals_ptr or None, weights_ptr or None
    f.n_points = int(n_points)
    f.dims = (ctypes.c_int32 * 3)(*[int(x) for x in grid_dim])
    f.bbox = (ctypes.c_float * 6)(*[float(x) for x in bbox])
    f.options = int(options)
    return int(lib.fvr_check_frame(ctypes.byref(f)))


def mc_table():
    """The library's generated marching-cubes table as numpy arrays
    (counts uint8[256], edges int8[256, 15])."""
    import numpy as np
    lib = load_library()
    counts = np.zeros(256, np.uint8)
    edges = np.zeros((256, 15), np.int8)
    _check(lib, lib.fvr_mc_table(counts.ctypes.data, edges.ctypes.data))
    return counts, edges


def _torch():
    import torch
    return torch


def _dev_f32(t, name, device, ncols):
    """t as a contiguous float32 (n, ncols) tensor on cuda:device (checked)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.get_device() != device:
        raise ValueError(f"{name} must live on cuda:{device}")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.dim() != 2 or t.shape[1] != ncols:
        raise ValueError(f"{name} has shape {tuple(t.shape)}")
    return t if t.is_contiguous() else t.contiguous()


class PreparedFrame:
    """One frame's marshalled fvr_reconstruct call (``Context.prepare``)."""

    def __init__(self, ctx, frame, keep, out, stream):
        self._ctx, self._f, self._keep, self._stream = ctx, frame, keep, stream
        self._out = tuple(out)
        self.vertices_buf, self.triangles_buf = self._out[0], self._out[1]
        m = _Mesh()
        _fill_mesh(m, self._out)
        self._m = m
        self._vcap, self._tcap = m.vertex_capacity, m.triangle_capacity
        self._args = (ctx.handle, ctypes.byref(frame), ctypes.byref(m))
        self._fn = ctx.lib.fvr_reconstruct

    def run(self):
        """Sec. III-B end to end on the frame's current contents; returns
        (n_vertices, n_triangles), the leading rows of the output buffers."""
        ctx = self._ctx
        if ctx._cur_stream != self._stream:
            _check(ctx.lib, ctx.lib.fvr_set_stream(ctx.handle, ctypes.c_void_p(self._stream)), ctx.handle)
            ctx._cur_stream = self._stream
        m = self._m
        m.vertex_capacity = self._vcap
        m.triangle_capacity = self._tcap
        st = self._fn(*self._args)
        if st:
            _check(ctx.lib, st, ctx.handle)
        return m.n_vertices, m.n_triangles

    def mesh(self) -> Mesh:
        """The last run's result as views of the output buffers."""
        return _result(self._m, self._out)


class Context:
    """An fvr_ctx on one device: resident FFT plans, twiddles and scratch."""

    def __init__(self, device: int | None = None):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.fvr_create(self.device, None, ctypes.byref(h)))
        self.handle = h
        self._cur_stream = None  # the stream last passed to fvr_set_stream (None: the null stream)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fvr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ------------------------------------------------------------
    def _stream(self):
        """Enqueue on torch's current stream of the device (the library call
        only when that stream changed)."""
        torch = _torch()
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._cur_stream:
            _check(self.lib, self.lib.fvr_set_stream(self.handle, ctypes.c_void_p(s)), self.handle)
            self._cur_stream = s

    def _frame(self, points, normals, weights, grid_dim, bbox, splat="gaussian", storage="f32"):
        points = _dev_f32(points, "points", self.device, 3)
        normals = _dev_f32(normals, "normals", self.device, 3)
        if normals.shape[0] != points.shape[0]:
            raise ValueError("points and normals differ in length")
        if weights is not None:
            weights = _dev_f32(weights.reshape(-1, 1), "weights", self.device, 1)
            if weights.shape[0] != points.shape[0]:
                raise ValueError("weights length differs from points")
        f = _Frame()
        m = points.shape[0]
        f.points = points.data_ptr() if m else None
        f.normals = normals.data_ptr() if m else None
        f.weights = weights.data_ptr() if (weights is not None and m) else None
        f.n_points = m
        gd = (grid_dim,) * 3 if isinstance(grid_dim, int) else tuple(grid_dim)
        f.dims[:] = [int(x) for x in gd]
        f.bbox[:] = [float(x) for x in _flat_bbox(bbox)]
        if splat not in SPLATS:
            raise ValueError(f"splat must be one of {sorted(SPLATS)}")
        if storage not in STORAGES:
            raise ValueError(f"storage must be one of {sorted(STORAGES)}")
        f.options = SPLATS[splat] | STORAGES[storage]
        return f, (points, normals, weights)

    def _run_mesh(self, call, dims, out, vcap, tcap, want_normals=False):
        torch = _torch()
        dev = f"cuda:{self.device}"
        if out is None:
            if vcap is None:
                nx, ny, nz = dims
                vcap = max(4096, 6 * (nx * ny + ny * nz + nx * nz))
            if tcap is None:
                tcap = 2 * vcap
        for attempt in range(2):
            if out is not None:
                bufs = tuple(out)
            else:
                bufs = (torch.empty((vcap, 3), dtype=torch.float32, device=dev),
                        torch.empty((tcap, 3), dtype=torch.int32, device=dev))
                if want_normals:
                    bufs += (torch.empty((vcap, 3), dtype=torch.float32, device=dev),)
            m = _Mesh()
            _fill_mesh(m, bufs)
            st = call(m)
            if st == -4 and attempt == 0 and out is None:
                vcap, tcap = max(m.n_vertices, 1), max(m.n_triangles, 1)
                continue
            _check(self.lib, st, self.handle)
            break
        return _result(m, bufs)

    # -- API ----------------------------------------------------------------
    def reconstruct(self, points, normals, weights=None, grid_dim=(128, 128, 128),
                    bbox=((-1, -1, -1), (1, 1, 1)), out=None, vertex_capacity=None,
                    triangle_capacity=None, vertex_normals=False, splat="gaussian",
                    storage="f32") -> Mesh:
        """Sec. III-B end to end: returns Mesh(vertices [V,3] f32, triangles
        [T,3] i32, level, n_rejected, open_surface, normals [V,3] f32 or
        None).  ``out`` = (verts, tris[, normals]) preallocated buffers, used
        without retry; ``vertex_normals`` asks for normals when out is None;
        ``splat`` is "gaussian" (eqs. (1)-(2)) or "nearest"; ``storage`` the
        spectra's storage between passes ("f32", "bf16", "fp16")."""
        f, keep = self._frame(points, normals, weights, grid_dim, bbox, splat, storage)
        self._stream()
        dims = tuple(f.dims)
        return self._run_mesh(lambda m: self.lib.fvr_reconstruct(self.handle, ctypes.byref(f),
                                                                 ctypes.byref(m)),
                              dims, out, vertex_capacity, triangle_capacity, vertex_normals)

    def depth_to_points(self, depth, cameras, step_threshold=0.05, box_radius=10, capacity=None):
        """The front end of Sec. III-A on the device: depth (K, H, W) float32
        tensor on this device (metres; <= 0 is background), cameras (K, 16)
        array (fx, fy, cx, cy, R row-major camera to world, t).  Returns
        (points [M,3], normals [M,3], weights [M]) float32 tensors."""
        import numpy as np
        torch = _torch()
        if depth.device.type != "cuda" or depth.device.index != self.device:
            raise ValueError(f"depth must live on cuda:{self.device}")
        if depth.dtype != torch.float32 or depth.dim() != 3:
            raise TypeError("depth must be a (K, H, W) float32 tensor")
        depth = depth.contiguous()
        K, H, W = depth.shape
        cams = np.ascontiguousarray(np.asarray(cameras, np.float32).reshape(K, 16))
        cap = K * H * W if capacity is None else int(capacity)
        dev = f"cuda:{self.device}"
        pts = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
        nrm = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
        w = torch.empty((max(cap, 1),), dtype=torch.float32, device=dev)
        dv = _DepthViews(depth.data_ptr(), cams.ctypes.data, K, H, W, float(step_threshold), int(box_radius))
        n = ctypes.c_int64()
        self._stream()
        _check(self.lib, self.lib.fvr_depth_to_points(self.handle, ctypes.byref(dv), pts.data_ptr(),
                                                      nrm.data_ptr(), w.data_ptr(), cap, ctypes.byref(n)),
               self.handle)
        m = n.value
        return pts[:m], nrm[:m], w[:m]

    def last_stats(self) -> dict:
        """Work counters of the last reconstruction or indicator call
        (``fvr_last_stats``): busy splat tiles, non-zero z planes, listed
        marching-cubes blocks, points used and rejected."""
        st = _Stats()
        _check(self.lib, self.lib.fvr_last_stats(self.handle, ctypes.byref(st)), self.handle)
        return {n: int(getattr(st, n)) for n, _ in _Stats._fields_}

    def reconstruct_noalloc(self, points, normals, weights=None, grid_dim=(128, 128, 128),
                            bbox=((-1, -1, -1), (1, 1, 1)), out=None, splat="gaussian", storage="f32") -> Mesh:
        """``reconstruct`` through ``fvr_reconstruct_noalloc``: the library
        allocates no device memory in the call (its scratch is the device's
        static array of FVR_NOALLOC_SCRATCH_BYTES).  ``out`` = (verts, tris)
        is required; a capacity shortfall or a frame beyond the static
        scratch raises FvrError."""
        if out is None:
            raise ValueError("reconstruct_noalloc needs preallocated out=(vertices, triangles)")
        f, keep = self._frame(points, normals, weights, grid_dim, bbox, splat, storage)
        self._stream()
        m = _Mesh()
        _fill_mesh(m, out)
        _check(self.lib, self.lib.fvr_reconstruct_noalloc(self.handle, ctypes.byref(f), ctypes.byref(m)),
               self.handle)
        return _result(m, out)

    def prepare(self, points, normals, weights=None, grid_dim=(128, 128, 128),
                bbox=((-1, -1, -1), (1, 1, 1)), out=None, vertex_capacity=None,
                triangle_capacity=None, splat="gaussian", storage="f32") -> "PreparedFrame":
        """A frame for repeated reconstruction: the tensors are checked and
        the call's arguments marshalled once.  ``run()`` then enqueues the
        same work as ``reconstruct`` on the stream that was current here,
        reading the tensors' contents at each call (a serving loop refills
        the same input and output buffers between runs).  The output
        buffers are ``out`` or allocated once; a capacity shortfall raises."""
        f, keep = self._frame(points, normals, weights, grid_dim, bbox, splat, storage)
        self._stream()
        torch = _torch()
        if out is None:
            nx, ny, nz = tuple(f.dims)
            vcap = vertex_capacity or max(4096, 6 * (nx * ny + ny * nz + nx * nz))
            tcap = triangle_capacity or 2 * vcap
            out = (torch.empty((vcap, 3), dtype=torch.float32, device=f"cuda:{self.device}"),
                   torch.empty((tcap, 3), dtype=torch.int32, device=f"cuda:{self.device}"))
        return PreparedFrame(self, f, keep, out, self._cur_stream)

    def indicator(self, points, normals, weights=None, grid_dim=(128, 128, 128),
                  bbox=((-1, -1, -1), (1, 1, 1)), splat="gaussian", storage="f32"):
        """Steps up to the iso-level: returns (A [Nz, Ny, Nx] f32 tensor, L)."""
        torch = _torch()
        f, keep = self._frame(points, normals, weights, grid_dim, bbox, splat, storage)
        self._stream()
        nx, ny, nz = tuple(f.dims)
        A = torch.empty((nz, ny, nx), dtype=torch.float32, device=f"cuda:{self.device}")
        lvl = ctypes.c_double()
        _check(self.lib, self.lib.fvr_indicator(self.handle, ctypes.byref(f), A.data_ptr(),
                                                ctypes.byref(lvl)), self.handle)
        return A, lvl.value

    def extract(self, field, bbox, level, with_cases=False, out=None, vertex_capacity=None,
                triangle_capacity=None, vertex_normals=False):
        """Marching cubes of a device field (Nz, Ny, Nx) at ``level``.
        Returns Mesh, plus the case bytes (Nz-1, Ny-1, Nx-1) if requested."""
        torch = _torch()
        if field.device.type != "cuda" or field.device.index != self.device:
            raise ValueError(f"field must live on cuda:{self.device}")
        if field.dtype != torch.float32 or field.dim() != 3:
            raise TypeError("field must be a 3D float32 tensor")
        field = field.contiguous()
        nz, ny, nx = field.shape
        d = (ctypes.c_int32 * 3)(nx, ny, nz)
        b = (ctypes.c_float * 6)(*[float(x) for x in _flat_bbox(bbox)])
        cases = None
        if with_cases:
            cases = torch.empty((nz - 1, ny - 1, nx - 1), dtype=torch.uint8,
                                device=f"cuda:{self.device}")
        self._stream()
        mesh = self._run_mesh(
            lambda m: self.lib.fvr_extract(self.handle, field.data_ptr(), d, b, float(level),
                                           ctypes.byref(m), cases.data_ptr() if cases is not None else None),
            (nx, ny, nz), out, vertex_capacity, triangle_capacity, vertex_normals)
        return (mesh, cases) if with_cases else mesh

    def debug_splat(self, points, normals, weights=None, grid_dim=(128, 128, 128),
                    bbox=((-1, -1, -1), (1, 1, 1)), splat="gaussian"):
        """The splat kernel's V field (3, Nz, Ny, Nx) f32."""
        torch = _torch()
        f, keep = self._frame(points, normals, weights, grid_dim, bbox, splat)
        self._stream()
        nx, ny, nz = tuple(f.dims)
        V = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=f"cuda:{self.device}")
        _check(self.lib, self.lib.fvr_debug_splat(self.handle, ctypes.byref(f), V.data_ptr()),
               self.handle)
        return V

    # -- timing -------------------------------------------------------------
    def timing(self, enable: bool = True):
        _check(self.lib, self.lib.fvr_timing_enable(self.handle, 1 if enable else 0), self.handle)

    def timing_select(self, names):
        """Record HIP events around the named kernels only."""
        index = {self.lib.fvr_timing_name(i).decode(): i for i in range(self.lib.fvr_timing_count())}
        mask = 0
        for n in names:
            mask |= 1 << index[n]
        _check(self.lib, self.lib.fvr_timing_select(self.handle, ctypes.c_uint32(mask)), self.handle)

    def timing_reset(self):
        _check(self.lib, self.lib.fvr_timing_reset(self.handle), self.handle)

    def timings(self) -> dict:
        """{kernel name: (total ms, launches)} from HIP events."""
        out = {}
        for i in range(self.lib.fvr_timing_count()):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            _check(self.lib, self.lib.fvr_timing_get(self.handle, i, ctypes.byref(ms), ctypes.byref(n)))
            out[self.lib.fvr_timing_name(i).decode()] = (ms.value, n.value)
        return out


def _flat_bbox(bbox):
    b = list(bbox)
    if len(b) == 2:
        return [float(x) for x in b[0]] + [float(x) for x in b[1]]
    if len(b) != 6:
        raise ValueError("bbox must be (lo, hi) or 6 floats")
    return [float(x) for x in b]


_default = {}


def _ctx(device=None) -> Context:
    torch = _torch()
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _default:
        _default[d] = Context(d)
    return _default[d]


def reconstruct(points, normals, weights=None, grid_dim=(128, 128, 128),
                bbox=((-1, -1, -1), (1, 1, 1)), **kw) -> Mesh:
    """Module-level convenience over a per-device default Context."""
    return _ctx(points.device.index).reconstruct(points, normals, weights, grid_dim, bbox, **kw)


def indicator(points, normals, weights=None, grid_dim=(128, 128, 128),
              bbox=((-1, -1, -1), (1, 1, 1)), **kw):
    return _ctx(points.device.index).indicator(points, normals, weights, grid_dim, bbox, **kw)


def extract(field, bbox, level, with_cases=False, **kw):
    return _ctx(field.device.index).extract(field, bbox, level, with_cases, **kw)


def debug_splat(points, normals, weights=None, grid_dim=(128, 128, 128),
                bbox=((-1, -1, -1), (1, 1, 1)), **kw):
    return _ctx(points.device.index).debug_splat(points, normals, weights, grid_dim, bbox, **kw)


class Batch:
    """An fvr_batch: frames reconstructed together as one captured HIP graph
    over ``slots`` per-slot contexts (scratch, status, stream each), frame i
    on slot i mod slots.  Each frame's mesh is the one ``Context.reconstruct``
    gives for it, bit for bit."""

    def __init__(self, slots: int = 4, device: int | None = None, graph: bool = True):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        st = self.lib.fvr_batch_create(self.device, None, int(slots), ctypes.byref(h))
        if st:
            raise FvrError(st, (self.lib.fvr_batch_last_error(None) or b"").decode())
        self.handle = h
        self.slots = int(slots)
        self.use_graph(graph)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fvr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def use_graph(self, enable: bool):
        self._check(self.lib.fvr_batch_use_graph(self.handle, 1 if enable else 0))

    def _check(self, st):
        if st:
            raise FvrError(st, (self.lib.fvr_batch_last_error(self.handle) or b"").decode())

    def prepare(self, frames, outs):
        """Marshal a list of frames once: ``frames`` holds (points, normals,
        weights, grid_dim, bbox) tuples of device tensors, ``outs`` the
        (vertices, triangles) buffers of each.  Returns a PreparedBatch whose
        ``run()`` reconstructs them all (the same call each time, so the
        captured graph is replayed)."""
        return PreparedBatch(self, frames, outs)

    def reconstruct(self, frames, outs):
        """One batch call; returns the list of Mesh results."""
        pb = self.prepare(frames, outs)
        pb.run()
        return pb.meshes()


class PreparedBatch:
    def __init__(self, batch, frames, outs):
        if len(frames) != len(outs):
            raise ValueError("one (vertices, triangles) pair per frame")
        self._batch = batch
        n = len(frames)
        self._n = n
        self._frames = (_Frame * max(n, 1))()
        self._meshes = (_Mesh * max(n, 1))()
        self._keep = []
        helper = Context.__new__(Context)  # marshalling only: no fvr_ctx is made
        helper.device = batch.device
        for i, (fr, o) in enumerate(zip(frames, outs)):
            points, normals, weights, grid_dim, bbox = fr[:5]
            f, keep = Context._frame(helper, points, normals, weights, grid_dim, bbox,
                                     fr[5] if len(fr) > 5 else "gaussian")
            self._frames[i] = f
            self._keep.append((keep, tuple(o)))
            _fill_mesh(self._meshes[i], tuple(o))

    def run(self):
        torch = _torch()
        b = self._batch
        # the batch forks from a stream of its own: work already queued on
        # torch's stream (uploads of the inputs) must be complete first
        torch.cuda.current_stream(b.device).synchronize()
        b._check(b.lib.fvr_batch_reconstruct(b.handle, self._frames, self._meshes, self._n))
        return [(m.n_vertices, m.n_triangles) for m in self._meshes[:self._n]]

    def meshes(self):
        return [_result(self._meshes[i], self._keep[i][1]) for i in range(self._n)]


class Server:
    """An fvr_server: continuous batching over ``slots`` device slots within
    a device-memory budget (``fvr_server_*``).  ``submit`` takes host arrays
    (numpy float32, or pinned torch CPU tensors), ``poll`` returns finished
    results with their meshes as numpy arrays."""

    def __init__(self, slots: int = 4, hbm_budget: int = 16 << 30, device: int | None = None):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        st = self.lib.fvr_server_create(self.device, int(slots), int(hbm_budget), ctypes.byref(h))
        if st:
            raise FvrError(st, (self.lib.fvr_server_last_error(None) or b"").decode())
        self.handle = h
        self._live = {}  # ticket -> (request, inputs and outputs kept alive)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fvr_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _host(a, name, ncols):
        import numpy as np
        try:
            import torch
            if isinstance(a, torch.Tensor):
                if a.device.type != "cpu" or a.dtype != torch.float32 or not a.is_contiguous():
                    raise TypeError(f"{name}: a contiguous float32 CPU tensor")
                return a, a.data_ptr(), bool(a.is_pinned())
        except ImportError:
            pass
        arr = np.ascontiguousarray(a, dtype=np.float32)
        if ncols > 1 and (arr.ndim != 2 or arr.shape[1] != ncols):
            raise ValueError(f"{name} has shape {arr.shape}")
        return arr, arr.ctypes.data, False

    def submit(self, points, normals, weights=None, grid_dim=(128, 128, 128), bbox=((-1, -1, -1), (1, 1, 1)),
               splat="gaussian", vertex_capacity=None, triangle_capacity=None, vertex_normals=False,
               user=None, storage="f32") -> int:
        import numpy as np
        if splat not in SPLATS:
            raise ValueError(f"splat must be one of {sorted(SPLATS)}")
        if storage not in STORAGES:
            raise ValueError(f"storage must be one of {sorted(STORAGES)}")
        p, pp, pin_p = self._host(points, "points", 3)
        n, pn, pin_n = self._host(normals, "normals", 3)
        keep = [p, n]
        pw, pin_w = None, True
        if weights is not None:
            w, pw, pin_w = self._host(weights, "weights", 1)
            keep.append(w)
        gd = (grid_dim,) * 3 if isinstance(grid_dim, int) else tuple(grid_dim)
        nx, ny, nz = (int(x) for x in gd)
        vcap = vertex_capacity or max(4096, 6 * (nx * ny + ny * nz + nx * nz))
        tcap = triangle_capacity or 2 * vcap
        verts = np.empty((vcap, 3), np.float32)
        tris = np.empty((tcap, 3), np.int32)
        nrm = np.empty((vcap, 3), np.float32) if vertex_normals else None
        q = _Request()
        q.points, q.normals, q.weights = pp, pn, pw
        q.n_points = int(p.shape[0])
        q.dims[:] = [nx, ny, nz]
        q.bbox[:] = [float(x) for x in _flat_bbox(bbox)]
        q.options = SPLATS[splat] | STORAGES[storage]
        q.flags = 1 if (pin_p and pin_n and pin_w) else 0
        q.vertices, q.triangles = verts.ctypes.data, tris.ctypes.data
        q.normals_out = nrm.ctypes.data if nrm is not None else None
        q.vertex_capacity, q.triangle_capacity = vcap, tcap
        t = ctypes.c_uint64()
        st = self.lib.fvr_server_submit(self.handle, ctypes.byref(q), ctypes.byref(t))
        if st:
            raise FvrError(st, (self.lib.fvr_server_last_error(self.handle) or b"").decode())
        self._live[t.value] = (q, keep, verts, tris, nrm, user)
        return t.value

    def poll(self, max_results: int = 64) -> list:
        out = (_Result * max_results)()
        n = ctypes.c_int()
        st = self.lib.fvr_server_poll(self.handle, out, max_results, ctypes.byref(n))
        if st:
            raise FvrError(st, (self.lib.fvr_server_last_error(self.handle) or b"").decode())
        res = []
        for r in out[:n.value]:
            q, keep, verts, tris, nrm, user = self._live.pop(r.ticket)
            ok = r.status == 0
            res.append({"ticket": r.ticket, "status": r.status, "error": r.error.decode(),
                        "vertices": verts[:r.n_vertices] if ok else None,
                        "triangles": tris[:r.n_triangles] if ok else None,
                        "normals": nrm[:r.n_vertices] if (ok and nrm is not None) else None,
                        "n_vertices": r.n_vertices, "n_triangles": r.n_triangles, "level": r.level,
                        "open_surface": bool(r.flags & FVR_FLAG_OPEN_SURFACE), "n_rejected": r.n_rejected,
                        "latency_ms": r.done_ms - r.submit_ms, "queue_ms": r.admit_ms - r.submit_ms,
                        "submit_ms": r.submit_ms, "done_ms": r.done_ms, "user": user})
        return res

    def info(self) -> dict:
        st = _ServerStats()
        self.lib.fvr_server_info(self.handle, ctypes.byref(st))
        return {n: int(getattr(st, n)) for n, _ in _ServerStats._fields_}

    def drain(self, timeout_s: float = 60.0) -> list:
        """Poll until every submitted request has a result."""
        import time
        out = []
        t0 = time.perf_counter()
        while self._live:
            out += self.poll()
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"{len(self._live)} requests unfinished")
        return out
