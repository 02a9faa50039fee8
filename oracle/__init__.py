"""FP64 CPU oracle for the volumetric FT surface reconstruction (Sec. III-B).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg import this module.  It shares no code with the
GPU library (``paper_1712_03084_amd``) and never imports it.

Steps, each a plain and literal rendering of the method:

  splat      eqs. (1)-(2): weighted Gaussian splat of normals, V = S / D
             (C loops, ``fvr_oracle.c``)
  indicator  forward 3D DFT of each component of V, integration filter
             j w_c / |w|^2, inverse 3D DFT, sum of the components
             (numpy's FFT as the transform primitive)
  level      mean of the trilinearly sampled A at the accepted input points
             (C loop, compensated sum)
  extract    marching cubes with the rule-generated table (``mc_rule``)
             and a welded, indexed mesh, with optional vertex normals
             (C loops)
  splat_nearest  the non-weighted splat: each normal to its nearest voxel,
             mean per voxel (C loop)
  frontend   depth maps to oriented, weighted points (Sec. III-A; numpy)

Readings of points the paper leaves open are stated where they are used.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import frontend, mc_rule  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fvr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

__all__ = ["build", "splat", "splat_nearest", "indicator", "level", "mc_table", "extract",
           "reconstruct", "geometry", "open_surface"]


def build(force: bool = True) -> str:
    """Compile the oracle's C part with gcc (no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_splat.argtypes = [P, P, P, i64, P, P, P, P, P, ctypes.c_int]
        lib.oracle_splat.restype = i64
        lib.oracle_splat_nearest.argtypes = [P, P, i64, P, P, P, P, P]
        lib.oracle_splat_nearest.restype = i64
        lib.oracle_level.argtypes = [P, P, P, P, i64, P]
        lib.oracle_level.restype = ctypes.c_double
        lib.oracle_marching_cubes.argtypes = [P, P, P, ctypes.c_double, P, P,
                                              P, i64, P, i64, P, P, P, ctypes.c_int, P]
        lib.oracle_marching_cubes.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f32c(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def geometry(dims, bbox):
    """Voxel size h, sigma1 and sigma2 (text after eq. 2) in float64."""
    b = np.asarray(bbox, np.float32).astype(np.float64)
    h = (b[3:] - b[:3]) / np.asarray(dims, np.float64)
    s1 = 0.5 * float(np.sqrt(np.sum(h * h)))
    return h, s1, s1 * np.sqrt(1.5)


def splat(points, normals, weights, dims, bbox, threads: int = 1):
    """Eqs. (1)-(2).  Returns (V, S, D, n_rejected); V and S have shape
    (3, Nz, Ny, Nx), D has shape (Nz, Ny, Nx).  weights None means all 1.
    threads > 1 splits the voxel planes over OpenMP threads; every voxel
    still sums its terms in input order (the same bits)."""
    lib = _load()
    p = _f32c(points).reshape(-1, 3)
    nrm = _f32c(normals).reshape(-1, 3)
    w = None if weights is None else _f32c(weights).reshape(-1)
    m = p.shape[0]
    d = np.asarray(dims, np.int32)
    b = np.asarray(bbox, np.float32)
    Nx, Ny, Nz = (int(x) for x in dims)
    S = np.empty((3, Nz, Ny, Nx))
    D = np.empty((Nz, Ny, Nx))
    V = np.empty((3, Nz, Ny, Nx))
    rej = lib.oracle_splat(_ptr(p), _ptr(nrm), _ptr(w), m, _ptr(d), _ptr(b),
                           _ptr(S), _ptr(D), _ptr(V), int(threads))
    return V, S, D, int(rej)


def splat_nearest(points, normals, dims, bbox):
    """The non-weighted splat of Sec. III-B: each sample to its nearest
    voxel, V = mean of the normals per voxel (0 where none).  Returns
    (V (3, Nz, Ny, Nx), counts (Nz, Ny, Nx) int64, n_rejected)."""
    lib = _load()
    p = _f32c(points).reshape(-1, 3)
    nrm = _f32c(normals).reshape(-1, 3)
    Nx, Ny, Nz = (int(x) for x in dims)
    S = np.empty((3, Nz, Ny, Nx))
    cnt = np.empty((Nz, Ny, Nx), np.int64)
    V = np.empty((3, Nz, Ny, Nx))
    rej = lib.oracle_splat_nearest(_ptr(p), _ptr(nrm), p.shape[0], _ptr(np.asarray(dims, np.int32)),
                                   _ptr(np.asarray(bbox, np.float32)), _ptr(S), _ptr(cnt), _ptr(V))
    return V, cnt, int(rej)


def _wavenumbers(n: int) -> np.ndarray:
    """Signed wavenumber kappa of each DFT bin: k for k < N/2, k - N above;
    the Nyquist bin k = N/2 gets -N/2."""
    return np.fft.fftfreq(n, d=1.0 / n)


def filter_factors(dims, bbox):
    """Per-axis spectral factors of the integration filter of Sec. III-B.

    Returns (wx, wy, wz, inv_w2) broadcastable to (Nz, Ny, Nx):
      w_a = 2 pi kappa_a / L_a (physical angular frequency; L_a = box extent)
      the derivative factor j w_a is zeroed on axis a's Nyquist plane
      (reading: the Nyquist derivative of a real sampled field is undefined;
      zeroing it keeps the filtered field real),
      inv_w2 = 1 / |w|^2 with 0 at the DC bin (the filter is singular there;
      zero makes A zero-mean).
    """
    Nx, Ny, Nz = (int(x) for x in dims)
    b = np.asarray(bbox, np.float32).astype(np.float64)
    L = b[3:] - b[:3]
    out = []
    for n, ext in ((Nx, L[0]), (Ny, L[1]), (Nz, L[2])):
        kap = _wavenumbers(n)
        w = 2.0 * np.pi * kap / ext
        out.append((w, np.where(np.arange(n) == n // 2, 0.0, w)))
    (wx, dx), (wy, dy), (wz, dz) = out
    w2 = wx[None, None, :] ** 2 + wy[None, :, None] ** 2 + wz[:, None, None] ** 2
    with np.errstate(divide="ignore"):
        inv = np.where(w2 > 0, 1.0 / np.where(w2 > 0, w2, 1.0), 0.0)
    return dx[None, None, :], dy[None, :, None], dz[:, None, None], inv


def indicator(V, dims, bbox, return_imag: bool = False, threads: int = 1):
    """Spectral integration of Sec. III-B, taken literally.

    For each component c: V^_c = DFT3(V_c) (unnormalised, exp(-i...)),
    A^_c = j w_c V^_c / |w|^2, A_c = inverse DFT3 (with 1/n); then
    A = sum_c Re(A_c).  Returns A with shape (Nz, Ny, Nx) (and the largest
    |Im| seen if requested).  The transform primitive is numpy's FFT; with
    threads > 1 it is scipy's FFT with that many workers over independent
    lines (a timing configuration: its rounding may differ in the last bits)."""
    dx, dy, dz, inv = filter_factors(dims, bbox)
    if threads > 1:
        import scipy.fft as sfft
        fftn = lambda x: sfft.fftn(x, workers=threads)  # noqa: E731
        ifftn = lambda x: sfft.ifftn(x, workers=threads)  # noqa: E731
    else:
        fftn, ifftn = np.fft.fftn, np.fft.ifftn
    A = np.zeros(V.shape[1:])
    imag = 0.0
    for c, dfac in enumerate((dx, dy, dz)):
        spec = fftn(V[c])
        a = ifftn(1j * dfac * spec * inv)
        imag = max(imag, float(np.max(np.abs(a.imag))))
        A += a.real
    return (A, imag) if return_imag else A


def level(A, points, dims, bbox):
    """Iso-level L: mean of trilinear A at accepted points.  Returns (L, n)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    p = _f32c(points).reshape(-1, 3)
    used = ctypes.c_int64(0)
    L = lib.oracle_level(_ptr(A), _ptr(np.asarray(dims, np.int32)),
                         _ptr(np.asarray(bbox, np.float32)), _ptr(p), p.shape[0],
                         ctypes.byref(used))
    return float(L), int(used.value)


_TABLE = None


def mc_table():
    """(tri_count uint8[256], tri_edges int8[256, 15]) from ``mc_rule``."""
    global _TABLE
    if _TABLE is None:
        _TABLE = mc_rule.build_table()
    return _TABLE


def extract(A, L, dims, bbox, with_cases: bool = True, threads: int = 1, with_normals: bool = False):
    """Marching cubes at level L.  Returns (verts (V,3) f64, tris (T,3) i32,
    cases uint8 (Nz-1, Ny-1, Nx-1) or None), plus the unit vertex normals
    -grad A (V,3) when with_normals (central differences at the edge's grid
    points, one-sided on the outer layer, interpolated with the vertex's t).
    threads > 1 spreads the z planes over OpenMP threads (same output)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    Nx, Ny, Nz = (int(x) for x in dims)
    count, edges = mc_table()
    cases = np.empty((Nz - 1, Ny - 1, Nx - 1), np.uint8) if with_cases else None
    nv, nt = ctypes.c_int64(0), ctypes.c_int64(0)
    args = (_ptr(A), _ptr(np.asarray(dims, np.int32)), _ptr(np.asarray(bbox, np.float32)),
            float(L), _ptr(count), _ptr(edges))
    # first pass sizes the output, second pass fills it
    lib.oracle_marching_cubes(*args, None, 0, None, 0, _ptr(cases),
                              ctypes.byref(nv), ctypes.byref(nt), int(threads), None)
    verts = np.empty((max(nv.value, 1), 3))
    tris = np.empty((max(nt.value, 1), 3), np.int32)
    nrm = np.empty((max(nv.value, 1), 3)) if with_normals else None
    rc = lib.oracle_marching_cubes(*args, _ptr(verts), nv.value, _ptr(tris), nt.value,
                                   None, ctypes.byref(nv), ctypes.byref(nt), int(threads), _ptr(nrm))
    assert rc == 0
    if with_normals:
        return verts[:nv.value], tris[:nt.value], cases, nrm[:nv.value]
    return verts[:nv.value], tris[:nt.value], cases


def open_surface(A, L) -> bool:
    """True if any voxel on the grid's outer layer is inside (A > L): the
    bbox was not extended enough for a closed surface (Sec. III-B)."""
    A = np.asarray(A)
    shell = np.ones(A.shape, bool)
    shell[1:-1, 1:-1, 1:-1] = False
    return bool(np.any(A[shell] > L))


def reconstruct(points, normals, weights, dims, bbox, with_cases=False, threads: int = 1,
                splat_variant: str = "gaussian", with_normals: bool = False):
    """The whole path: splat, spectral integration, level, marching cubes.
    threads > 1 runs the splat, the transforms and marching cubes on that
    many host threads (see each step).  splat_variant "nearest" takes the
    non-weighted splat; with_normals adds the vertex normals."""
    if splat_variant == "nearest":
        V, _, rej = splat_nearest(points, normals, dims, bbox)
    else:
        V, _, _, rej = splat(points, normals, weights, dims, bbox, threads=threads)
    A = indicator(V, dims, bbox, threads=threads)
    L, used = level(A, points, dims, bbox)
    if used == 0:
        L = 0.0
    ex = extract(A, L, dims, bbox, with_cases=with_cases, threads=threads, with_normals=with_normals)
    verts, tris, cases = ex[:3]
    out = dict(V=V, A=A, level=L, n_used=used, n_rejected=rej, verts=verts,
               tris=tris, cases=cases, open_surface=open_surface(A, L))
    if with_normals:
        out["normals"] = ex[3]
    return out
