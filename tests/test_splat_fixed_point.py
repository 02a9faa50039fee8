"""The splat's fixed-point accumulation, emulated on the CPU (eqs. (1)-(2)).

The GPU splat sums every term g W N_c (and g W) as an integer count of a
power-of-two unit, so that the sums are exact and independent of the order
of the additions.  These tests model that rounding in numpy (the Gaussian
factors in float64, each term rounded to the unit, int64 sums, V = r S / D)
and compare the result with the FP64 oracle, to show where a choice of unit
holds the parity bar and where it fails:

* ``frame30`` - the earlier design: one unit per frame, 2^(e - 30) with 2^e
  bounding the frame's largest W |N_c| (or W), terms rounded half up.  A
  voxel reached only by the far footprint corners of a low-weight point gets
  terms of a few units, or zero, once a point 10^4 times heavier sits
  anywhere in the frame.
* ``tile`` - the current design: the unit is 2^(e - E_t), with 2^e
  bounding the largest W |N_c| (or W) divided by 1 - 2^-10 (headroom for the
  rounding of the kernel's Gaussian factors), and
  E_t = min(48, 62 - ceil(log2 N_t)) for a tile whose bins hold N_t points
  (so that N_t terms of at most 2^E_t units cannot overflow an int64 sum,
  and a run of 8 terms stays below 2^51, where the f64 run sums of the
  kernel are exact integers), each term rounded to the nearest unit on its
  own.  Its error bound relative to r N_max is
  2^(1 - E_t) R e^(32/3) plus the float32 evaluation error of the terms,
  where R is the ratio of the frame's largest weight to the smallest weight
  reaching the voxel (the far footprint corner lies under 2 voxels per axis
  from the point: d^2 < 4 |h|^2 = (32/3) sigma2^2).

The emulation shares nothing with the HIP library; it restates the unit
rule so that the rule can be checked against the oracle without a GPU.
"""
import math

import numpy as np
import pytest

import oracle
import synth

LOG2E = 1.4426950408889634


def _tile_shape(nx):
    """The kernel's default splat tile: 2 x 2 rows up to N_x = 128, 2 x 4
    above, within 2048 voxels per channel plane."""
    r = 4 if nx <= 128 else 8
    while r > 4 and r * nx > 2048:
        r //= 2
    tz = 4 if r >= 8 else 2
    return r // tz, tz


def _origin_f32(x, bmin, bmax, n):
    """Footprint origin floor((x - bmin)/h - 1/2) with every operation in
    float32 (the shared reading of the footprint rule), and the offset of the
    point from that origin's centre in voxels, in float64."""
    x = x.astype(np.float32)
    h = np.float32(np.float32(bmax) - np.float32(bmin)) / np.float32(n)
    v = (x - np.float32(bmin)) / h - np.float32(0.5)
    fl = np.floor(v)
    h64 = (float(bmax) - float(bmin)) / n
    off = (x.astype(np.float64) - float(bmin)) / h64 - 0.5 - fl
    return fl.astype(np.int64), off


def emulate_splat(f, scheme):
    """V (3, Nz, Ny, Nx) as the fixed-point splat with unit rule ``scheme``
    computes it, up to the float32 evaluation of the Gaussian factors."""
    Nx, Ny, Nz = f.dims
    b = np.asarray(f.bbox, np.float32)
    p, nrm = f.points, f.normals.astype(np.float64)
    w = np.ones(len(p)) if f.weights is None else f.weights.astype(np.float64)
    acc = np.all((p >= b[:3]) & (p <= b[3:]), axis=1)
    p, nrm, w = p[acc], nrm[acc], w[acc]
    n = np.asarray(f.dims)
    i0 = np.empty((len(p), 3), np.int64)
    fr = np.empty((len(p), 3))
    for a in range(3):
        i0[:, a], fr[:, a] = _origin_f32(p[:, a], b[a], b[a + 3], n[a])
        i0[:, a] = np.clip(i0[:, a], -1, n[a] - 1)
    h = (b[3:].astype(np.float64) - b[:3]) / n
    s1sq = 0.25 * np.sum(h * h)
    e1 = -h * h / s1sq * LOG2E
    e2 = -h * h / (1.5 * s1sq) * LOG2E
    wn = w[:, None] * nrm
    def unit_exp(mx):
        fr, e = math.frexp(mx)
        return e + 1 if scheme == "tile" and fr >= 1.0 - 2.0 ** -10 else e

    eS = unit_exp(float(np.max(np.abs(wn)))) if len(p) else 0
    eD = unit_exp(float(np.max(w))) if len(p) else 0

    # per-voxel unit exponent E (frame30: 30 everywhere)
    E = np.full((Nz, Ny, Nx), 30, np.int64)
    if scheme == "tile":
        ty, tz = _tile_shape(Nx)
        bins = np.zeros((Nz + 1, Ny + 1), np.int64)
        np.add.at(bins, (i0[:, 2] + 1, i0[:, 1] + 1), 1)
        for z0 in range(0, Nz, tz):
            for y0 in range(0, Ny, ty):
                lo_z, hi_z = max(z0 - 2, -1), min(z0 + tz, Nz - 1)
                lo_y, hi_y = max(y0 - 2, -1), min(y0 + ty, Ny - 1)
                nt = int(bins[lo_z + 1:hi_z + 2, lo_y + 1:hi_y + 2].sum())
                et = min(48, 62 - max(nt - 1, 0).bit_length())
                E[z0:z0 + tz, y0:y0 + ty, :] = et
    elif scheme != "frame30":
        raise ValueError(scheme)

    S = np.zeros((4, Nz, Ny, Nx), np.int64)   # S_x, S_y, S_z, D in units
    mag = np.zeros((4, Nz, Ny, Nx))           # sum of |terms| in units (headroom)
    for oz in range(-1, 3):
        for oy in range(-1, 3):
            for ox in range(-1, 3):
                q = i0 + np.array([ox, oy, oz])
                ok = np.all((q >= 0) & (q < n), axis=1)
                d = fr[ok] - np.array([ox, oy, oz])
                g1 = np.exp2(d * d @ e1)
                g2 = np.exp2(d * d @ e2)
                qx, qy, qz = q[ok, 0], q[ok, 1], q[ok, 2]
                et = E[qz, qy, qx]
                for c in range(4):
                    term = g2 * w[ok] if c == 3 else g1 * wn[ok, c]
                    e = eD if c == 3 else eS
                    x = term * np.exp2((et - e).astype(np.float64))
                    t = np.floor(x + 0.5) if scheme == "frame30" else np.rint(x)
                    np.add.at(S[c], (qz, qy, qx), t.astype(np.int64))
                    np.add.at(mag[c], (qz, qy, qx), np.abs(t))
    V = np.zeros((3, Nz, Ny, Nx))
    Df = S[3].astype(np.float64)
    nz = Df > 0
    for c in range(3):
        # units 2^(eS - E) and 2^(eD - E): the tile exponent cancels in S / D
        V[c][nz] = math.sqrt(1.5) * math.ldexp(1.0, eS - eD) * S[c].astype(np.float64)[nz] / Df[nz]
    big = float(mag.max()) if mag.size else 0.0
    return V, big


def _rel_err(f, scheme):
    V, big = emulate_splat(f, scheme)
    Vo, _, _, _ = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
    return float(np.abs(V - Vo).max() / np.abs(Vo).max()), big


def _bound(weight_ratio, E=48, eps=2.0 ** -21):
    """Error bound of the tile rule relative to r N_max (module docstring)."""
    return 2.0 ** (1 - E) * weight_ratio * math.exp(32.0 / 3.0) + 2 * eps


def test_frame_unit_fails_at_a_wide_weight_range():
    """The input class that motivated the tile unit: the frame-global 2^-30
    unit puts isolated W = 0.01 points next to W = 100 points far outside
    the 1e-4 parity bar."""
    f = synth.isolated_weights_frame((0.01, 100.0), grid=32, seed=1)
    err, _ = _rel_err(f, "frame30")
    assert err > 1e-3
    err_tile, _ = _rel_err(f, "tile")
    assert err_tile <= _bound(1e4, eps=0.0) < 1e-5


@pytest.mark.parametrize("weights", [(1.0, 1.0), (0.05, 2.0), (0.01, 100.0), (1e-4, 100.0)])
def test_tile_unit_within_its_bound(weights):
    f = synth.isolated_weights_frame(weights, grid=32, seed=2, pairs=3)
    ratio = max(weights) / min(weights)
    err, big = _rel_err(f, "tile")
    # the emulation computes the Gaussians in float64: only the unit's term
    assert err <= _bound(ratio, eps=0.0)
    assert big < 2 ** 63


def test_tile_unit_on_overlapping_footprints_with_spread_weights():
    """Dense random points whose weights span 5 decades: every voxel mixes
    terms of very different size."""
    base = synth.sphere_frame(seed=4, m=3000, grid=16, radius=0.6)
    f = synth.spread_weights(base, decades=5.0, seed=4)
    ratio = float(f.weights.max() / f.weights.min())
    assert ratio > 5e4
    err, big = _rel_err(f, "tile")
    assert err <= _bound(ratio, eps=0.0)
    assert err < 1e-5
    assert big < 2 ** 63


def test_tile_exponent_keeps_int64_headroom_for_dense_bins():
    """Thousands of points in one bin lower the tile's exponent so that
    their sum still fits an int64 (and the result still meets the bar)."""
    rng = np.random.default_rng(5)
    m = 6000
    p = np.tile(np.array([[0.031, -0.017, 0.012]]), (m, 1)) + rng.normal(0, 1e-3, (m, 3))
    n = rng.standard_normal((m, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    f = synth.Frame(p.astype(np.float32), n.astype(np.float32),
                    rng.uniform(0.5, 2.0, m).astype(np.float32), (16, 16, 16),
                    (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0))
    err, big = _rel_err(f, "tile")
    assert big < 2 ** 63
    assert err < 1e-9
