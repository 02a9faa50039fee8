"""Pins for the oracle's splat (eqs. (1)-(2), Sec. III-B).

Each test checks the oracle against something other than itself: a
hand-derived closed form (tests/golden/single_point_splat.txt), an invariant
that the definition implies, or brute force over the footprint rule.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "single_point_splat.txt")


def _grid(n=16, e=1.0):
    return (n, n, n), (-e, -e, -e, e, e, e)


def _point_at_u(u, dims, bbox):
    """World position whose voxel-centre coordinate is u (per axis)."""
    b = np.asarray(bbox, np.float64)
    h = (b[3:] - b[:3]) / np.asarray(dims)
    return (b[:3] + (np.asarray(u, float) + 0.5) * h).astype(np.float32)


def test_single_point_matches_hand_derived_values():
    dims, bbox = _grid(16)
    k = 7
    x = _point_at_u([k + 0.25] * 3, dims, bbox)
    nrm = np.array([0.3, -0.5, 0.8], np.float32)
    V, S, D, rej = oracle.splat(x[None], nrm[None], np.array([2.5], np.float32), dims, bbox)
    assert rej == 0
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 10
    for dx, dy, dz, val in rows:
        qx, qy, qz = k + int(dx), k + int(dy), k + int(dz)
        for c in range(3):
            got = V[c, qz, qy, qx]
            assert got == pytest.approx(float(val) * float(nrm[c]), rel=1e-12, abs=1e-15)


def test_single_point_support_is_exactly_the_4cube_of_nearest_centres():
    """Brute force: per axis, the footprint is the 4 voxel centres nearest X."""
    dims, bbox = (12, 10, 14), (-0.6, -0.5, -0.7, 0.6, 0.5, 0.7)
    rng = np.random.default_rng(3)
    b = np.asarray(bbox, np.float64)
    h = (b[3:] - b[:3]) / np.asarray(dims)
    for _ in range(20):
        u = rng.uniform(2.0, np.asarray(dims) - 3.0)
        x = _point_at_u(u, dims, bbox)
        V, _, D, _ = oracle.splat(x[None], np.array([[1, 1, 1]], np.float32), None, dims, bbox)
        expect = np.zeros(D.shape, bool)
        near = []
        for a in range(3):
            centres = b[a] + (np.arange(dims[a]) + 0.5) * h[a]
            near.append(np.sort(np.argsort(np.abs(centres - float(x[a])), kind="stable")[:4]))
        expect[np.ix_(near[2], near[1], near[0])] = True
        assert np.array_equal(D > 0, expect)
        assert np.count_nonzero(V[0]) == 64


def test_single_point_independent_of_weight_and_density_normalised():
    dims, bbox = _grid(16)
    x = _point_at_u([6.4, 7.9, 8.1], dims, bbox)[None]
    n = np.array([[0.0, 0.6, -0.8]], np.float32)
    V1, *_ = oracle.splat(x, n, np.array([1.0], np.float32), dims, bbox)
    V2, *_ = oracle.splat(x, n, np.array([37.0], np.float32), dims, bbox)
    assert np.allclose(V1, V2, rtol=1e-13, atol=0)


def test_weighted_mean_of_coincident_points():
    """Two points at one location: V is the W-weighted mean of their normals
    times the single-point profile (the w = W/d normalisation of eq. (1))."""
    dims, bbox = _grid(16)
    x = _point_at_u([7.25] * 3, dims, bbox)
    n1 = np.array([1.0, 0.0, 0.0], np.float32)
    n2 = np.array([0.0, 1.0, 0.0], np.float32)
    w1, w2 = 1.0, 3.0
    V, *_ = oracle.splat(np.stack([x, x]), np.stack([n1, n2]),
                         np.array([w1, w2], np.float32), dims, bbox)
    centre = math.sqrt(1.5) * math.exp(-4 * 3 * 0.25 ** 2 / 9)
    assert V[0, 7, 7, 7] == pytest.approx(centre * w1 / (w1 + w2), rel=1e-12)
    assert V[1, 7, 7, 7] == pytest.approx(centre * w2 / (w1 + w2), rel=1e-12)
    assert V[2, 7, 7, 7] == 0.0


def test_global_weight_scale_invariance_and_linearity_in_normals():
    rng = np.random.default_rng(5)
    dims, bbox = (12, 16, 10), (-0.5, -0.8, -0.4, 0.5, 0.8, 0.4)
    m = 400
    x = rng.uniform([-0.45, -0.75, -0.35], [0.45, 0.75, 0.35], (m, 3)).astype(np.float32)
    na = rng.standard_normal((m, 3)).astype(np.float32)
    nb = rng.standard_normal((m, 3)).astype(np.float32)
    w = rng.uniform(0.1, 2.0, m).astype(np.float32)
    Va, *_ = oracle.splat(x, na, w, dims, bbox)
    Vs, *_ = oracle.splat(x, na, (w * 4.0).astype(np.float32), dims, bbox)
    assert np.allclose(Va, Vs, rtol=1e-12, atol=1e-14)
    Vb, *_ = oracle.splat(x, nb, w, dims, bbox)
    Vab, *_ = oracle.splat(x, (na + nb).astype(np.float32), w, dims, bbox)
    # na + nb is rounded to float32 on input; compare against the same rounding
    assert np.allclose(Vab, Va + Vb, rtol=1e-6, atol=1e-6)


def test_integer_voxel_translation_is_a_shift():
    rng = np.random.default_rng(6)
    dims, bbox = _grid(16)
    m = 200
    u = rng.uniform(3.0, 9.0, (m, 3))
    n = rng.standard_normal((m, 3)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, m).astype(np.float32)
    V0, *_ = oracle.splat(_point_at_u(u, dims, bbox), n, w, dims, bbox)
    V1, *_ = oracle.splat(_point_at_u(u + [3, 2, 1], dims, bbox), n, w, dims, bbox)
    shifted = np.roll(V0, shift=(1, 2, 3), axis=(1, 2, 3))
    assert np.allclose(V1, shifted, rtol=1e-5, atol=1e-6)


def test_rejects_points_outside_bbox_and_empty_density_gives_zero():
    dims, bbox = _grid(8)
    x = np.array([[0.0, 0.0, 0.0], [1.5, 0.0, 0.0], [0.0, -1.01, 0.0], [1.0, 1.0, 1.0]], np.float32)
    n = np.ones((4, 3), np.float32)
    V, S, D, rej = oracle.splat(x, n, None, dims, bbox)
    assert rej == 2   # the corner point (1,1,1) lies on the bbox and is accepted
    assert np.all(V[:, D == 0] == 0)
    V, S, D, rej = oracle.splat(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32),
                                None, dims, bbox)
    assert rej == 0 and not V.any() and not D.any()


def test_footprint_clipped_at_grid_border():
    """A point in the first half voxel: offsets below 0 are dropped, not wrapped."""
    dims, bbox = _grid(8)
    x = _point_at_u([-0.3, 3.25, 3.25], dims, bbox)
    V, _, D, _ = oracle.splat(x[None], np.array([[1, 0, 0]], np.float32), None, dims, bbox)
    # floor(-0.3) = -1 -> x offsets -2..1, only 0 and 1 exist
    assert np.array_equal(np.nonzero(D.any(axis=(0, 1)))[0], [0, 1])
    assert not D[:, :, -1].any()


def test_nearest_splat_single_point_and_mean():
    """Non-weighted splat (Sec. III-B, simplest version): one point puts its
    normal on the one voxel that contains it; coincident points give the
    mean of their normals; nothing else is touched; weights play no part."""
    dims = (8, 6, 10)
    bbox = (-1.0, -0.75, -1.25, 1.0, 0.75, 1.25)   # h = 0.25 on every axis
    p = np.array([[0.1, 0.3, -0.6]], np.float32)    # cell (4, 4, 2): well inside
    n = np.array([[0.2, -0.5, 0.7]], np.float32)
    V, cnt, rej = oracle.splat_nearest(p, n, dims, bbox)
    assert rej == 0 and cnt.sum() == 1 and cnt[2, 4, 4] == 1
    expect = np.zeros_like(V)
    expect[:, 2, 4, 4] = n[0]
    np.testing.assert_array_equal(V, expect)
    rng = np.random.default_rng(3)
    q = np.tile(p, (5, 1)) + rng.uniform(-0.05, 0.05, (5, 3)).astype(np.float32)
    nn = rng.standard_normal((5, 3)).astype(np.float32)
    V, cnt, _ = oracle.splat_nearest(q, nn, dims, bbox)
    assert cnt[2, 4, 4] == 5 and cnt.sum() == 5
    np.testing.assert_allclose(V[:, 2, 4, 4], nn.astype(np.float64).mean(0), rtol=0, atol=1e-15)


def test_nearest_splat_counts_faces_and_rejection():
    """Points on the bbox's upper faces fall in the last cell (clamped);
    points outside are rejected; every accepted point is counted once."""
    dims = (4, 4, 4)
    bbox = (0.0, 0.0, 0.0, 1.0, 1.0, 1.0)
    p = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0], [1.5, 0.5, 0.5], [0.5, 0.5, 0.5]], np.float32)
    n = np.ones((4, 3), np.float32)
    V, cnt, rej = oracle.splat_nearest(p, n, dims, bbox)
    assert rej == 1 and cnt.sum() == 3
    assert cnt[3, 3, 3] == 1 and cnt[0, 0, 0] == 1 and cnt[2, 2, 2] == 1
    rng = np.random.default_rng(4)
    q = rng.uniform(-0.2, 1.2, (2000, 3)).astype(np.float32)
    V, cnt, rej = oracle.splat_nearest(q, rng.standard_normal((2000, 3)).astype(np.float32), dims, bbox)
    inside = np.all((q >= 0) & (q <= 1), axis=1)
    assert rej == int((~inside).sum()) and cnt.sum() == int(inside.sum())
