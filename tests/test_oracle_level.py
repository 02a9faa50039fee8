"""Pins for the oracle's iso-level (Sec. III-B: L is the mean of A at the input
sample locations).  Trilinear interpolation reproduces affine functions of the
voxel-centre coordinate exactly, so affine fields give a closed form."""
import numpy as np
import pytest

import oracle


def _u_of(points, dims, bbox):
    b = np.asarray(bbox, np.float32).astype(np.float64)
    h = (b[3:] - b[:3]) / np.asarray(dims)
    return (points.astype(np.float64) - b[:3]) / h - 0.5


def test_constant_field():
    dims, bbox = (8, 10, 12), (-1, -1, -1, 1, 1, 1)
    rng = np.random.default_rng(0)
    p = rng.uniform(-1, 1, (500, 3)).astype(np.float32)
    L, n = oracle.level(np.full(dims[::-1], 2.75), p, dims, bbox)
    assert n == 500 and L == pytest.approx(2.75, rel=1e-15)


@pytest.mark.parametrize("dims,bbox", [((8, 10, 12), (-1, -1, -1, 1, 1, 1)),
                                       ((16, 6, 10), (0.2, -0.5, 1.0, 1.0, 0.1, 2.0))])
def test_affine_field_closed_form_with_border_clamp(dims, bbox):
    """A(q) = a.q + c  ->  L = mean(a.clamp(u, 0, N-1) + c) over accepted points."""
    rng = np.random.default_rng(1)
    b = np.asarray(bbox, np.float64)
    p = rng.uniform(b[:3], b[3:], (2000, 3)).astype(np.float32)
    a = np.array([0.7, -1.3, 0.4])
    c = 0.25
    qz, qy, qx = np.meshgrid(*(np.arange(n) for n in dims[::-1]), indexing="ij")
    A = a[0] * qx + a[1] * qy + a[2] * qz + c
    u = np.clip(_u_of(p, dims, bbox), 0, np.asarray(dims) - 1)
    expect = np.mean(u @ a + c)
    L, n = oracle.level(A, p, dims, bbox)
    assert n == 2000
    assert L == pytest.approx(expect, rel=1e-12, abs=1e-12)


def test_points_outside_bbox_are_ignored():
    dims, bbox = (8, 8, 8), (-1, -1, -1, 1, 1, 1)
    rng = np.random.default_rng(2)
    A = rng.standard_normal(dims)
    p = rng.uniform(-0.9, 0.9, (100, 3)).astype(np.float32)
    L0, n0 = oracle.level(A, p, dims, bbox)
    far = np.array([[2, 0, 0], [0, -3, 0], [0, 0, 1.0001]], np.float32)
    L1, n1 = oracle.level(A, np.concatenate([p[:50], far, p[50:]]), dims, bbox)
    assert n0 == n1 == 100 and L1 == L0


def test_no_points_gives_zero():
    L, n = oracle.level(np.ones((8, 8, 8)), np.zeros((0, 3), np.float32), (8, 8, 8),
                        (-1, -1, -1, 1, 1, 1))
    assert (L, n) == (0.0, 0)


def test_sample_at_voxel_centre_is_the_voxel_value():
    dims, bbox = (8, 8, 8), (0, 0, 0, 1, 1, 1)
    rng = np.random.default_rng(3)
    A = rng.standard_normal(dims)
    q = (3, 5, 2)  # (qx, qy, qz)
    p = np.array([[(q[0] + 0.5) / 8, (q[1] + 0.5) / 8, (q[2] + 0.5) / 8]], np.float32)
    L, _ = oracle.level(A, p, dims, bbox)
    assert L == pytest.approx(A[q[2], q[1], q[0]], rel=1e-12)
