"""End-to-end pins for the oracle: the whole Sec. III-B path on inputs whose
true surface is known analytically."""
import collections

import numpy as np
import pytest

import oracle
import synth


def _closed_manifold(tris):
    und = collections.Counter()
    dire = collections.Counter()
    for t in tris:
        for i in range(3):
            a, b = int(t[i]), int(t[(i + 1) % 3])
            und[(min(a, b), max(a, b))] += 1
            dire[(a, b)] += 1
    return all(v == 2 for v in und.values()) and all(v == 1 for v in dire.values()), len(und)


def test_sphere_config_recovers_radius_within_one_voxel():
    f = synth.sphere_frame(seed=0, m=50_000, grid=64)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    h = 2.0 / 64
    v, t = r["verts"], r["tris"]
    assert r["n_rejected"] == 0 and r["n_used"] == 50_000
    assert np.max(np.abs(np.linalg.norm(v, axis=1) - 0.8)) <= h
    ok, ne = _closed_manifold(t)
    assert ok
    assert len(v) - ne + len(t) == 2
    vol = np.einsum("ij,ij->i", v[t[:, 0]], np.cross(v[t[:, 1]], v[t[:, 2]])).sum() / 6
    assert vol > 0                       # outward winding: inside is high
    assert abs(vol / (4 / 3 * np.pi * 0.8 ** 3) - 1) < 0.01
    assert not r["open_surface"]
    # the indicator is zero-mean and larger inside than outside
    A = r["A"]
    assert abs(A.mean()) < 1e-12
    assert A[32, 32, 32] > r["level"] > A[0, 0, 0]


def test_inverted_normals_flip_the_indicator():
    """Inward normals negate V and hence A: the mesh is the same surface with
    the level negated (A -> -A, L -> -L)."""
    f = synth.sphere_frame(seed=2, m=8000, grid=32)
    r1 = oracle.reconstruct(f.points, f.normals, None, f.dims, f.bbox)
    r2 = oracle.reconstruct(f.points, -f.normals, None, f.dims, f.bbox)
    assert np.allclose(r2["A"], -r1["A"], atol=1e-14)
    assert r2["level"] == pytest.approx(-r1["level"], abs=1e-15)


def test_empty_input_gives_empty_mesh_and_zero_level():
    z = np.zeros((0, 3), np.float32)
    r = oracle.reconstruct(z, z, None, (16, 16, 16), (-1, -1, -1, 1, 1, 1))
    assert r["level"] == 0.0 and len(r["verts"]) == 0 and len(r["tris"]) == 0


def test_human_proxy_vertices_near_analytic_surface():
    f = synth.human_proxy_frame(seed=7, views=4, m=120_000, grid=96, ss=2)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    h = 2.0 / 96
    d = synth.proxy_distance(f.info["prims"], r["verts"])
    assert np.median(d) <= h
    ok, _ = _closed_manifold(r["tris"])
    assert ok
    assert not r["open_surface"]


def test_open_surface_flag_definition():
    """oracle.open_surface against its definition (Sec. III-B: the bbox must
    be extended enough that the surface closes inside it): True iff some
    voxel of the grid's outer layer has A > L, checked on each face, an
    edge, a corner, an interior voxel and a tie."""
    shape = (5, 6, 7)  # (Nz, Ny, Nx)
    L = 0.5
    A = np.zeros(shape)
    assert oracle.open_surface(A, L) is False
    interior = A.copy()
    interior[2, 3, 3] = 1.0
    assert oracle.open_surface(interior, L) is False
    on_border = [(0, 2, 3), (4, 2, 3), (2, 0, 3), (2, 5, 3), (2, 2, 0), (2, 2, 6),
                 (0, 0, 3), (4, 5, 6)]
    for idx in on_border:
        B = A.copy()
        B[idx] = 1.0
        assert oracle.open_surface(B, L) is True, idx
    tie = A.copy()
    tie[0, 0, 0] = L  # inside means A > L strictly
    assert oracle.open_surface(tie, L) is False
    # a ball field: closed when it fits the box, open when the box cuts it
    z, y, x = np.meshgrid(*[np.linspace(-1, 1, 9)] * 3, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    assert oracle.open_surface(0.6 - r, 0.0) is False
    assert oracle.open_surface(1.1 - r, 0.0) is True


def test_threaded_oracle_matches_the_single_threaded_one():
    """The all-cores configuration of the oracle (the benchmark's CPU
    baseline) splits voxel planes and marching-cubes planes over threads
    without changing any sum or numbering: splat and mesh are bit-identical;
    the transforms (scipy's FFT with workers) agree to rounding."""
    f = synth.sphere_frame(seed=6, m=8_000, grid=24)
    V1, S1, D1, r1 = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
    V4, S4, D4, r4 = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox, threads=4)
    assert r1 == r4 and np.array_equal(S1, S4) and np.array_equal(D1, D4) and np.array_equal(V1, V4)
    A1 = oracle.indicator(V1, f.dims, f.bbox)
    A4 = oracle.indicator(V1, f.dims, f.bbox, threads=4)
    assert np.abs(A1 - A4).max() <= 1e-12 * (A1.max() - A1.min())
    L, _ = oracle.level(A1, f.points, f.dims, f.bbox)
    v1, t1, c1 = oracle.extract(A1, L, f.dims, f.bbox)
    v4, t4, c4 = oracle.extract(A1, L, f.dims, f.bbox, threads=4)
    assert np.array_equal(v1, v4) and np.array_equal(t1, t4) and np.array_equal(c1, c4)
    assert len(t1) > 1000
