"""Pins for the oracle's marching cubes (end of Sec. III-B) and its
rule-generated table; the paper claims a watertight, manifold mesh (Sec. I).

Table-level checks are exhaustive over the 256 cases and all face-adjacent
pairs.  Mesh-level checks use signed-distance fields with known topology
(sphere chi = 2, torus chi = 0, two spheres chi = 4), convergence of volume and
area, brute-force counts, and random fields.
"""
import collections
import itertools

import numpy as np
import pytest

import oracle
from oracle import mc_rule

CORNERS = [(k & 1, (k >> 1) & 1, (k >> 2) & 1) for k in range(8)]


def _edge_geom(e):
    """Cube edge e as a pair of corner offsets (independent decoding of the
    documented numbering: id = 4 axis + b_lo + 2 b_hi)."""
    axis = e // 4
    r = e % 4
    o = [a for a in range(3) if a != axis]
    lo = [0, 0, 0]
    lo[o[0]] = r % 2
    lo[o[1]] = r // 2
    hi = list(lo)
    hi[axis] = 1
    return tuple(lo), tuple(hi)


def _table():
    count, edges = oracle.mc_table()
    return [[tuple(int(x) for x in edges[c, 3 * t:3 * t + 3]) for t in range(count[c])]
            for c in range(256)]


TABLE = _table()


def test_trivial_and_single_corner_cases():
    assert TABLE[0] == [] and TABLE[255] == []
    for k in range(8):
        assert len(TABLE[1 << k]) == 1
        assert len(TABLE[255 ^ (1 << k)]) == 1
    assert max(len(t) for t in TABLE) <= mc_rule.MAX_TRIS


def test_every_table_edge_is_a_crossing_edge_and_every_crossing_edge_used():
    for case in range(256):
        inside = [(case >> k) & 1 for k in range(8)]
        crossing = set()
        for e in range(12):
            lo, hi = _edge_geom(e)
            if inside[CORNERS.index(lo)] != inside[CORNERS.index(hi)]:
                crossing.add(e)
        used = {e for tri in TABLE[case] for e in tri}
        assert used == crossing, case


def _face_boundary(case, axis, side):
    """Directed boundary edges of the case's triangle set lying in one face,
    as pairs of edge-midpoint coordinates."""
    cnt = collections.Counter()
    for tri in TABLE[case]:
        for i in range(3):
            cnt[(tri[i], tri[(i + 1) % 3])] += 1
    segs = set()
    for (a, b), k in cnt.items():
        if (b, a) in cnt:
            continue  # interior edge of the case's patch
        ma = tuple(np.add(*_edge_geom(a)) / 2)
        mb = tuple(np.add(*_edge_geom(b)) / 2)
        if ma[axis] == side and mb[axis] == side:
            segs.add((ma, mb))
    return segs


def test_patch_boundaries_lie_on_faces_and_are_closed_loops():
    for case in range(256):
        cnt = collections.Counter()
        for tri in TABLE[case]:
            for i in range(3):
                cnt[(tri[i], tri[(i + 1) % 3])] += 1
        assert all(v == 1 for v in cnt.values()), case      # consistent orientation
        boundary = [(a, b) for (a, b) in cnt if (b, a) not in cnt]
        for a, b in boundary:
            ma = np.add(*_edge_geom(a)) / 2
            mb = np.add(*_edge_geom(b)) / 2
            on_common_face = any(ma[x] == mb[x] and ma[x] in (0, 1) for x in range(3))
            assert on_common_face, (case, a, b)
        outs = collections.Counter(a for a, _ in boundary)
        ins = collections.Counter(b for _, b in boundary)
        assert outs == ins


def test_face_consistency_for_all_face_adjacent_case_pairs():
    """Brute force: for every pair of cells sharing a face with equal corner
    values on it, the two patches meet along the same segments with opposite
    directions (crack free and consistently oriented)."""
    for axis in range(3):
        for case_lo in range(256):
            # the neighbour above shares our side-1 face as its side-0 face
            mine = _face_boundary(case_lo, axis, 1)
            for other_bits in range(16):
                case_hi = 0
                j = 0
                for k in range(8):
                    if CORNERS[k][axis] == 0:
                        src = k + (1 << axis)   # corner on the shared face
                        if (case_lo >> src) & 1:
                            case_hi |= 1 << k
                    else:
                        if (other_bits >> j) & 1:
                            case_hi |= 1 << k
                        j += 1
                theirs = _face_boundary(case_hi, axis, 0)
                shift = lambda p: tuple(p[x] + (1 if x == axis else 0) for x in range(3))
                theirs_shifted = {(shift(b), shift(a)) for a, b in theirs}
                assert mine == theirs_shifted, (axis, case_lo, case_hi)


def _grid_field(n, fn, lo=-1.0, hi=1.0):
    dims = (n, n, n)
    bbox = (lo, lo, lo, hi, hi, hi)
    h = (hi - lo) / n
    c = lo + (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return fn(X, Y, Z), dims, bbox, h


def _topology(verts, tris):
    und = collections.Counter()
    dire = collections.Counter()
    for t in tris:
        for i in range(3):
            a, b = int(t[i]), int(t[(i + 1) % 3])
            und[(min(a, b), max(a, b))] += 1
            dire[(a, b)] += 1
    # vertex links: each vertex's one-ring is a single cycle
    link = collections.defaultdict(dict)
    for t in tris:
        for i in range(3):
            link[int(t[i])][int(t[(i + 1) % 3])] = int(t[(i + 2) % 3])
    bad_link = 0
    for v, nxt in link.items():
        s = next(iter(nxt))
        c, k = nxt[s], 1
        while c != s and c in nxt and k <= len(nxt):
            c = nxt[c]
            k += 1
        bad_link += (k != len(nxt) or c != s)
    chi = len(verts) - len(und) + len(tris)
    return dict(bad_edges=sum(v != 2 for v in und.values()),
                bad_directed=sum(v != 1 for v in dire.values()),
                bad_links=bad_link, unused=len(verts) - len(link), chi=chi)


def _volume_area(v, t):
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()
    return vol, area


@pytest.mark.parametrize("n", [24, 40])
def test_sdf_sphere_closed_manifold_outward(n):
    R = 0.6
    A, dims, bbox, h = _grid_field(n, lambda X, Y, Z: R - np.sqrt(X * X + Y * Y + Z * Z))
    v, t, cases = oracle.extract(A, 0.0, dims, bbox)
    top = _topology(v, t)
    assert top == dict(bad_edges=0, bad_directed=0, bad_links=0, unused=0, chi=2)
    vol, area = _volume_area(v, t)
    assert vol > 0
    assert abs(vol - 4 / 3 * np.pi * R ** 3) / (4 / 3 * np.pi * R ** 3) < 2.0 * h * h / R ** 2
    assert abs(area - 4 * np.pi * R ** 2) / (4 * np.pi * R ** 2) < 0.02
    # vertices lie on the sphere up to the linear-interpolation error
    assert np.max(np.abs(np.linalg.norm(v, axis=1) - R)) < 0.25 * h


def test_sphere_volume_converges_second_order():
    R = 0.55
    errs = []
    for n in (16, 32):
        A, dims, bbox, h = _grid_field(n, lambda X, Y, Z: R - np.sqrt(X * X + Y * Y + Z * Z))
        v, t, _ = oracle.extract(A, 0.0, dims, bbox)
        errs.append(abs(_volume_area(v, t)[0] - 4 / 3 * np.pi * R ** 3))
    assert errs[1] < errs[0] / 2.5


def test_sdf_torus_and_two_spheres_euler_characteristic():
    Rt, rt = 0.5, 0.2
    A, dims, bbox, _ = _grid_field(36, lambda X, Y, Z: rt - np.sqrt((np.sqrt(X * X + Y * Y) - Rt) ** 2 + Z * Z))
    v, t, _ = oracle.extract(A, 0.0, dims, bbox)
    top = _topology(v, t)
    assert top["bad_edges"] == top["bad_directed"] == top["bad_links"] == 0 and top["chi"] == 0
    A, dims, bbox, _ = _grid_field(32, lambda X, Y, Z: np.maximum(
        0.3 - np.sqrt((X - 0.45) ** 2 + Y * Y + Z * Z), 0.3 - np.sqrt((X + 0.45) ** 2 + Y * Y + Z * Z)))
    v, t, _ = oracle.extract(A, 0.0, dims, bbox)
    top = _topology(v, t)
    assert top["bad_edges"] == top["bad_directed"] == top["bad_links"] == 0 and top["chi"] == 4


@pytest.mark.parametrize("seed", range(4))
def test_random_fields_closed_manifold_and_brute_force_counts(seed):
    rng = np.random.default_rng(seed)
    dims = (9, 7, 8)
    A = rng.standard_normal(dims[::-1])
    A[0], A[-1], A[:, 0], A[:, -1], A[:, :, 0], A[:, :, -1] = (-5,) * 6
    bbox = (0, 0, 0, 0.9, 0.7, 0.8)
    L = 0.1
    v, t, cases = oracle.extract(A, L, dims, bbox)
    top = _topology(v, t)
    assert top == dict(bad_edges=0, bad_directed=0, bad_links=0, unused=0, chi=top["chi"])
    inside = A > L
    n_edges = (np.count_nonzero(inside[:, :, 1:] != inside[:, :, :-1]) +
               np.count_nonzero(inside[:, 1:, :] != inside[:, :-1, :]) +
               np.count_nonzero(inside[1:, :, :] != inside[:-1, :, :]))
    assert len(v) == n_edges
    expect_cases = np.zeros(cases.shape, np.int64)
    for k, (ox, oy, oz) in enumerate(CORNERS):
        expect_cases |= inside[oz:oz + dims[2] - 1, oy:oy + dims[1] - 1, ox:ox + dims[0] - 1].astype(np.int64) << k
    assert np.array_equal(cases, expect_cases)
    count, _ = oracle.mc_table()
    assert len(t) == int(count[cases].astype(np.int64).sum())


def test_vertices_on_affine_level_plane():
    """For an affine field the interpolated vertices lie exactly on A = L."""
    n = 12
    a = np.array([0.8, -0.5, 0.3])
    A, dims, bbox, _ = _grid_field(n, lambda X, Y, Z: a[0] * X + a[1] * Y + a[2] * Z)
    L = 0.07
    v, t, _ = oracle.extract(A, L, dims, bbox)
    assert len(v) > 0
    assert np.max(np.abs(v @ a - L)) < 1e-12
    # triangle normals point toward decreasing A (outward from the inside A > L)
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    assert np.all(nrm @ a < 0)


def test_vertex_order_is_grid_edge_order():
    """Vertices come in (linear index of the lower grid point, axis) order."""
    rng = np.random.default_rng(9)
    dims = (6, 5, 7)
    A = rng.standard_normal(dims[::-1])
    v, t, _ = oracle.extract(A, 0.0, dims, (0, 0, 0, 6, 5, 7))
    h = 1.0
    q = np.floor(v / h - 0.5 + 1e-9).astype(int)
    frac = v / h - 0.5 - q
    axis = np.argmax(frac > 1e-9, axis=1)
    lin = q[:, 0] + dims[0] * (q[:, 1] + dims[1] * q[:, 2])
    key = lin * 3 + axis
    assert np.all(np.diff(key) > 0)


def test_ties_count_as_outside():
    """inside(q) <=> A(q) > L strictly: voxels exactly at the level are outside,
    so a crossing between A = L and A > L puts the vertex on the A = L point."""
    rng = np.random.default_rng(4)
    dims = (7, 6, 8)
    A = rng.integers(0, 3, dims[::-1]).astype(np.float64)
    A[0], A[-1], A[:, 0], A[:, -1], A[:, :, 0], A[:, :, -1] = (0.0,) * 6
    v, t, cases = oracle.extract(A, 1.0, dims, (0, 0, 0, 7, 6, 8))
    inside = A > 1.0
    expect = np.zeros(cases.shape, np.int64)
    for k, (ox, oy, oz) in enumerate(CORNERS):
        expect |= inside[oz:oz + dims[2] - 1, oy:oy + dims[1] - 1, ox:ox + dims[0] - 1].astype(np.int64) << k
    assert np.array_equal(cases, expect)
    n_edges = (np.count_nonzero(inside[:, :, 1:] != inside[:, :, :-1]) +
               np.count_nonzero(inside[:, 1:, :] != inside[:, :-1, :]) +
               np.count_nonzero(inside[1:, :, :] != inside[:-1, :, :]))
    assert len(v) == n_edges


def test_vertex_normals_of_an_affine_field_are_exact():
    """For A = c - <a, p>, central and one-sided differences are exact, so
    every vertex normal -grad A / |grad A| is a / |a| (the outward
    direction: A is larger inside)."""
    dims = (9, 7, 8)
    bbox = (0.0, 0.0, 0.0, 0.9, 1.4, 0.8)
    h = np.array([0.1, 0.2, 0.1])
    a = np.array([0.3, -0.5, 0.8])
    z, y, x = np.meshgrid(*[(np.arange(n) + 0.5) * hh for n, hh in zip(dims[::-1], h[::-1])],
                          indexing="ij")
    A = 0.4 - (a[0] * x + a[1] * y + a[2] * z)
    v, t, _, nrm = oracle.extract(A, 0.0, dims, bbox, with_normals=True)
    assert len(v) > 20
    np.testing.assert_allclose(nrm, np.tile(a / np.linalg.norm(a), (len(v), 1)), atol=1e-12)


def test_vertex_normals_of_a_sphere_are_radial_and_outward():
    """SDF ball A = R - |p|: normals are the radial direction up to O(h^2),
    unit length, and agree with the winding of the triangles around them."""
    n = 32
    dims = (n, n, n)
    bbox = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    c = (np.arange(n) + 0.5) * (2.0 / n) - 1.0
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    A = 0.7 - np.sqrt(x * x + y * y + z * z)
    v, t, _, nrm = oracle.extract(A, 0.0, dims, bbox, with_normals=True)
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=1), 1.0, atol=1e-12)
    radial = v / np.linalg.norm(v, axis=1, keepdims=True)
    assert np.max(np.arccos(np.clip(np.sum(nrm * radial, axis=1), -1, 1))) < 0.03
    fn = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    assert np.all(np.sum(fn * (nrm[t[:, 0]] + nrm[t[:, 1]] + nrm[t[:, 2]]), axis=1) > 0)
