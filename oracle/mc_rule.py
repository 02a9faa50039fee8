"""Marching-cubes triangle table generated from a stated rule (oracle side).

TEST INFRASTRUCTURE ONLY.  The paper extracts the surface A(q) = L with
marching cubes (end of Sec. III-B) and claims a watertight, manifold mesh
(Sec. I).  It prints no table, so the table is generated here from a rule
that guarantees both properties; nothing is copied from a published table.

Cube conventions
  corner k sits at offset (k & 1, (k >> 1) & 1, (k >> 2) & 1); inside <=> A > L
  edge id = 4 * axis + b_lo + 2 * b_hi, where b_lo and b_hi are the offset
  bits of the two other axes taken in x < y < z order.

Rule
  R1 faces: a face with two crossing edges gets one segment between them.  A
     face with four crossings (inside corners on a diagonal) gets two
     segments, each cutting off one inside corner, so inside corners on that
     face stay separated.  Both cells sharing a face see the same corner
     values, hence the same segments: the mesh is crack free.
  R2 loops: every crossing edge lies on exactly two faces, so the segments
     chain into closed loops.
  R3 orientation: each segment is directed so that, seen from outside the
     cube, the inside corners lie on its right.  The loop's right-hand normal
     then points from inside (A > L) to outside.
  R4 triangulation: a fan, anchored at the first loop vertex - walking the
     loop in its direction from its smallest edge id - whose fan adds no
     diagonal joining two edges of one cube face.  (A diagonal inside a face
     could be emitted by both cells sharing that face and give an edge of
     four triangles; such an anchor exists for every loop, which
     ``build_table`` asserts.)
  R5 loops are emitted in order of their smallest edge id.
"""
from __future__ import annotations

import numpy as np

MAX_TRIS = 5          # the rule never needs more than five triangles per case
ROW = 3 * MAX_TRIS    # int8 entries per case in the flat table


def corner_offset(k: int) -> tuple:
    return (k & 1, (k >> 1) & 1, (k >> 2) & 1)


def corner_index(off) -> int:
    return off[0] + 2 * off[1] + 4 * off[2]


def edge_corners(e: int) -> tuple:
    """(low corner, high corner) of cube edge e."""
    axis, r = divmod(e, 4)
    others = [b for b in range(3) if b != axis]
    lo = [0, 0, 0]
    lo[others[0]] = r & 1
    lo[others[1]] = (r >> 1) & 1
    hi = list(lo)
    hi[axis] = 1
    return corner_index(lo), corner_index(hi)


def faces():
    """The six faces as (axis, side)."""
    return [(a, s) for a in range(3) for s in (0, 1)]


def face_edges(axis: int, side: int) -> list:
    return [e for e in range(12)
            if e // 4 != axis and corner_offset(edge_corners(e)[0])[axis] == side]


def face_corners(axis: int, side: int) -> list:
    return [k for k in range(8) if corner_offset(k)[axis] == side]


def edges_share_face(e1: int, e2: int) -> bool:
    return any(e1 in face_edges(a, s) and e2 in face_edges(a, s) for a, s in faces())


def _midpoint(e: int) -> np.ndarray:
    c0, c1 = edge_corners(e)
    return (np.array(corner_offset(c0), float) + np.array(corner_offset(c1), float)) / 2


def _directed(axis, side, e1, e2, inside_side_corner):
    """Direct the segment e1-e2 so the given inside corner is on its right
    when the face is seen from outside the cube."""
    n_out = np.zeros(3)
    n_out[axis] = 1.0 if side == 1 else -1.0
    p, q = _midpoint(e1), _midpoint(e2)
    left = np.cross(n_out, q - p)
    s = float(np.dot(left, np.array(corner_offset(inside_side_corner), float) - (p + q) / 2))
    assert s != 0.0
    return (e1, e2) if s < 0 else (e2, e1)


def case_loops(case: int) -> list:
    """Closed, oriented loops of crossing-edge ids for one case (R1-R3, R5)."""
    inside = [(case >> k) & 1 for k in range(8)]
    crossing = lambda e: inside[edge_corners(e)[0]] != inside[edge_corners(e)[1]]
    nxt = {}
    for axis, side in faces():
        fe = [e for e in face_edges(axis, side) if crossing(e)]
        if not fe:
            continue
        fc = face_corners(axis, side)
        segs = []
        if len(fe) == 2:
            ref = next(k for k in fc if inside[k])
            segs.append(_directed(axis, side, fe[0], fe[1], ref))
        else:
            assert len(fe) == 4
            for k in fc:
                if inside[k]:
                    around = [e for e in fe if k in edge_corners(e)]
                    assert len(around) == 2
                    segs.append(_directed(axis, side, around[0], around[1], k))
        for a, b in segs:
            assert a not in nxt, "two segments leave one edge"
            nxt[a] = b
    assert sorted(nxt) == sorted(nxt.values()), "segments do not close"
    loops, seen = [], set()
    for start in sorted(nxt):
        if start in seen:
            continue
        loop, e = [], start
        while e not in seen:
            seen.add(e)
            loop.append(e)
            e = nxt[e]
        assert e == start
        loops.append(loop)
    return loops


def triangulate(loop: list) -> list:
    """R4: fan from the first clean anchor."""
    k = len(loop)
    for s in range(k):
        anchor = loop[s]
        if all(not edges_share_face(anchor, loop[(s + i) % k]) for i in range(2, k - 1)):
            return [(anchor, loop[(s + i) % k], loop[(s + i + 1) % k]) for i in range(1, k - 1)]
    raise AssertionError(f"no clean fan anchor for loop {loop}")


def case_triangles(case: int) -> list:
    out = []
    for loop in case_loops(case):
        out.extend(triangulate(loop))
    return out


def build_table():
    """Return (tri_count uint8[256], tri_edges int8[256, 15]) with -1 padding."""
    count = np.zeros(256, np.uint8)
    edges = np.full((256, ROW), -1, np.int8)
    for case in range(256):
        tris = case_triangles(case)
        assert len(tris) <= MAX_TRIS
        count[case] = len(tris)
        for t, tri in enumerate(tris):
            edges[case, 3 * t:3 * t + 3] = tri
    return count, edges
