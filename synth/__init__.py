"""Seeded synthetic input frames for the volumetric FT reconstruction.

This module produces oriented, confidence-weighted point sets of the kind the
method consumes (the raw points X_k(u), normals N_k(u) and weights W_k(u) of
Sec. III-A).  It holds none of the reconstruction's arithmetic: no splatting,
no transforms, no level or mesh extraction.  Both the oracle tests and the GPU
path draw their inputs from here, so the two sides always see identical data.

Two families:

* ``sphere_frame`` - points sampled uniformly on a sphere with exact outward
  normals, Gaussian position noise and unit weights (the small correctness
  workload).
* ``human_proxy_frame`` - a union of capsules and ellipsoids with human
  proportions (1.80 m tall, seeded pose jitter), seen by K simulated depth
  cameras on a 2.5 m circle.  Each camera ray-casts a depth map, depth noise
  grows with z^2, normals come from cross products of neighbouring
  back-projected samples, and weights are cos(view angle) / z^2.  This stands
  in for the paper's multi-Kinect2 captures (Sec. II-A, Sec. V), whose data is
  not available.

All arrays are returned as C-contiguous float32 (points M x 3, normals M x 3,
weights M), plus the grid dims (Nx, Ny, Nz) and bbox (xmin, ymin, zmin, xmax,
ymax, zmax) as plain Python tuples.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Frame",
    "sphere_frame",
    "human_proxy_frame",
    "config_frame",
    "CONFIGS",
    "isolated_weights_frame",
    "spread_weights",
    "repose",
    "subsample",
    "batch_frames",
    "depth_views",
    "BATCH_GRIDS",
]


@dataclass
class Frame:
    points: np.ndarray   # (M, 3) float32, world units (m)
    normals: np.ndarray  # (M, 3) float32
    weights: np.ndarray  # (M,)  float32, >= 0
    dims: tuple          # (Nx, Ny, Nz)
    bbox: tuple          # (xmin, ymin, zmin, xmax, ymax, zmax)
    name: str = ""
    info: dict = None

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------------------
# Sphere
# ---------------------------------------------------------------------------
def sphere_frame(seed: int = 0, m: int = 50_000, radius: float = 0.8,
                 noise: float = 0.005, grid: int = 64,
                 half_extent: float = 1.0) -> Frame:
    """Uniform points on a sphere of ``radius`` centred in [-e, e]^3.

    Directions d = g/|g| with g ~ N(0, I3) (uniform on S^2); X = radius*d + eps
    with eps ~ N(0, noise^2 I3); N = d exactly; W = 1.  Generated in float64
    and rounded to float32.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, 3))
    d = g / np.linalg.norm(g, axis=1, keepdims=True)
    x = radius * d + noise * rng.standard_normal((m, 3))
    e = float(half_extent)
    return Frame(_f32(x), _f32(d), np.ones(m, np.float32), (grid, grid, grid),
                 (-e, -e, -e, e, e, e), name=f"sphere_{grid}^3_{m}",
                 info={"seed": seed, "radius": radius, "noise": noise})


# ---------------------------------------------------------------------------
# Human proxy: primitives and pose
# ---------------------------------------------------------------------------
def _rot(axis: str, ang: float) -> np.ndarray:
    c, s = math.cos(ang), math.sin(ang)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], float)
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], float)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], float)


def _proxy_primitives(rng: np.random.Generator) -> list:
    """Return a posed list of primitives for one seeded pose.

    Each entry is ("capsule", p0, p1, r) or ("ellipsoid", centre, R, radii)
    where R's columns are the ellipsoid's local axes in world coordinates.
    Rest pose: y up, feet at y = 0, facing +z, top of the head at 1.80 m.
    """
    def ang(sd_deg, lo=-60.0, hi=60.0):
        return math.radians(float(np.clip(rng.normal(0.0, sd_deg), lo, hi)))

    I = np.eye(3)
    prims = []
    # trunk (rigid)
    prims.append(("ellipsoid", np.array([0.0, 1.32, 0.0]), I, np.array([0.18, 0.20, 0.11])))
    prims.append(("ellipsoid", np.array([0.0, 0.95, 0.0]), I, np.array([0.17, 0.11, 0.11])))
    # neck + head chain, rotating about the neck base
    neck0 = np.array([0.0, 1.50, 0.0])
    Rn = _rot("x", ang(10, -30, 30)) @ _rot("z", ang(8, -25, 25))
    neck1 = neck0 + Rn @ np.array([0.0, 0.10, 0.0])
    head_c = neck0 + Rn @ np.array([0.0, 0.19, 0.0])
    prims.append(("capsule", neck0, neck1, 0.05))
    prims.append(("ellipsoid", head_c, Rn, np.array([0.075, 0.11, 0.09])))
    for side in (-1.0, 1.0):
        # arm chain about the shoulder, forearm about the elbow
        sh = np.array([0.20 * side, 1.45, 0.0])
        el_rest = np.array([0.24 * side, 1.17, 0.0])
        wr_rest = np.array([0.26 * side, 0.92, 0.0])
        Rs = _rot("x", ang(20)) @ _rot("z", side * math.radians(abs(np.clip(rng.normal(0, 15), -45, 45))))
        el = sh + Rs @ (el_rest - sh)
        Re = Rs @ _rot("x", -math.radians(abs(np.clip(rng.normal(0, 20), -80, 80))))
        wr = el + Re @ (wr_rest - el_rest)
        hand_c = wr + Re @ np.array([0.0, -0.08, 0.0])
        prims.append(("capsule", sh, el, 0.045))
        prims.append(("capsule", el, wr, 0.038))
        prims.append(("ellipsoid", hand_c, Re, np.array([0.03, 0.08, 0.045])))
        # leg chain about the hip, shin about the knee
        hp = np.array([0.09 * side, 0.90, 0.0])
        kn_rest = np.array([0.10 * side, 0.50, 0.0])
        an_rest = np.array([0.10 * side, 0.09, 0.0])
        Rh = _rot("x", ang(12, -40, 40)) @ _rot("z", side * math.radians(abs(np.clip(rng.normal(0, 6), -20, 20))))
        kn = hp + Rh @ (kn_rest - hp)
        Rk = Rh @ _rot("x", math.radians(abs(np.clip(rng.normal(0, 15), -70, 70))))
        an = kn + Rk @ (an_rest - kn_rest)
        foot_c = an + Rk @ np.array([0.0, -0.045, 0.05])
        prims.append(("capsule", hp, kn, 0.075))
        prims.append(("capsule", kn, an, 0.055))
        prims.append(("ellipsoid", foot_c, Rk, np.array([0.05, 0.045, 0.12])))
    # whole-body yaw about the vertical axis through the origin
    Ry = _rot("y", float(rng.uniform(0.0, 2.0 * math.pi)))
    out = []
    for p in prims:
        if p[0] == "capsule":
            out.append(("capsule", Ry @ p[1], Ry @ p[2], p[3]))
        else:
            out.append(("ellipsoid", Ry @ p[1], Ry @ p[2], p[3]))
    return out


def proxy_inside(prims: list, x: np.ndarray) -> np.ndarray:
    """Boolean mask of points (P, 3) inside the union of the primitives."""
    inside = np.zeros(x.shape[0], bool)
    for p in prims:
        if p[0] == "capsule":
            _, a, b, r = p
            ba = b - a
            t = np.clip(((x - a) @ ba) / (ba @ ba), 0.0, 1.0)
            d = x - (a + t[:, None] * ba)
            inside |= np.einsum("ij,ij->i", d, d) <= r * r
        else:
            _, c, R, rad = p
            loc = ((x - c) @ R) / rad
            inside |= np.einsum("ij,ij->i", loc, loc) <= 1.0
    return inside


def proxy_distance(prims: list, x: np.ndarray, iters: int = 0) -> np.ndarray:
    """Approximate unsigned distance of points to the union's surface.

    Capsules use the exact distance; ellipsoids use the radial scaling
    approximation |x| (1 - 1/|x/r|) which is exact for spheres.  The union's
    surface distance is taken as |min signed distance|, exact away from the
    primitive intersections.
    """
    best = np.full(x.shape[0], np.inf)
    for p in prims:
        if p[0] == "capsule":
            _, a, b, r = p
            ba = b - a
            t = np.clip(((x - a) @ ba) / (ba @ ba), 0.0, 1.0)
            d = np.linalg.norm(x - (a + t[:, None] * ba), axis=1) - r
        else:
            _, c, R, rad = p
            loc = (x - c) @ R
            k = np.linalg.norm(loc / rad, axis=1)
            k = np.maximum(k, 1e-12)
            d = np.linalg.norm(loc, axis=1) * (1.0 - 1.0 / k)
        best = np.minimum(best, d)
    return np.abs(best)


def _ray_hits(prims: list, o: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Nearest positive hit distance along unit rays d (P,3) from origin o (3,)."""
    t_best = np.full(d.shape[0], np.inf)
    for p in prims:
        if p[0] == "ellipsoid":
            _, c, R, rad = p
            ol = (R.T @ (o - c)) / rad
            dl = (d @ R) / rad
            a = np.einsum("ij,ij->i", dl, dl)
            b = dl @ ol
            cc = ol @ ol - 1.0
            h = b * b - a * cc
            ok = h >= 0
            t = np.full_like(a, np.inf)
            t[ok] = (-b[ok] - np.sqrt(h[ok])) / a[ok]
            t[t <= 0] = np.inf
        else:
            _, p0, p1, r = p
            ba = p1 - p0
            oa = o - p0
            baba = ba @ ba
            bard = d @ ba
            baoa = ba @ oa
            rdoa = d @ oa
            oaoa = oa @ oa
            a = baba - bard * bard
            b = baba * rdoa - baoa * bard
            c = baba * oaoa - baoa * baoa - r * r * baba
            h = b * b - a * c
            t = np.full(d.shape[0], np.inf)
            ok = (h >= 0) & (a > 1e-12)
            tb = np.full(d.shape[0], np.inf)
            tb[ok] = (-b[ok] - np.sqrt(h[ok])) / a[ok]
            y = baoa + tb * bard
            body = ok & (y > 0) & (y < baba) & (tb > 0)
            t[body] = tb[body]
            # end caps (spheres at p0 and p1)
            for centre in (p0, p1):
                oc = o - centre
                bc = d @ oc
                cc = oc @ oc - r * r
                hc = bc * bc - cc
                okc = hc >= 0
                tc = np.full(d.shape[0], np.inf)
                tc[okc] = -bc[okc] - np.sqrt(hc[okc])
                tc[tc <= 0] = np.inf
                t = np.minimum(t, tc)
        t_best = np.minimum(t_best, t)
    return t_best


# Depth camera model: 512 x 424 depth map, 70 x 60 degree field of view.
CAM_W, CAM_H = 512, 424
CAM_FX = (CAM_W / 2) / math.tan(math.radians(35.0))
CAM_FY = (CAM_H / 2) / math.tan(math.radians(30.0))
CAM_CX, CAM_CY = (CAM_W - 1) / 2.0, (CAM_H - 1) / 2.0


def _camera(theta, dist=2.5, height=1.0):
    """Camera centre C and camera-to-world rotation (columns: right, down,
    forward) of a view at angle theta on the circle, looking at the body axis."""
    C = np.array([dist * math.sin(theta), height, dist * math.cos(theta)])
    f = np.array([0.0, height, 0.0]) - C
    f /= np.linalg.norm(f)
    up = np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return C, np.stack([right, down, f], axis=1)


def _render_view(prims, theta, rng, dist=2.5, height=1.0, ss=4,
                 noise_mm=1.5, jump=0.05):
    """Ray-cast one depth view and return (points, normals, weights) in world."""
    C, Rcw = _camera(theta, dist, height)  # camera -> world (columns)

    # pixel window covering the body (project a padded world box)
    corners = np.array([[x, y, z] for x in (-1.0, 1.0) for y in (-0.05, 1.9)
                        for z in (-1.0, 1.0)])
    loc = (corners - C) @ Rcw
    us = CAM_FX * loc[:, 0] / loc[:, 2] + CAM_CX
    vs = CAM_FY * loc[:, 1] / loc[:, 2] + CAM_CY
    u0 = max(int(math.floor(us.min())) - 2, 0)
    u1 = min(int(math.ceil(us.max())) + 2, CAM_W)
    v0 = max(int(math.floor(vs.min())) - 2, 0)
    v1 = min(int(math.ceil(vs.max())) + 2, CAM_H)

    # supersampled sample grid: ss x ss rays per depth pixel
    ju = (np.arange(u0 * ss, u1 * ss) + 0.5) / ss - 0.5
    jv = (np.arange(v0 * ss, v1 * ss) + 0.5) / ss - 0.5
    uu, vv = np.meshgrid(ju, jv)                      # (H', W')
    dc = np.stack([(uu - CAM_CX) / CAM_FX, (vv - CAM_CY) / CAM_FY,
                   np.ones_like(uu)], axis=-1)        # camera-space ray, z = 1
    dn = np.linalg.norm(dc, axis=-1)
    dw = (dc / dn[..., None]) @ Rcw.T                 # unit world rays
    t = _ray_hits(prims, C, dw.reshape(-1, 3)).reshape(uu.shape)
    z = t / dn                                        # depth along the optical axis
    hit = np.isfinite(z)
    zn = np.where(hit, z, 0.0)
    zn = zn + hit * rng.standard_normal(z.shape) * (noise_mm * 1e-3) * zn ** 2
    Xc = dc * zn[..., None]                           # camera-space points

    # normals from cross products of neighbours one depth pixel away
    s = ss
    ok = hit.copy()
    ok[:, :s] = ok[:, -s:] = ok[:s, :] = ok[-s:, :] = False
    sl = (slice(s, -s), slice(s, -s))
    xr, xl = Xc[s:-s, 2 * s:], Xc[s:-s, :-2 * s]
    xd, xu = Xc[2 * s:, s:-s], Xc[:-2 * s, s:-s]
    nb_ok = (hit[s:-s, 2 * s:] & hit[s:-s, :-2 * s] & hit[2 * s:, s:-s] & hit[:-2 * s, s:-s])
    zc = zn[sl]
    for nb in (zn[s:-s, 2 * s:], zn[s:-s, :-2 * s], zn[2 * s:, s:-s], zn[:-2 * s, s:-s]):
        nb_ok &= np.abs(nb - zc) <= jump
    inner = np.zeros_like(ok)
    inner[sl] = nb_ok
    ok &= inner
    n = np.zeros_like(Xc)
    n[sl] = np.cross(xr - xl, xd - xu)
    nn = np.linalg.norm(n, axis=-1)
    ok &= nn > 0
    p = Xc[ok]
    nrm = n[ok] / nn[ok][:, None]
    facing = np.einsum("ij,ij->i", nrm, p) > 0       # must face the camera
    nrm[facing] *= -1.0
    pz = p[:, 2]
    xhat = -p / np.linalg.norm(p, axis=1, keepdims=True)
    w = np.maximum(np.einsum("ij,ij->i", xhat, nrm), 0.0) * (1.0 / pz) ** 2
    pw = C + p @ Rcw.T
    nw = nrm @ Rcw.T
    return pw, nw, w


def human_proxy_frame(seed: int = 1, views: int = 4, m: int = 400_000,
                      grid=128, box: float = 2.0, ss: int = 4,
                      centre=(0.0, 0.9, 0.0)) -> Frame:
    """Multi-view depth capture of the posed human proxy.

    ``views`` cameras at 360/views degree spacing on a 2.5 m circle at 1.0 m
    height look at the body axis.  Each renders ss x ss rays per depth pixel;
    the union of all views' valid samples is subsampled (seeded, without
    replacement, original order kept) to exactly ``m`` points, or all of them
    if fewer exist.  The bbox is a cube of side ``box`` centred at ``centre``.
    """
    rng = np.random.default_rng(seed)
    prims = _proxy_primitives(rng)
    P, N, W = [], [], []
    for k in range(views):
        p, n, w = _render_view(prims, 2.0 * math.pi * k / views, rng, ss=ss)
        P.append(p)
        N.append(n)
        W.append(w)
    P = np.concatenate(P)
    N = np.concatenate(N)
    W = np.concatenate(W)
    total = P.shape[0]
    if m is not None and total > m:
        idx = np.sort(rng.choice(total, size=m, replace=False))
        P, N, W = P[idx], N[idx], W[idx]
    g = (grid, grid, grid) if isinstance(grid, int) else tuple(grid)
    h = box / 2.0
    c = centre
    bbox = (c[0] - h, c[1] - h, c[2] - h, c[0] + h, c[1] + h, c[2] + h)
    return Frame(_f32(P), _f32(N), _f32(W), g, bbox,
                 name=f"human_proxy_{views}v_{g[0]}x{g[1]}x{g[2]}_{P.shape[0]}",
                 info={"seed": seed, "views": views, "samples": total, "ss": ss,
                       "prims": prims})


# Workloads: small correctness case, and the multi-view human proxy cases.
CONFIGS = {
    "sphere64": dict(kind="sphere", seed=0, m=50_000, grid=64),
    "proxy128": dict(kind="proxy", seed=1, views=4, m=400_000, grid=128),
    "proxy256": dict(kind="proxy", seed=1000, views=6, m=700_000, grid=256),
}


def config_frame(name: str, seed: int | None = None) -> Frame:
    c = dict(CONFIGS[name])
    kind = c.pop("kind")
    if seed is not None:
        c["seed"] = seed
    if kind == "sphere":
        return sphere_frame(**c)
    return human_proxy_frame(**c)


# ---------------------------------------------------------------------------
# Wide weight ranges (confidence weights that reach zero at silhouettes)
# ---------------------------------------------------------------------------
def isolated_weights_frame(weights=(0.01, 100.0), grid: int = 32, seed: int = 0,
                           spacing_voxels: float = 9.0, pairs: int = 1) -> Frame:
    """Groups of single points with very different weights on a small grid.

    Each group places one point per entry of ``weights`` on a line along x,
    ``spacing_voxels`` voxels apart (far enough that their 4^3 footprints do
    not overlap when the spacing exceeds 4), at seeded sub-voxel offsets, with
    seeded unit normals.  Groups are stacked along y and z.  The bbox is
    [-1, 1]^3 and the grid ``grid``^3.
    """
    rng = np.random.default_rng(seed)
    h = 2.0 / grid
    P, N, W = [], [], []
    for g in range(pairs):
        base = np.array([-0.5, -0.5 + 0.45 * (g % 3), -0.5 + 0.45 * (g // 3)])
        for j, w in enumerate(weights):
            off = rng.uniform(0.0, 1.0, 3) * h
            P.append(base + np.array([j * spacing_voxels * h, 0.0, 0.0]) + off)
            n = rng.standard_normal(3)
            N.append(n / np.linalg.norm(n))
            W.append(w)
    m = len(P)
    return Frame(_f32(np.array(P)), _f32(np.array(N)), _f32(np.array(W)),
                 (grid, grid, grid), (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0),
                 name=f"isolated_weights_{m}", info={"seed": seed, "weights": tuple(weights)})


def spread_weights(frame: Frame, decades: float = 4.0, seed: int = 0) -> Frame:
    """The same frame with every weight multiplied by 10^U(-decades/2, decades/2)
    (seeded), so the weights span about ``decades`` more powers of ten."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(-0.5 * decades, 0.5 * decades, frame.n_points)
    w = frame.weights.astype(np.float64) * 10.0 ** f
    info = dict(frame.info or {})
    info["weight_decades"] = decades
    return Frame(frame.points, frame.normals, _f32(w), frame.dims, frame.bbox,
                 name=frame.name + f"_w{decades:g}dec", info=info)


# ---------------------------------------------------------------------------
# Cheap variants of a captured frame
# ---------------------------------------------------------------------------
def repose(frame: Frame, seed: int, max_shift: float = 0.05) -> Frame:
    """The same capture with the whole rig turned about the vertical axis
    through the box centre by a seeded yaw in [0, 2 pi) and shifted by a
    seeded horizontal offset of at most ``max_shift`` (metres) per axis:
    points and normals are rotated, weights kept.  Ray-casting a human-proxy
    frame takes seconds; a pool of many distinct frames for a benchmark is
    made from a few captures this way (each variant lands on different
    voxels and tiles, so no two frames share their binned data)."""
    rng = np.random.default_rng(seed)
    yaw = rng.uniform(0.0, 2.0 * math.pi)
    shift = rng.uniform(-max_shift, max_shift, 2)
    c, s_ = math.cos(yaw), math.sin(yaw)
    R = np.array([[c, 0.0, s_], [0.0, 1.0, 0.0], [-s_, 0.0, c]])
    b = np.asarray(frame.bbox, np.float64)
    ctr = 0.5 * (b[:3] + b[3:])
    ctr[1] = 0.0
    p = (frame.points.astype(np.float64) - ctr) @ R.T + ctr
    p[:, 0] += shift[0]
    p[:, 2] += shift[1]
    n = frame.normals.astype(np.float64) @ R.T
    info = dict(frame.info or {})
    info.update(repose_seed=seed, yaw=yaw, shift=tuple(shift))
    return Frame(_f32(p), _f32(n), frame.weights.copy(), frame.dims, frame.bbox,
                 name=frame.name + f"_repose{seed}", info=info)


def subsample(frame: Frame, m: int, seed: int) -> Frame:
    """``m`` of the frame's points (seeded, without replacement, original
    order kept), or all of them if it has fewer."""
    if frame.n_points <= m:
        return frame
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(frame.n_points, size=m, replace=False))
    return Frame(frame.points[idx], frame.normals[idx], frame.weights[idx], frame.dims, frame.bbox,
                 name=frame.name + f"_m{m}", info=frame.info)


# Batched workload: 16 frames of uneven size.
BATCH_GRIDS = (96, 128, 160, 192)
_BATCH_CAPTURES = ((2, 7), (4, 5), (6, 4))  # (views, supersampling): >= 800k samples each


def batch_frames(n: int = 16, seed: int = 4000, captures: dict | None = None):
    """Frames of the batched workload: frame f draws (seeded by seed + f) a
    capture of 2, 4 or 6 views of the human proxy, a point count
    M ~ U[100k, 800k], a grid from {96, 128, 160, 192}^3 and a repose of the
    rig (yaw and shift), over the same 2.0 m box.  The three captures are
    ray-cast once (seeds seed + views; at 4x4 to 6x6 rays per depth pixel so
    that each holds at least 800k samples) and passed in ``captures`` to
    reuse them.  Returns (frames, captures)."""
    if captures is None:
        captures = {v: human_proxy_frame(seed=seed + v, views=v, m=None, grid=128, ss=ss)
                    for v, ss in _BATCH_CAPTURES}
    views = sorted(captures)
    out = []
    for f in range(n):
        rng = np.random.default_rng(seed + f)
        v = views[int(rng.integers(0, len(views)))]
        m = int(rng.integers(100_000, 800_001))
        g = int(BATCH_GRIDS[int(rng.integers(0, len(BATCH_GRIDS)))])
        fr = repose(subsample(captures[v], m, seed=seed + 100 + f), seed=seed + 200 + f)
        out.append(Frame(fr.points, fr.normals, fr.weights, (g, g, g), fr.bbox,
                         name=f"batch{seed}_{f}_{v}v_{g}_{fr.n_points}",
                         info={"views": v, "m": fr.n_points, "grid": g}))
    return out, captures


# ---------------------------------------------------------------------------
# Raw depth maps (the input of the front end of Sec. III-A)
# ---------------------------------------------------------------------------
def depth_views(seed: int = 1, views: int = 4, noise_mm: float = 1.5, dist: float = 2.5,
                height: float = 1.0):
    """K full depth maps of the posed human proxy at the camera's native
    512 x 424 resolution, one ray per pixel: depth along the optical axis in
    metres (0 where the ray misses), noise N(0, (noise_mm (z / 1 m)^2)^2).

    Returns (depth (K, 424, 512) float32, cams (K, 16) float32, prims): each
    camera row is fx, fy, cx, cy, then the camera-to-world rotation R (3 x 3,
    row-major; columns right, down, forward) and the centre t, so that pixel
    (u, v) at depth D is the camera-space point ((u - cx) D / fx,
    (v - cy) D / fy, D) and the world point R x + t."""
    rng = np.random.default_rng(seed)
    prims = _proxy_primitives(rng)
    depth = np.zeros((views, CAM_H, CAM_W), np.float32)
    cams = np.zeros((views, 16), np.float32)
    uu, vv = np.meshgrid(np.arange(CAM_W, dtype=np.float64), np.arange(CAM_H, dtype=np.float64))
    dc = np.stack([(uu - CAM_CX) / CAM_FX, (vv - CAM_CY) / CAM_FY, np.ones_like(uu)], axis=-1)
    dn = np.linalg.norm(dc, axis=-1)
    for k in range(views):
        C, Rcw = _camera(2.0 * math.pi * k / views, dist, height)
        dw = (dc / dn[..., None]) @ Rcw.T
        t = _ray_hits(prims, C, dw.reshape(-1, 3)).reshape(uu.shape)
        z = t / dn
        hit = np.isfinite(z)
        zn = np.where(hit, z, 0.0)
        zn = zn + hit * rng.standard_normal(z.shape) * (noise_mm * 1e-3) * zn ** 2
        depth[k] = zn
        cams[k, :4] = (CAM_FX, CAM_FY, CAM_CX, CAM_CY)
        cams[k, 4:13] = Rcw.reshape(-1)
        cams[k, 13:16] = C
    return depth, cams, prims
