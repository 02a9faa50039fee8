"""Pins of the oracle's front end (Sec. III-A: raw points, organized-
triangulation normals, confidence weights W1 W2), against closed forms and
brute force."""
import numpy as np

from oracle import frontend

FX, FY, CX, CY = 300.0, 280.0, 15.5, 11.5
H, W = 24, 32


def _cams(R=None, t=None):
    c = np.zeros((1, 16), np.float32)
    c[0, :4] = (FX, FY, CX, CY)
    c[0, 4:13] = (np.eye(3) if R is None else R).reshape(-1)
    c[0, 13:16] = (0.0, 0.0, 0.0) if t is None else t
    return c


def _rays():
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    return np.stack([(u - CX) / FX, (v - CY) / FY, np.ones_like(u)], axis=-1)


def test_fronto_parallel_plane():
    z0 = 2.0
    depth = np.full((1, H, W), z0, np.float32)
    P, N, Wt, valid = frontend.depth_front_end(depth, _cams(), tau=0.05, radius=3)
    assert valid.all() and len(P) == H * W
    r = _rays().reshape(-1, 3)
    np.testing.assert_allclose(P, r * z0, rtol=0, atol=1e-12)             # exact back-projection
    np.testing.assert_allclose(N, np.tile([0.0, 0.0, -1.0], (H * W, 1)), atol=1e-12)   # faces the camera
    cosang = 1.0 / np.linalg.norm(r, axis=1)                                # W1 = cos(view angle)
    w2 = frontend.box_counts(np.ones((H, W), bool), 3).reshape(-1) / 49.0
    np.testing.assert_allclose(Wt, cosang * w2, rtol=1e-12)
    # W2 closed forms: interior 1, corner (r+1)^2/(2r+1)^2, edge (r+1)/(2r+1)
    b = frontend.box_counts(np.ones((H, W), bool), 3) / 49.0
    assert b[10, 10] == 1.0 and b[0, 0] == 16 / 49 and b[0, 10] == 4 / 7


def test_tilted_plane_normals_and_world_transform():
    n = np.array([0.3, -0.4, -0.866])
    n /= np.linalg.norm(n)
    dplane = -2.0                                           # n . X = d, in front of the camera
    depth = (dplane / (_rays() @ n))[None].astype(np.float32)
    ang = 0.7
    R = np.array([[np.cos(ang), 0, np.sin(ang)], [0, 1, 0], [-np.sin(ang), 0, np.cos(ang)]])
    t = np.array([1.0, 0.5, -2.0])
    P, N, Wt, valid = frontend.depth_front_end(depth, _cams(R, t), tau=1.0, radius=2)
    assert valid.all()
    facing = n if n[2] < 0 else -n                          # the side seen by the camera
    # the float32 depths put the points up to 2^-24 D off the plane, a
    # normal error of order f 2^-24 (2e-5 at f = 300)
    np.testing.assert_allclose(N, np.tile(R @ facing, (len(N), 1)), atol=1e-4)
    Ploc = (P - t) @ R                                      # back to camera coordinates
    np.testing.assert_allclose(Ploc @ n, dplane, atol=1e-5)


def test_step_discontinuity_and_isolated_pixels():
    depth = np.full((1, H, W), 2.0, np.float32)
    depth[0, :, W // 2:] = 2.5                              # a 0.5 m step
    depth[0, 5, 3] = 0.0                                    # a hole
    depth[0, 0:3, 0:3] = 0.0
    depth[0, 1, 1] = 2.0                                    # an isolated foreground pixel
    P, N, Wt, valid = frontend.depth_front_end(depth, _cams(), tau=0.05, radius=2)
    assert not valid[0, 1, 1] and not valid[0, 5, 3]
    assert valid[0, 10, W // 2 - 1] and valid[0, 10, W // 2]
    np.testing.assert_allclose(N, np.tile([0.0, 0.0, -1.0], (len(N), 1)), atol=1e-12)
    # a pixel next to the hole lost the triangles through the hole only
    assert valid[0, 5, 2] and valid[0, 5, 4]


def test_box_counts_brute_force():
    rng = np.random.default_rng(0)
    m = rng.random((9, 12)) < 0.6
    for r in (0, 1, 2, 5):
        bc = frontend.box_counts(m, r)
        for y in range(9):
            for x in range(12):
                s = sum(int(m[yy, xx]) for yy in range(y - r, y + r + 1) for xx in range(x - r, x + r + 1)
                        if 0 <= yy < 9 and 0 <= xx < 12)
                assert bc[y, x] == s


def test_sphere_normals_face_the_camera_and_are_radial():
    c0 = np.array([0.05, -0.03, 2.2])
    rad = 0.5
    d = _rays()
    dn = d / np.linalg.norm(d, axis=-1, keepdims=True)
    b = dn @ c0
    disc = b * b - (c0 @ c0 - rad * rad)
    tt = np.where(disc > 0, b - np.sqrt(np.maximum(disc, 0)), np.nan)
    depth = np.where(np.isfinite(tt), tt / np.linalg.norm(d, axis=-1), 0.0)[None].astype(np.float32)
    P, N, Wt, valid = frontend.depth_front_end(depth, _cams(), tau=0.2, radius=2)
    assert len(P) > 100
    assert np.all(np.sum(N * P, axis=1) < 0)                # towards the camera (at the origin)
    radial = (P - c0) / np.linalg.norm(P - c0, axis=1, keepdims=True)
    cosr = np.sum(N * radial, axis=1) / np.linalg.norm(N, axis=1)
    inner = Wt > 0.3 * Wt.max()
    assert np.min(cosr[inner]) > 0.99
    # raster order within the view
    vv, uu = np.nonzero(valid[0])
    np.testing.assert_allclose(P[:, 2], depth[0][vv, uu].astype(np.float64), atol=1e-12)
