"""FP64 oracle of the front end of Sec. III-A: depth maps to raw oriented,
confidence-weighted points.

TEST INFRASTRUCTURE ONLY (tests, smoke check and benchmark CPU baseline are
its only users); it shares no code with the GPU library.

Per view k and foreground pixel u (depth D > 0 and finite):
  X^loc(u) = Pi_k^-1(u, D) = ((u_x - c_x) D / f_x, (u_y - c_y) D / f_y, D)
  N^loc(u) = mean of the unit normals of the triangles of the organized
             triangulation in which u is a vertex (Sec. III-A; reading of the
             "terrain step discontinuity constraint triangulation"): each
             2 x 2 pixel quad a=(x,y), b=(x+1,y), c=(x,y+1), d=(x+1,y+1) is
             split along a-d when |D_a - D_d| <= |D_b - D_c|, else along b-c;
             a triangle is kept when its three pixels are foreground and no
             two of its depths differ by more than tau.  The normal of a
             triangle (p0, p1, p2) - (a, b, d), (a, d, c), (a, b, c) or
             (b, d, c) - is (p2 - p0) x (p1 - p0) normalised, the winding that
             faces the camera.
  W1(u) = max(<-X^loc/|X^loc|, N^loc>, 0)
  W2(u) = foreground pixels in the (2r+1) x (2r+1) square around u (outside
          the image: background) / (2r+1)^2       (r = 10 in the paper)
  W = W1 W2; world X = R X^loc + t, N = R N^loc.
Pixels in no kept triangle give no point.  Output: view by view, raster
order.  The integer decisions (foreground, diagonal, step test) are taken in
float32 on the float32 depths, as the GPU takes them; everything else is
float64.
"""
from __future__ import annotations

import numpy as np

__all__ = ["depth_front_end", "box_counts"]


def box_counts(mask: np.ndarray, r: int) -> np.ndarray:
    """Number of True pixels in the (2r+1)^2 square around each pixel
    (outside the image counts as False), by 2D prefix sums."""
    H, W = mask.shape
    S = np.zeros((H + 1, W + 1), np.int64)
    S[1:, 1:] = np.cumsum(np.cumsum(mask.astype(np.int64), 0), 1)
    y = np.arange(H)
    x = np.arange(W)
    y0 = np.clip(y - r, 0, H)[:, None]
    y1 = np.clip(y + r + 1, 0, H)[:, None]
    x0 = np.clip(x - r, 0, W)[None, :]
    x1 = np.clip(x + r + 1, 0, W)[None, :]
    return S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]


def depth_front_end(depth, cams, tau: float = 0.05, radius: int = 10):
    """Returns (points (M,3) f64, normals (M,3) f64, weights (M,) f64,
    valid (K,H,W) bool) for depth (K,H,W) and cams (K,16) as described in
    the module docstring."""
    depth = np.asarray(depth, np.float32)
    cams = np.asarray(cams, np.float32)
    K, H, W = depth.shape
    tau32 = np.float32(tau)
    P, N, Wt, valid = [], [], [], np.zeros((K, H, W), bool)
    for k in range(K):
        D32 = depth[k]
        fg = np.isfinite(D32) & (D32 > 0)
        Dt = np.where(fg, D32, np.float32(0.0)).astype(np.float32)   # background as 0
        fx, fy, cx, cy = (float(v) for v in cams[k, :4])
        R = cams[k, 4:13].astype(np.float64).reshape(3, 3)
        t = cams[k, 13:16].astype(np.float64)
        v, u = np.mgrid[0:H, 0:W].astype(np.float64)
        D = Dt.astype(np.float64)
        X = np.stack([(u - cx) * D / fx, (v - cy) * D / fy, D], axis=-1)
        nsum = np.zeros((H, W, 3))
        ncnt = np.zeros((H, W), np.int64)
        # quad corners a=(y,x) b=(y,x+1) c=(y+1,x) d=(y+1,x+1) for x < W-1, y < H-1
        a = (slice(0, H - 1), slice(0, W - 1))
        b = (slice(0, H - 1), slice(1, W))
        c = (slice(1, H), slice(0, W - 1))
        d = (slice(1, H), slice(1, W))
        ad = np.abs(Dt[a] - Dt[d]) <= np.abs(Dt[b] - Dt[c])           # float32 decision
        ys, xs = np.mgrid[0:H - 1, 0:W - 1]
        corner = {"a": (ys, xs), "b": (ys, xs + 1), "c": (ys + 1, xs), "d": (ys + 1, xs + 1)}
        for use, tri in ((ad, ("a", "b", "d")), (ad, ("a", "d", "c")),
                         (~ad, ("a", "b", "c")), (~ad, ("b", "d", "c"))):
            i0, i1, i2 = (corner[n] for n in tri)
            d0, d1, d2 = Dt[i0], Dt[i1], Dt[i2]
            keep = use & (d0 > 0) & (d1 > 0) & (d2 > 0)
            keep &= (np.abs(d0 - d1) <= tau32) & (np.abs(d0 - d2) <= tau32) & (np.abs(d1 - d2) <= tau32)
            p0, p1, p2 = X[i0], X[i1], X[i2]
            n = np.cross(p2 - p0, p1 - p0)
            ln = np.linalg.norm(n, axis=-1)
            keep &= ln > 0
            n = n / np.where(ln > 0, ln, 1.0)[..., None]
            for iy, ix in (i0, i1, i2):
                np.add.at(nsum, (iy[keep], ix[keep]), n[keep])
                np.add.at(ncnt, (iy[keep], ix[keep]), 1)
        ok = fg & (ncnt > 0)
        valid[k] = ok
        Nl = nsum[ok] / ncnt[ok][:, None]
        Xl = X[ok]
        w1 = np.maximum(-np.sum(Xl * Nl, axis=1) / np.linalg.norm(Xl, axis=1), 0.0)
        w2 = box_counts(fg, radius)[ok] / float((2 * radius + 1) ** 2)
        P.append(Xl @ R.T + t)
        N.append(Nl @ R.T)
        Wt.append(w1 * w2)
    return np.concatenate(P), np.concatenate(N), np.concatenate(Wt), valid
