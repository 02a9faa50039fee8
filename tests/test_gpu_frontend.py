"""The depth front end (Sec. III-A) on the GPU against the oracle, and the
whole path from depth maps to a mesh."""
import numpy as np
import pytest

import oracle
import synth
from oracle import frontend

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_03084_amd as fvr  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fvr.Context(0)


@pytest.fixture(scope="module")
def views():
    return synth.depth_views(seed=1, views=4)


@pytest.mark.parametrize("tau,radius", [(0.05, 10), (0.02, 3), (1.0, 0)])
def test_front_end_parity(ctx, views, tau, radius):
    depth, cams, prims = views
    print(f"[front end] 4 views 512x424, tau {tau}, radius {radius}", flush=True)
    P, N, W = ctx.depth_to_points(torch.from_numpy(depth).cuda(), cams, tau, radius)
    Po, No, Wo, valid = frontend.depth_front_end(depth, cams, tau, radius)
    assert P.shape[0] == len(Po) == int(valid.sum())        # the same pixels, the same order
    ep = np.abs(P.cpu().numpy() - Po).max()
    en = np.abs(N.cpu().numpy() - No).max()
    ew = np.abs(W.cpu().numpy() - Wo).max()
    print(f"  {len(Po)} points: max err position {ep:.3g} m, normal {en:.3g}, weight {ew:.3g}", flush=True)
    assert ep <= 1e-5 and en <= 1e-4 and ew <= 1e-5


def test_front_end_capacity_and_invalid_arguments(ctx, views):
    depth, cams, _ = views
    d = torch.from_numpy(depth).cuda()
    with pytest.raises(fvr.FvrError) as e:
        ctx.depth_to_points(d, cams, capacity=10)
    assert e.value.status == -4
    bad = cams.copy()
    bad[0, 0] = 0.0
    with pytest.raises(fvr.FvrError) as e:
        ctx.depth_to_points(d, bad)
    assert e.value.status == -1


def test_depth_maps_to_mesh(ctx, views):
    """Depth maps in, mesh out, on the device: the mesh lies on the
    analytic proxy surface (median distance under a quarter voxel) and
    matches the oracle's reconstruction of the oracle's points."""
    from scipy.spatial import cKDTree
    depth, cams, prims = views
    P, N, W = ctx.depth_to_points(torch.from_numpy(depth).cuda(), cams)
    dims, bbox = (128, 128, 128), (-1.0, -0.1, -1.0, 1.0, 1.9, 1.0)
    mesh = ctx.reconstruct(P, N, W, grid_dim=dims, bbox=bbox)
    v = mesh.vertices.cpu().numpy().astype(np.float64)
    h = 2.0 / 128
    d = synth.proxy_distance(prims, v) / h
    Po, No, Wo, _ = frontend.depth_front_end(depth, cams)
    r = oracle.reconstruct(Po.astype(np.float32), No.astype(np.float32), Wo.astype(np.float32), dims, bbox)
    hd = max(cKDTree(r["verts"]).query(v)[0].max(), cKDTree(v).query(r["verts"])[0].max())
    print(f"[depth->mesh] {len(P)} points, {len(v)} vertices: median distance {np.median(d):.3f} h, "
          f"Hausdorff to the oracle {hd / h:.3g} h", flush=True)
    assert np.median(d) < 0.25 and len(v) > 1000
    assert hd <= 0.01 * h
