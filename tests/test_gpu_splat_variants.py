"""The non-weighted (nearest-voxel) splat of Sec. III-B against the oracle,
and the quality comparison of the two splats on the human proxy (distance
of the mesh vertices to the analytic surface)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_03084_amd as fvr  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fvr.Context(0)


def _dev(f):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (f.points, f.normals, f.weights)]


def _random_frame(seed, m, dims, bbox):
    rng = np.random.default_rng(seed)
    b = np.asarray(bbox, np.float64)
    p = rng.uniform(b[:3] - 0.05 * (b[3:] - b[:3]), b[3:] + 0.05 * (b[3:] - b[:3]), (m, 3))
    n = rng.standard_normal((m, 3))
    return synth.Frame(p.astype(np.float32), n.astype(np.float32),
                       rng.uniform(0.0, 3.0, m).astype(np.float32), dims, bbox)


CASES = [
    ("sphere64", lambda: synth.sphere_frame(seed=0, m=50_000, grid=64)),
    ("random ragged 30x24x40", lambda: _random_frame(5, 40_000, (30, 24, 40), (0.0, 0.0, 0.0, 1.2, 0.9, 1.5))),
    ("random dense 16^3 (many points per voxel)",
     lambda: _random_frame(6, 60_000, (16, 16, 16), (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0))),
]


@pytest.mark.parametrize("name,make", CASES)
def test_nearest_splat_parity(ctx, name, make):
    f = make()
    dev = _dev(f)
    V = ctx.debug_splat(*dev, grid_dim=f.dims, bbox=f.bbox, splat="nearest").cpu().numpy()
    Vo, cnt, _ = oracle.splat_nearest(f.points, f.normals, f.dims, f.bbox)
    ev = np.abs(V - Vo).max() / np.abs(Vo).max()
    assert np.array_equal(np.abs(V).sum(0) > 0, (cnt > 0) & (np.abs(Vo).sum(0) > 0))
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox, splat="nearest")
    Ao = oracle.indicator(Vo, f.dims, f.bbox)
    Lo, _ = oracle.level(Ao, f.points, f.dims, f.bbox)
    rng_ = Ao.max() - Ao.min()
    ea = np.abs(A.cpu().numpy() - Ao).max() / rng_
    print(f"[nearest] {name}: V rel {ev:.3g}, A rel {ea:.3g}, L rel {abs(L - Lo) / rng_:.3g}", flush=True)
    assert ev <= 1e-6
    assert ea <= 1e-5 and abs(L - Lo) <= 1e-5 * rng_


def test_nearest_splat_end_to_end_and_weights_ignored(ctx):
    from scipy.spatial import cKDTree
    f = synth.sphere_frame(seed=1, m=50_000, grid=64)
    p, n, w = _dev(f)
    mesh = ctx.reconstruct(p, n, w, grid_dim=f.dims, bbox=f.bbox, splat="nearest")
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox, splat_variant="nearest")
    v = mesh.vertices.cpu().numpy().astype(np.float64)
    hd = max(cKDTree(r["verts"]).query(v)[0].max(), cKDTree(v).query(r["verts"])[0].max())
    h = 2.0 / 64
    print(f"[nearest] sphere e2e: V={len(v)} (oracle {len(r['verts'])}) Hausdorff/h={hd / h:.3g}")
    assert hd <= 0.01 * h and len(v) == len(r["verts"])
    other = ctx.reconstruct(p, n, torch.rand_like(w) * 5, grid_dim=f.dims, bbox=f.bbox, splat="nearest")
    assert torch.equal(other.vertices, mesh.vertices) and torch.equal(other.triangles, mesh.triangles)


def test_weighted_and_nearest_splat_quality_on_the_proxy(ctx):
    """Distance of the mesh vertices to the analytic human-proxy surface, for
    the weighted splat of eqs. (1)-(2) and the non-weighted one (the paper's
    real-time mode), on the 4-view 128^3 configuration."""
    f = synth.config_frame("proxy128")
    prims = f.info["prims"]
    h = 2.0 / 128
    dev = _dev(f)
    res = {}
    for variant in ("gaussian", "nearest"):
        mesh = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox, splat=variant)
        d = synth.proxy_distance(prims, mesh.vertices.cpu().numpy().astype(np.float64)) / h
        res[variant] = (float(np.median(d)), float(np.percentile(d, 95)), mesh.vertices.shape[0])
        print(f"[quality] {variant}: vertices {res[variant][2]}, distance to the analytic surface "
              f"median {res[variant][0]:.3f} h, p95 {res[variant][1]:.3f} h", flush=True)
    for variant, (med, p95, nv) in res.items():
        assert med <= 1.0 and nv > 1000
