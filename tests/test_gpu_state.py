"""GPU: reproducibility, state carried between calls, and degenerate inputs.

The splat sums in exact integer fixed point, so the indicator, the level and
the mesh are bit-identical from run to run; a context that has served other
grid shapes must give the same results as a fresh one (its plans, occupancy
flags, per-point codes and scratch persist between calls).
"""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _frame_dev(f):
    return _dev(f.points), _dev(f.normals), None if f.weights is None else _dev(f.weights)


def _random_frame(seed, m, dims, bbox):
    rng = np.random.default_rng(seed)
    b = np.asarray(bbox, np.float64)
    p = rng.uniform(b[:3], b[3:], (m, 3))
    n = rng.standard_normal((m, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    w = rng.uniform(0.05, 2.0, m)
    return synth.Frame(p.astype(np.float32), n.astype(np.float32), w.astype(np.float32),
                       tuple(dims), tuple(float(x) for x in bbox))


def _mesh_np(mesh):
    return mesh.vertices.cpu().numpy(), mesh.triangles.cpu().numpy()


def _hausdorff(a, b):
    from scipy.spatial import cKDTree
    if len(a) == 0 and len(b) == 0:
        return 0.0
    return float(max(cKDTree(b).query(a)[0].max(), cKDTree(a).query(b)[0].max()))


def test_repeated_calls_are_bit_identical(ctx):
    f = synth.config_frame("proxy128")
    print(f"[repeat] proxy128 {f.n_points} points", flush=True)
    dev = _frame_dev(f)
    A1, L1 = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    A2, L2 = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    assert torch.equal(A1, A2) and L1 == L2
    m1 = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    m2 = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    assert torch.equal(m1.vertices, m2.vertices) and torch.equal(m1.triangles, m2.triangles)
    assert m1.level == m2.level == L1


def test_context_reuse_across_grid_shapes(ctx):
    a = synth.sphere_frame(seed=3, m=30_000, grid=64)
    b = _random_frame(5, 20_000, (30, 24, 40), (0.0, 0.0, 0.0, 1.2, 0.9, 1.5))
    c = synth.config_frame("proxy128")
    print("[reuse] 64^3 sphere, 30x24x40 random, proxy128, then the sphere again", flush=True)
    first = _mesh_np(ctx.reconstruct(*_frame_dev(a), grid_dim=a.dims, bbox=a.bbox))
    ctx.reconstruct(*_frame_dev(b), grid_dim=b.dims, bbox=b.bbox)
    ctx.reconstruct(*_frame_dev(c), grid_dim=c.dims, bbox=c.bbox)
    again = _mesh_np(ctx.reconstruct(*_frame_dev(a), grid_dim=a.dims, bbox=a.bbox))
    fresh_ctx = fvr.Context(0)
    fresh = _mesh_np(fresh_ctx.reconstruct(*_frame_dev(a), grid_dim=a.dims, bbox=a.bbox))
    fresh_ctx.close()
    for x, y in ((first, again), (first, fresh)):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


def test_proxy128_end_to_end(ctx):
    """The 4-view, 400k-point, 128^3 configuration at full size."""
    f = synth.config_frame("proxy128")
    dev = _frame_dev(f)
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    mesh = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    Ao = r["A"]
    rng_ = Ao.max() - Ao.min()
    err = np.abs(A.cpu().numpy() - Ao).max()
    h = (f.bbox[3] - f.bbox[0]) / f.dims[0]
    hd = _hausdorff(mesh.vertices.cpu().numpy().astype(np.float64), r["verts"])
    print(f"[proxy128] A rel err={err / rng_:.3g} V={mesh.vertices.shape[0]} (oracle {len(r['verts'])}) "
          f"Hausdorff/h={hd / h:.3g}", flush=True)
    assert err <= 1e-4 * rng_
    assert abs(L - r["level"]) <= 1e-4 * rng_
    assert hd <= 0.01 * h
    assert abs(mesh.vertices.shape[0] - len(r["verts"])) <= 0.001 * len(r["verts"])


def _indicator_vs_oracle(ctx, f):
    A, L = ctx.indicator(*_frame_dev(f), grid_dim=f.dims, bbox=f.bbox)
    V, _, _, _ = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
    Ao = oracle.indicator(V, f.dims, f.bbox)
    Lo, _ = oracle.level(Ao, f.points, f.dims, f.bbox)
    return A.cpu().numpy(), L, Ao, Lo


def test_single_point(ctx):
    p = np.array([[0.013, -0.021, 0.007]], np.float32)
    n = np.array([[0.6, 0.0, 0.8]], np.float32)
    f = synth.Frame(p, n, np.array([1.5], np.float32), (32, 32, 32), (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0))
    A, L, Ao, Lo = _indicator_vs_oracle(ctx, f)
    rng_ = Ao.max() - Ao.min()
    assert rng_ > 0
    assert np.abs(A - Ao).max() <= 1e-4 * rng_
    assert abs(L - Lo) <= 1e-4 * rng_


def test_points_on_bbox_faces(ctx):
    """Points on the closed box's faces and corners are accepted (footprint
    origins -1 and N - 1), like the oracle."""
    rng = np.random.default_rng(8)
    bbox = (-1.0, -0.5, -0.75, 1.0, 0.5, 0.75)
    lo, hi = np.array(bbox[:3]), np.array(bbox[3:])
    p = rng.uniform(lo, hi, (4000, 3))
    for a in range(3):  # pin a third of the points to one face each
        p[a::3, a] = np.where(rng.random(p[a::3].shape[0]) < 0.5, lo[a], hi[a])
    p[:8] = np.array([[lo[0] if i & 1 else hi[0], lo[1] if i & 2 else hi[1], lo[2] if i & 4 else hi[2]]
                      for i in range(8)])
    n = rng.standard_normal((4000, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    f = synth.Frame(p.astype(np.float32), n.astype(np.float32), None, (24, 16, 20), bbox)
    A, L, Ao, Lo = _indicator_vs_oracle(ctx, f)
    rng_ = Ao.max() - Ao.min()
    assert np.abs(A - Ao).max() <= 1e-4 * rng_
    mesh = ctx.reconstruct(*_frame_dev(f), grid_dim=f.dims, bbox=f.bbox)
    assert mesh.n_rejected == 0


def test_zero_weights_give_an_empty_surface(ctx):
    f = synth.sphere_frame(seed=1, m=5000, grid=32)
    w = np.zeros(f.n_points, np.float32)
    g = synth.Frame(f.points, f.normals, w, f.dims, f.bbox)
    A, L = ctx.indicator(*_frame_dev(g), grid_dim=g.dims, bbox=g.bbox)
    assert float(A.abs().max()) == 0.0 and L == 0.0
    mesh = ctx.reconstruct(*_frame_dev(g), grid_dim=g.dims, bbox=g.bbox)
    assert mesh.vertices.shape[0] == 0 and mesh.triangles.shape[0] == 0


def test_one_dense_bin(ctx):
    """Thousands of points sharing one footprint-origin row (one bin): long
    bin lists and many items per tile."""
    rng = np.random.default_rng(4)
    m = 6000
    # y in [0.05, 0.06], z in [-0.047, -0.037]: footprint origins 16 and 14 (h = 0.0625)
    p = np.stack([rng.uniform(-0.9, 0.9, m), 0.05 + rng.uniform(0.0, 0.01, m),
                  -0.047 + rng.uniform(0.0, 0.01, m)], 1)
    n = rng.standard_normal((m, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    f = synth.Frame(p.astype(np.float32), n.astype(np.float32), rng.uniform(0.1, 1.0, m).astype(np.float32),
                    (32, 32, 32), (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0))
    A, L, Ao, Lo = _indicator_vs_oracle(ctx, f)
    rng_ = Ao.max() - Ao.min()
    assert np.abs(A - Ao).max() <= 1e-4 * rng_
    assert abs(L - Lo) <= 1e-4 * rng_


def test_prepared_frame_matches_reconstruct_and_reads_refilled_inputs(ctx):
    """Context.prepare marshals the call once; each run() must equal
    reconstruct() on the buffers' current contents, bit for bit."""
    fa = synth.config_frame("sphere64")
    fb = synth.config_frame("sphere64", seed=5)
    assert fb.n_points == fa.n_points and fb.dims == fa.dims and fb.bbox == fa.bbox
    print(f"[prepared] sphere64 {fa.n_points} points, seeds 0 and 5 through one staging buffer",
          flush=True)
    pa, pb = _frame_dev(fa), _frame_dev(fb)
    ref_a = _mesh_np(ctx.reconstruct(*pa, grid_dim=fa.dims, bbox=fa.bbox))
    ref_b = _mesh_np(ctx.reconstruct(*pb, grid_dim=fb.dims, bbox=fb.bbox))
    assert not np.array_equal(ref_a[0], ref_b[0])
    staging = tuple(t.clone() for t in pa)
    nv_max = max(len(ref_a[0]), len(ref_b[0]))
    nt_max = max(len(ref_a[1]), len(ref_b[1]))
    out = (torch.empty((nv_max, 3), dtype=torch.float32, device="cuda"),
           torch.empty((nt_max, 3), dtype=torch.int32, device="cuda"))
    prep = ctx.prepare(*staging, grid_dim=fa.dims, bbox=fa.bbox, out=out)
    for want, src in ((ref_a, pa), (ref_b, pb), (ref_a, pa)):
        for dst, s in zip(staging, src):
            dst.copy_(s)
        nv, nt = prep.run()
        got = _mesh_np(prep.mesh())
        assert (nv, nt) == (len(want[0]), len(want[1]))
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_prepared_frame_reports_a_capacity_shortfall(ctx):
    f = synth.config_frame("sphere64")
    print("[prepared] capacity shortfall", flush=True)
    dev = _frame_dev(f)
    full = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    out = (torch.empty((16, 3), dtype=torch.float32, device="cuda"),
           torch.empty((16, 3), dtype=torch.int32, device="cuda"))
    prep = ctx.prepare(*dev, grid_dim=f.dims, bbox=f.bbox, out=out)
    with pytest.raises(fvr.FvrError) as e:
        prep.run()
    assert "CAPACITY" in str(e.value)
    # the required counts are reported in the prepared call's mesh struct
    assert prep._m.n_vertices == full.vertices.shape[0]
    assert prep._m.n_triangles == full.triangles.shape[0]


def test_level_finished_by_the_block_classification_has_the_same_bits():
    """At N_x = N_y = 256 the marching-cubes block classification reduces the
    level's block partials itself; the result must equal the separate final
    reduction that fvr_indicator runs, bit for bit."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fvr.Context(0)
    f = synth.config_frame("sphere64")
    dims = (256, 256, 96)
    print(f"[level fold] sphere {f.n_points} points on {dims}", flush=True)
    dev = _frame_dev(f)
    _, L = c.indicator(*dev, grid_dim=dims, bbox=f.bbox)
    m = c.reconstruct(*dev, grid_dim=dims, bbox=f.bbox)
    assert m.level == L
    assert m.vertices.shape[0] > 0
    c.close()
