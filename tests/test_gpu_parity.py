"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (float32 path vs double oracle):
  splat V        max |V_gpu - V_orc| <= 1e-5 * max |V_orc|
  indicator A    max |A_gpu - A_orc| <= 1e-4 * (max A_orc - min A_orc)   (stated target)
  level L        |L_gpu - L_orc|     <= 1e-4 * range(A_orc)
  marching cubes on the oracle's field rounded to float32 with L rounded to
                 float32: case bytes, vertex/triangle counts and triangle index
                 arrays bit-exact; vertex positions within 1e-4 h
  end to end     symmetric vertex Hausdorff distance to the oracle mesh <= 0.01 h
"""
import collections
import math

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
    w = None if f.weights is None else _dev(f.weights)
    return _dev(f.points), _dev(f.normals), w


def _random_frame(seed, m, dims, bbox, outside_frac=0.05):
    rng = np.random.default_rng(seed)
    b = np.asarray(bbox, np.float64)
    lo, hi = b[:3], b[3:]
    ext = hi - lo
    p = rng.uniform(lo - outside_frac * ext, hi + outside_frac * ext, (m, 3))
    n = rng.standard_normal((m, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    w = rng.uniform(0.05, 2.0, m)
    return synth.Frame(p.astype(np.float32), n.astype(np.float32), w.astype(np.float32),
                       tuple(dims), tuple(float(x) for x in bbox))


def _hausdorff(a, b):
    from scipy.spatial import cKDTree
    if len(a) == 0 and len(b) == 0:
        return 0.0
    d1 = cKDTree(b).query(a)[0].max()
    d2 = cKDTree(a).query(b)[0].max()
    return float(max(d1, d2))


def _closed(tris):
    und = collections.Counter()
    for t in tris:
        for i in range(3):
            a, b = int(t[i]), int(t[(i + 1) % 3])
            und[(min(a, b), max(a, b))] += 1
    return all(v == 2 for v in und.values()), len(und)


SPLAT_CASES = [
    ("sphere64", None),
    ("ragged_aniso", ((20, 12, 18), (-0.5, -0.3, -0.45, 0.5, 0.3, 0.45))),
    ("paper_shape", ((32, 64, 32), (-0.5, -1.0, -0.5, 0.5, 1.0, 0.5))),
    ("mixed_radix", ((30, 24, 40), (0.0, 0.0, 0.0, 1.2, 0.9, 1.5))),
]


def _case_frame(name, spec, seed=11, m=20000):
    if name == "sphere64":
        return synth.sphere_frame(seed=0, m=50_000, grid=64)
    dims, bbox = spec
    return _random_frame(seed, m, dims, bbox)


@pytest.mark.parametrize("name,spec", SPLAT_CASES)
def test_splat_parity(ctx, name, spec):
    print(f"[splat] {name}", flush=True)
    f = _case_frame(name, spec)
    V = ctx.debug_splat(*_frame_dev(f), grid_dim=f.dims, bbox=f.bbox).cpu().numpy()
    Vo, _, _, _ = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
    scale = np.abs(Vo).max()
    err = np.abs(V - Vo).max()
    print(f"  max|V|={scale:.4g} max err={err:.3g} rel={err / scale:.3g}")
    assert err <= 1e-5 * scale
    # identical support: the footprint decision is the same float32 formula
    assert np.array_equal(np.abs(V).sum(0) > 0, np.abs(Vo).sum(0) > 0)


INDICATOR_CASES = SPLAT_CASES + [
    ("paper_r6_shape", ((64, 128, 64), (-0.6, -1.2, -0.6, 0.6, 1.2, 0.6))),
    ("radix_96_160_192", ((96, 160, 192), (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0))),
    # the z pass's column kx = Nx/2 in blocks of 4 ky lines, the last of
    # 30 lines with two masked
    ("nyquist_lines_z", ((64, 30, 32), (-0.4, -0.19, -0.2, 0.4, 0.19, 0.2))),
]


@pytest.mark.parametrize("name,spec", INDICATOR_CASES)
def test_indicator_and_level_parity(ctx, name, spec):
    print(f"[indicator] {name}", flush=True)
    f = _case_frame(name, spec, m=60000)
    A, L = ctx.indicator(*_frame_dev(f), grid_dim=f.dims, bbox=f.bbox)
    A = A.cpu().numpy()
    Vo, _, _, _ = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
    Ao = oracle.indicator(Vo, f.dims, f.bbox)
    Lo, _ = oracle.level(Ao, f.points, f.dims, f.bbox)
    rng_ = Ao.max() - Ao.min()
    err = np.abs(A - Ao).max()
    print(f"  range={rng_:.4g} max err={err:.3g} rel={err / rng_:.3g}  L={L:.8g} Lo={Lo:.8g}")
    assert err <= 1e-4 * rng_
    assert abs(L - Lo) <= 1e-4 * rng_


def _mc_compare(ctx, Ao, Lo, dims, bbox):
    A32 = Ao.astype(np.float32)
    L32 = np.float32(Lo)
    mesh, cases = ctx.extract(_dev(A32), bbox, float(L32), with_cases=True)
    vo, to, co = oracle.extract(A32.astype(np.float64), float(L32), dims, bbox)
    assert np.array_equal(cases.cpu().numpy(), co)
    assert mesh.vertices.shape[0] == len(vo)
    assert mesh.triangles.shape[0] == len(to)
    assert np.array_equal(mesh.triangles.cpu().numpy(), to)
    h = (np.asarray(bbox[3:], np.float64) - np.asarray(bbox[:3], np.float64)) / np.asarray(dims)
    dv = np.abs(mesh.vertices.cpu().numpy().astype(np.float64) - vo).max(0) if len(vo) else np.zeros(3)
    print(f"  V={len(vo)} T={len(to)} max vertex err / h = {dv / h}")
    assert np.all(dv <= 1e-4 * h)
    return mesh


def _splat_and_indicator_errors(ctx, f):
    dev = _frame_dev(f)
    V = ctx.debug_splat(*dev, grid_dim=f.dims, bbox=f.bbox).cpu().numpy()
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    Vo, _, _, _ = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
    Ao = oracle.indicator(Vo, f.dims, f.bbox)
    Lo, _ = oracle.level(Ao, f.points, f.dims, f.bbox)
    ev = np.abs(V - Vo).max() / np.abs(Vo).max()
    rng_ = Ao.max() - Ao.min()
    ea = np.abs(A.cpu().numpy() - Ao).max() / rng_
    el = abs(L - Lo) / rng_
    support = np.array_equal(np.abs(V).sum(0) > 0, np.abs(Vo).sum(0) > 0)
    return ev, ea, el, support


@pytest.mark.parametrize("weights,bar", [((0.01, 100.0), 1e-5), ((1e-4, 1.0, 100.0), 1e-4)])
def test_splat_isolated_points_with_a_wide_weight_range(ctx, weights, bar):
    """Light points far from heavy ones (W = W1 W2 reaches 0 at silhouettes,
    Sec. III-A): a voxel that only a light point reaches keeps a relative
    accuracy set by the weight ratio R, not lost to the frame's largest
    weight.  The splat's fixed-point bound is 2^-47 R e^(32/3) of max |V|
    (2.9e-5 at R = 1e4, 3e-4 at R = 1e6, where the far footprint corner of a
    light point is all a voxel holds); the bar is 1e-5 at R = 1e4 and 1e-4
    at R = 1e6."""
    f = synth.isolated_weights_frame(weights, grid=32, seed=3, pairs=9)
    ev, ea, el, support = _splat_and_indicator_errors(ctx, f)
    print(f"[wide W {weights}] V rel={ev:.3g} A rel={ea:.3g} L rel={el:.3g}", flush=True)
    assert ev <= bar
    assert ea <= 1e-5 and el <= 1e-5
    assert support


def test_splat_proxy128_with_weights_over_four_decades(ctx):
    """The 4-view human proxy at 128^3 with every weight multiplied by a
    seeded 10^U(-2, 2): overlapping footprints mix terms 10^4 apart."""
    f = synth.spread_weights(synth.config_frame("proxy128"), decades=4.0, seed=7)
    assert f.weights.max() / f.weights[f.weights > 0].min() > 1e4
    ev, ea, el, support = _splat_and_indicator_errors(ctx, f)
    print(f"[proxy128 W x 10^U(-2,2)] V rel={ev:.3g} A rel={ea:.3g} L rel={el:.3g}", flush=True)
    assert ev <= 1e-5
    assert ea <= 1e-5 and el <= 1e-5
    assert support


def test_marching_cubes_bit_exact_on_oracle_field_sphere(ctx):
    f = synth.sphere_frame(seed=0, m=50_000, grid=64)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    _mc_compare(ctx, r["A"], r["level"], f.dims, f.bbox)


def test_vertex_normals_on_oracle_field(ctx):
    """Vertex normals -grad A (central differences interpolated along the
    edge, normalised) against the oracle's, vertex by vertex, on the
    oracle's field rounded to float32; and outward on the sphere."""
    f = synth.sphere_frame(seed=0, m=50_000, grid=64)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    A32 = r["A"].astype(np.float32)
    L32 = np.float32(r["level"])
    mesh = ctx.extract(_dev(A32), f.bbox, float(L32), vertex_normals=True)
    vo, to, _, no = oracle.extract(A32.astype(np.float64), float(L32), f.dims, f.bbox, with_normals=True)
    n = mesh.normals.cpu().numpy().astype(np.float64)
    err = np.abs(n - no).max()
    v = mesh.vertices.cpu().numpy().astype(np.float64)
    cosr = np.sum(n * v / np.linalg.norm(v, axis=1, keepdims=True), axis=1)
    print(f"  normals: max err {err:.3g}, min cos to radial {cosr.min():.4f}")
    assert n.shape == no.shape and err <= 1e-5
    assert cosr.min() > 0.95
    # the whole path returns the same normals for its own field
    dev = _frame_dev(f)
    rec = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox, vertex_normals=True)
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    ext = ctx.extract(A, f.bbox, L, vertex_normals=True)
    assert torch.equal(rec.normals, ext.normals) and torch.equal(rec.vertices, ext.vertices)


@pytest.mark.parametrize("seed,dims", [(0, (36, 22, 30)), (1, (36, 22, 30)), (2, (30, 14, 18)),
                                       (3, (7, 5, 9))])
def test_marching_cubes_bit_exact_random_fields(ctx, seed, dims):
    """Random fields exercise every case family, ragged block tails, surfaces
    that reach the grid border, and rows whose length is not a multiple of 4."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal(dims[::-1])
    _mc_compare(ctx, A, 0.1, dims, (0.0, 0.0, 0.0) + tuple(0.1 * d for d in dims))


def test_marching_cubes_unaligned_field(ctx):
    """A field view starting one float into its allocation (not 16-byte aligned)."""
    rng = np.random.default_rng(8)
    dims = (16, 12, 10)
    A = rng.standard_normal(dims[::-1]).astype(np.float32)
    buf = torch.empty(A.size + 1, dtype=torch.float32, device="cuda")
    view = buf[1:].view(dims[::-1])
    view.copy_(torch.from_numpy(A).cuda())
    bbox = (0.0, 0.0, 0.0, 1.6, 1.2, 1.0)
    mesh, cases = ctx.extract(view, bbox, 0.2, with_cases=True)
    vo, to, co = oracle.extract(A.astype(np.float64), float(np.float32(0.2)), dims, bbox)
    assert np.array_equal(cases.cpu().numpy(), co)
    assert np.array_equal(mesh.triangles.cpu().numpy(), to)


def test_marching_cubes_ties_are_outside(ctx):
    rng = np.random.default_rng(5)
    dims = (16, 10, 12)
    A = rng.integers(0, 3, dims[::-1]).astype(np.float64)
    _mc_compare(ctx, A, 1.0, dims, (0.0, 0.0, 0.0, 1.6, 1.0, 1.2))


def test_reconstruct_sphere_end_to_end(ctx):
    f = synth.sphere_frame(seed=0, m=50_000, grid=64)
    mesh = ctx.reconstruct(*_frame_dev(f), grid_dim=f.dims, bbox=f.bbox)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    v = mesh.vertices.cpu().numpy().astype(np.float64)
    t = mesh.triangles.cpu().numpy()
    h = 2.0 / 64
    hd = _hausdorff(v, r["verts"])
    print(f"  V={len(v)} (oracle {len(r['verts'])}) T={len(t)} Hausdorff/h={hd / h:.3g} "
          f"L={mesh.level:.8g} Lo={r['level']:.8g}")
    assert hd <= 0.01 * h
    assert np.max(np.abs(np.linalg.norm(v, axis=1) - 0.8)) <= h
    ok, ne = _closed(t)
    assert ok and len(v) - ne + len(t) == 2
    assert mesh.n_rejected == 0 and not mesh.open_surface


@pytest.mark.slow
def test_full_size_human_proxy_256(ctx):
    """The headline workload: 6-view human proxy, 700k points, 256^3."""
    print("[full] generating human proxy 6 views 256^3", flush=True)
    f = synth.config_frame("proxy256")
    dev = _frame_dev(f)
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    mesh = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    print("[full] oracle", flush=True)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    Ao = r["A"]
    rng_ = Ao.max() - Ao.min()
    err = np.abs(A.cpu().numpy() - Ao).max()
    h = 2.0 / 256
    hd = _hausdorff(mesh.vertices.cpu().numpy().astype(np.float64), r["verts"])
    print(f"  A rel err={err / rng_:.3g} L={L:.8g} Lo={r['level']:.8g} V={mesh.vertices.shape[0]} "
          f"(oracle {len(r['verts'])}) Hausdorff/h={hd / h:.3g}")
    assert err <= 1e-4 * rng_
    assert abs(L - r["level"]) <= 1e-4 * rng_
    assert abs(mesh.level - r["level"]) <= 1e-4 * rng_
    assert hd <= 0.01 * h
    assert abs(mesh.vertices.shape[0] - len(r["verts"])) <= 0.001 * len(r["verts"])
    ok, _ = _closed(mesh.triangles.cpu().numpy())
    assert ok
    # reconstruct settles most marching-cubes blocks from the row ranges of A
    # without reading it; extract classifies every point of the same field
    full = ctx.extract(A, f.bbox, L)
    assert torch.equal(full.vertices, mesh.vertices) and torch.equal(full.triangles, mesh.triangles)
    assert full.open_surface == mesh.open_surface


def test_row_range_skip_on_an_open_surface_256(ctx):
    """A sphere cut by a 256^3 box: whole blocks of cells lie inside (all above
    the level), are settled from the row ranges and must raise the open-surface
    flag; the mesh must equal the full classification of the same field."""
    f = synth.sphere_frame(seed=4, m=200_000, grid=256, half_extent=0.7)
    print("[skip] sphere r=0.8 in [-0.7, 0.7]^3, 256^3", flush=True)
    dev = _frame_dev(f)
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    mesh = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    full = ctx.extract(A, f.bbox, L)
    assert mesh.open_surface and full.open_surface
    assert mesh.vertices.shape[0] > 0
    assert torch.equal(full.vertices, mesh.vertices) and torch.equal(full.triangles, mesh.triangles)


@pytest.mark.parametrize("dims", [(256, 256, 96), (128, 128, 48), (128, 128, 16)])
def test_fused_inverse_passes(ctx, dims):
    """N_x = N_y = 256 and N_x = N_y = 128 take the fused inverse y/x pass
    whatever N_z is: indicator against the oracle, mesh against the full
    classification of the same field."""
    half = tuple(d / dims[0] for d in dims)
    f = _random_frame(21 + dims[2], 60_000, dims, tuple(-x for x in half) + half)
    print(f"[fused] random frame {dims}", flush=True)
    dev = _frame_dev(f)
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    Vo, _, _, _ = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
    Ao = oracle.indicator(Vo, f.dims, f.bbox)
    Lo, _ = oracle.level(Ao, f.points, f.dims, f.bbox)
    rng_ = Ao.max() - Ao.min()
    err = np.abs(A.cpu().numpy() - Ao).max()
    print(f"  range={rng_:.4g} rel err={err / rng_:.3g} L={L:.8g} Lo={Lo:.8g}")
    assert err <= 1e-4 * rng_
    assert abs(L - Lo) <= 1e-4 * rng_
    mesh = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    full = ctx.extract(A, f.bbox, L)
    assert mesh.vertices.shape[0] > 0
    assert torch.equal(full.vertices, mesh.vertices) and torch.equal(full.triangles, mesh.triangles)
    assert full.open_surface == mesh.open_surface


@pytest.mark.parametrize("dims", [(128, 128, 128), (64, 64, 48), (96, 160, 192), (160, 96, 64)])
def test_row_range_skip_after_unfused_inverse_passes(ctx, dims):
    """Grids other than N_x = N_y = 256 run the inverse y and x passes apart
    (register pencils on power-of-two lengths, mixed-radix passes on the
    others); the x pass leaves the row ranges of A for the marching-cubes
    block list: the mesh must equal the full classification of the same
    field."""
    half = tuple(0.5 * d / 64.0 for d in dims)
    f = _random_frame(30 + dims[0] + dims[2], 80_000, dims, tuple(-h for h in half) + half)
    print(f"[skip] random frame {dims}", flush=True)
    dev = _frame_dev(f)
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    mesh = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    full = ctx.extract(A, f.bbox, L)
    assert mesh.vertices.shape[0] > 0
    assert torch.equal(full.vertices, mesh.vertices) and torch.equal(full.triangles, mesh.triangles)
    assert full.open_surface == mesh.open_surface and mesh.level == L


def test_row_range_skip_on_an_open_surface_128(ctx):
    """The open-surface flag from blocks settled by row ranges, on the
    unfused inverse passes."""
    f = synth.sphere_frame(seed=5, m=100_000, grid=128, half_extent=0.7)
    dev = _frame_dev(f)
    A, L = ctx.indicator(*dev, grid_dim=f.dims, bbox=f.bbox)
    mesh = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
    full = ctx.extract(A, f.bbox, L)
    assert mesh.open_surface and full.open_surface
    assert torch.equal(full.vertices, mesh.vertices) and torch.equal(full.triangles, mesh.triangles)


def test_empty_and_all_rejected(ctx):
    z = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    mesh = ctx.reconstruct(z, z, None, grid_dim=(16, 16, 16), bbox=(-1, -1, -1, 1, 1, 1))
    assert mesh.vertices.shape[0] == 0 and mesh.triangles.shape[0] == 0 and mesh.level == 0.0
    p = torch.full((100, 3), 5.0, device="cuda")
    mesh = ctx.reconstruct(p, p, None, grid_dim=(16, 16, 16), bbox=(-1, -1, -1, 1, 1, 1))
    assert mesh.n_rejected == 100 and mesh.vertices.shape[0] == 0 and mesh.level == 0.0


def test_invalid_values_rejected(ctx):
    f = synth.sphere_frame(seed=3, m=1000, grid=16)
    p, n, w = _frame_dev(f)
    p2 = p.clone()
    p2[17, 1] = float("nan")
    with pytest.raises(fvr.FvrError) as e:
        ctx.reconstruct(p2, n, w, grid_dim=f.dims, bbox=f.bbox)
    assert e.value.status == -1
    w2 = w.clone()
    w2[3] = -1.0
    with pytest.raises(fvr.FvrError) as e:
        ctx.reconstruct(p, n, w2, grid_dim=f.dims, bbox=f.bbox)
    assert e.value.status == -1
    with pytest.raises(fvr.FvrError) as e:
        ctx.reconstruct(p, n, w, grid_dim=(14, 16, 16), bbox=f.bbox)
    assert e.value.status == -2
    # the context still works afterwards
    mesh = ctx.reconstruct(p, n, w, grid_dim=f.dims, bbox=f.bbox)
    assert mesh.vertices.shape[0] > 0


def test_capacity_shortfall_reports_counts_then_retry(ctx):
    f = synth.sphere_frame(seed=0, m=20_000, grid=32)
    p, n, w = _frame_dev(f)
    full = ctx.reconstruct(p, n, w, grid_dim=f.dims, bbox=f.bbox)
    small = (torch.empty((8, 3), dtype=torch.float32, device="cuda"),
             torch.full((8, 3), -7, dtype=torch.int32, device="cuda"))
    with pytest.raises(fvr.FvrError) as e:
        ctx.reconstruct(p, n, w, grid_dim=f.dims, bbox=f.bbox, out=small)
    assert e.value.status == -4
    # the triangle array is not written on a shortfall
    assert bool((small[1] == -7).all())
    retried = ctx.reconstruct(p, n, w, grid_dim=f.dims, bbox=f.bbox, vertex_capacity=8,
                              triangle_capacity=8)
    assert torch.equal(retried.vertices, full.vertices)
    assert torch.equal(retried.triangles, full.triangles)


@pytest.mark.parametrize("dims", [(512, 16, 16), (16, 512, 16), (16, 16, 512)])
def test_maximum_axis_length(ctx, dims):
    print(f"[max axis] {dims}", flush=True)
    bbox = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    f = _random_frame(21, 20000, dims, bbox)
    A, L = ctx.indicator(*_frame_dev(f), grid_dim=dims, bbox=bbox)
    Vo, _, _, _ = oracle.splat(f.points, f.normals, f.weights, dims, bbox)
    Ao = oracle.indicator(Vo, dims, bbox)
    rng_ = Ao.max() - Ao.min()
    err = np.abs(A.cpu().numpy() - Ao).max()
    print(f"  rel err={err / rng_:.3g}")
    assert err <= 1e-4 * rng_


def test_open_surface_flag(ctx):
    f = synth.sphere_frame(seed=4, m=30_000, grid=32, half_extent=0.7)
    mesh = ctx.reconstruct(*_frame_dev(f), grid_dim=f.dims, bbox=f.bbox)
    r = oracle.reconstruct(f.points, f.normals, f.weights, f.dims, f.bbox)
    assert mesh.n_rejected == r["n_rejected"] > 0
    assert mesh.open_surface == r["open_surface"]
    g = synth.sphere_frame(seed=4, m=30_000, grid=32)
    assert not ctx.reconstruct(*_frame_dev(g), grid_dim=g.dims, bbox=g.bbox).open_surface
