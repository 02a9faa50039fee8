"""fvr_reconstruct_noalloc against fvr_reconstruct (same kernels; scratch from
the device's static array instead of the context's own memory): identical
meshes, level and flags, over consecutive calls whose later frames are
smaller (the static scratch keeps the previous call's contents)."""
import numpy as np
import pytest

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
    return _dev(f.points), _dev(f.normals), (None if f.weights is None else _dev(f.weights))


def _out(vcap, tcap):
    return (torch.full((vcap, 3), -1.0, dtype=torch.float32, device="cuda"),
            torch.full((tcap, 3), -1, dtype=torch.int32, device="cuda"))


def _same(a, b):
    assert torch.equal(a.vertices, b.vertices)
    assert torch.equal(a.triangles, b.triangles)
    assert a.level == b.level
    assert a.n_rejected == b.n_rejected and a.open_surface == b.open_surface


FRAMES = [
    ("proxy128 (400k points, 128^3)", lambda: synth.config_frame("proxy128")),
    ("sphere 64^3 (50k points)", lambda: synth.sphere_frame(seed=0, m=50_000, grid=64)),
    ("sphere 256x256x16 slab, cut by the box (fused inverse pass)",
     lambda: synth.Frame(*_slab(), (256, 256, 16), (-1.0, -1.0, -0.0625, 1.0, 1.0, 0.0625))),
    ("sphere 32^3 (5k points)", lambda: synth.sphere_frame(seed=2, m=5_000, grid=32)),
]


def _slab():
    f = synth.sphere_frame(seed=5, m=100_000, grid=64)
    return f.points, f.normals, f.weights


def test_noalloc_matches_reconstruct_over_consecutive_calls(ctx):
    out = _out(200_000, 400_000)
    for name, make in FRAMES:
        print(f"[noalloc] {name}", flush=True)
        f = make()
        dev = _frame_dev(f)
        got = ctx.reconstruct_noalloc(*dev, grid_dim=f.dims, bbox=f.bbox, out=out)
        ref = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox)
        print(f"  V={ref.vertices.shape[0]} T={ref.triangles.shape[0]} L={ref.level:.8g}", flush=True)
        _same(got, ref)
        # and again, after the normal path ran on the context's own memory
        again = ctx.reconstruct_noalloc(*dev, grid_dim=f.dims, bbox=f.bbox, out=out)
        _same(again, ref)


def test_noalloc_with_16bit_spectrum_storage(ctx):
    """The storage option bits pass through: the 16-bit spectra (half the
    bytes) are carved from the same static array."""
    out = _out(200_000, 400_000)
    for name, make, storage in [
            ("proxy128, bf16", lambda: synth.config_frame("proxy128"), "bf16"),
            ("sphere 48^3 (mixed-radix passes), fp16", lambda: synth.sphere_frame(seed=6, m=30_000, grid=48),
             "fp16")]:
        print(f"[noalloc] {name}", flush=True)
        f = make()
        dev = _frame_dev(f)
        got = ctx.reconstruct_noalloc(*dev, grid_dim=f.dims, bbox=f.bbox, out=out, storage=storage)
        ref = ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox, storage=storage)
        _same(got, ref)


def test_noalloc_refuses_a_frame_beyond_the_static_scratch(ctx):
    f = synth.sphere_frame(seed=1, m=20_000, grid=256)
    dev = _frame_dev(f)
    out = _out(1000, 2000)
    print("[noalloc] 256^3 frame: refused", flush=True)
    with pytest.raises(fvr.FvrError) as e:
        ctx.reconstruct_noalloc(*dev, grid_dim=f.dims, bbox=f.bbox, out=out)
    assert e.value.status == -3
    assert "FVR_NOALLOC_SCRATCH_BYTES" in str(e.value)
    # nothing was written and the context still works on both paths
    assert bool((out[1] == -1).all())
    g = synth.sphere_frame(seed=0, m=20_000, grid=32)
    dg = _frame_dev(g)
    _same(ctx.reconstruct_noalloc(*dg, grid_dim=g.dims, bbox=g.bbox, out=_out(20_000, 40_000)),
          ctx.reconstruct(*dg, grid_dim=g.dims, bbox=g.bbox))


def test_noalloc_from_a_second_context_on_the_device(ctx):
    other = fvr.Context(0)
    f = synth.sphere_frame(seed=3, m=30_000, grid=48)
    dev = _frame_dev(f)
    print("[noalloc] second context, 48^3", flush=True)
    _same(other.reconstruct_noalloc(*dev, grid_dim=f.dims, bbox=f.bbox, out=_out(50_000, 100_000)),
          ctx.reconstruct(*dev, grid_dim=f.dims, bbox=f.bbox))
    other.close()
