"""Batched reconstruction (16 frames of uneven grids and point counts as one
captured HIP graph) against the single-frame path: every frame's mesh,
level and flags bit-identical to its own fvr_reconstruct call."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1712_03084_amd as fvr  # noqa: E402

_CACHE = {}


def _frames():
    if "frames" not in _CACHE:
        print("[batch] generating 16 frames of the batched workload", flush=True)
        _CACHE["frames"], _ = synth.batch_frames(16, seed=4000)
    return _CACHE["frames"]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fvr.Context(0)


def _dev(f):
    d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (f.points, f.normals, f.weights)]
    return (d[0], d[1], d[2], f.dims, f.bbox)


def _outs(n, vcap=300_000):
    return [(torch.full((vcap, 3), -1.0, device="cuda"),
             torch.full((2 * vcap, 3), -1, dtype=torch.int32, device="cuda")) for _ in range(n)]


def _same(a, b):
    assert torch.equal(a.vertices, b.vertices)
    assert torch.equal(a.triangles, b.triangles)
    assert a.level == b.level and a.open_surface == b.open_surface and a.n_rejected == b.n_rejected


@pytest.fixture(scope="module")
def reference(ctx):
    frames = _frames()
    devs = [_dev(f) for f in frames]
    refs = []
    for f, d in zip(frames, devs):
        m = ctx.reconstruct(d[0], d[1], d[2], grid_dim=f.dims, bbox=f.bbox)
        refs.append(fvr.Mesh(m.vertices.clone(), m.triangles.clone(), m.level, m.n_rejected,
                             m.open_surface))
    return frames, devs, refs


@pytest.mark.parametrize("slots,graph", [(4, True), (4, False), (1, True), (16, True)])
def test_batch_equals_single_frames(reference, slots, graph):
    frames, devs, refs = reference
    print(f"[batch] slots={slots} graph={graph}: grids "
          f"{[f.dims[0] for f in frames]}", flush=True)
    b = fvr.Batch(slots=slots, graph=graph)
    outs = _outs(len(frames))
    meshes = b.reconstruct(devs, outs)
    for i, (got, ref) in enumerate(zip(meshes, refs)):
        assert got.vertices.shape[0] > 0, i
        _same(got, ref)
    b.close()


def test_graph_replays_with_eager_work_between(ctx, reference):
    """The captured graph is launched again and again; the program's own
    eager work and synchronisations run between the replays, and every
    replay's results are checked."""
    frames, devs, refs = reference
    b = fvr.Batch(slots=4, graph=True)
    outs = _outs(len(frames))
    pb = b.prepare(devs, outs)
    for rep in range(3):
        print(f"[batch] replay {rep}", flush=True)
        for o in outs:
            o[0].fill_(-1.0)
            o[1].fill_(-1)
        pb.run()
        for got, ref in zip(pb.meshes(), refs):
            _same(got, ref)
        # eager work between replays: a single-frame call and a torch op
        d = devs[rep]
        ctx.reconstruct(d[0], d[1], d[2], grid_dim=frames[rep].dims, bbox=frames[rep].bbox)
        torch.cuda.synchronize()
    b.close()


def test_batch_capacity_shortfall_in_one_frame(reference):
    frames, devs, refs = reference
    b = fvr.Batch(slots=4)
    outs = _outs(len(frames))
    outs[5] = (torch.empty((10, 3), device="cuda"), torch.full((10, 3), -7, dtype=torch.int32, device="cuda"))
    pb = b.prepare(devs, outs)
    with pytest.raises(fvr.FvrError) as e:
        pb.run()
    assert e.value.status == -4
    counts = [(m.n_vertices, m.n_triangles) for m in pb._meshes[:len(frames)]]
    assert counts[5] == (refs[5].vertices.shape[0], refs[5].triangles.shape[0])
    assert bool((outs[5][1] == -7).all())
    for i, (got, ref) in enumerate(zip(pb.meshes(), refs)):
        if i != 5:
            _same(got, ref)
    b.close()


def test_tuned_plans_keep_parity_and_batch_equality(ctx):
    """Non-default radix orders and splat tiles (what the autotuner may pick)
    keep the indicator within the parity bar against the oracle, and the
    batch still equals the single-frame path bit for bit."""
    import oracle
    from paper_1712_03084_amd import autotune as at
    frames = _frames()[:6]
    shapes = sorted({f.dims for f in frames})
    try:
        for d in shapes:
            base = at.get_tuning(d)
            cand = at.candidates(d)
            trial = {"radices": [c[-1] for c in cand["radices"]], "splat_tile": cand["splat_tile"][0]}
            print(f"[tuned] {d}: {base} -> {trial}", flush=True)
            at.set_tuning(d, trial)
        f = frames[0]
        d = _dev(f)
        A, L = ctx.indicator(d[0], d[1], d[2], grid_dim=f.dims, bbox=f.bbox)
        Vo, _, _, _ = oracle.splat(f.points, f.normals, f.weights, f.dims, f.bbox)
        Ao = oracle.indicator(Vo, f.dims, f.bbox)
        rng_ = Ao.max() - Ao.min()
        err = float(np.abs(A.cpu().numpy() - Ao).max())
        print(f"[tuned] {f.dims} A rel err {err / rng_:.3g}", flush=True)
        assert err <= 1e-4 * rng_
        devs = [_dev(g) for g in frames]
        refs = [ctx.reconstruct(x[0], x[1], x[2], grid_dim=g.dims, bbox=g.bbox) for x, g in zip(devs, frames)]
        refs = [fvr.Mesh(m.vertices.clone(), m.triangles.clone(), m.level, m.n_rejected, m.open_surface)
                for m in refs]
        b = fvr.Batch(slots=3)
        for got, ref in zip(b.reconstruct(devs, _outs(len(frames))), refs):
            _same(got, ref)
        b.close()
    finally:
        for d in shapes:
            at.set_tuning(d, None)


def test_autotuner_search_and_cache(ctx, tmp_path):
    """The autotuner times candidates on a frame, keeps the fastest (never
    slower than the default it measured), writes the JSON cache, and load()
    applies it again."""
    from paper_1712_03084_amd import autotune as at
    f = [g for g in _frames() if g.dims[0] == 96][0]
    d = _dev(f)
    try:
        res = at.tune(ctx, d[0], d[1], d[2], f.dims, f.bbox, reps=5)
        print(f"[autotune] {f.dims}: {res}", flush=True)
        assert res["us"] <= res["default_us"] and res["tried"] > 10
        path = at.save_entry(f.dims, res, path=str(tmp_path / "tune.json"))
        at.set_tuning(f.dims, None)
        assert at.load(path) == 1
        assert at.get_tuning(f.dims) == res["params"]
    finally:
        at.set_tuning(f.dims, None)
