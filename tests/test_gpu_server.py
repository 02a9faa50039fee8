"""The serving loop with continuous batching: each request's mesh equals the
single-frame reconstruction of the same frame bit for bit, alone or in a
mix of grids and splats running side by side; admission within a
device-memory budget; refusal and capacity shortfall per request."""
import time

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


@pytest.fixture(scope="module")
def mix():
    cap = synth.config_frame("proxy128")
    frames = [
        (synth.sphere_frame(seed=0, m=50_000, grid=64), "gaussian"),
        (cap, "gaussian"),
        (synth.repose(cap, seed=3), "nearest"),
        (synth.Frame(*[a for a in (synth.repose(cap, seed=4).points, cap.normals, cap.weights)],
                     (192, 192, 192), cap.bbox), "gaussian"),
        (synth.Frame(cap.points, cap.normals, cap.weights, (256, 256, 256), cap.bbox), "gaussian"),
        (synth.sphere_frame(seed=2, m=20_000, grid=32), "nearest"),
    ]
    return frames


def _reference(ctx, f, splat, storage="f32"):
    d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (f.points, f.normals, f.weights)]
    m = ctx.reconstruct(*d, grid_dim=f.dims, bbox=f.bbox, splat=splat, vertex_normals=True, storage=storage)
    return m.vertices.cpu().numpy(), m.triangles.cpu().numpy(), m.normals.cpu().numpy(), m.level


def _check(res, ref):
    assert res["status"] == 0, res["error"]
    v, t, n, L = ref
    assert np.array_equal(res["vertices"], v) and np.array_equal(res["triangles"], t)
    assert np.array_equal(res["normals"], n) and res["level"] == L


def test_each_result_equals_its_frame_alone(ctx, mix):
    refs = [_reference(ctx, f, sp) for f, sp in mix]
    srv = fvr.Server(slots=4, hbm_budget=64 << 30)
    tickets = {}
    for rep in range(2):                 # the same frames twice: 12 requests side by side
        for i, (f, sp) in enumerate(mix):
            t = srv.submit(f.points, f.normals, f.weights, f.dims, f.bbox, splat=sp, vertex_normals=True,
                           user=i)
            tickets[t] = i
    results = srv.drain()
    info = srv.info()
    print(f"[server] {len(results)} results, max in flight {info['max_in_flight']}, "
          f"device bytes {info['device_bytes'] / 2**20:.0f} MiB", flush=True)
    assert len(results) == 2 * len(mix) and info["max_in_flight"] >= 2
    for r in results:
        _check(r, refs[r["user"]])
    srv.close()


def test_16bit_storage_requests_among_float32_ones(ctx, mix):
    """Requests with bf16 / fp16 spectra (192^3 on the mixed-radix passes)
    interleaved with float32 ones on the same slots: each equals its frame
    reconstructed alone with the same storage."""
    cases = [(mix[1], "bf16"), (mix[3], "bf16"), (mix[0], "f32"), (mix[4], "fp16"), (mix[3], "f32"),
             (mix[5], "fp16")]
    refs = [_reference(ctx, f, sp, storage) for (f, sp), storage in cases]
    srv = fvr.Server(slots=3, hbm_budget=64 << 30)
    for i, ((f, sp), storage) in enumerate(cases):
        srv.submit(f.points, f.normals, f.weights, f.dims, f.bbox, splat=sp, vertex_normals=True, user=i,
                   storage=storage)
    results = srv.drain()
    assert len(results) == len(cases)
    for r in results:
        _check(r, refs[r["user"]])
    with pytest.raises(ValueError):
        srv.submit(mix[0][0].points, mix[0][0].normals, None, (64, 64, 64), mix[0][0].bbox, storage="fp8")
    srv.close()


def test_pinned_inputs_and_admission_within_a_budget(ctx, mix):
    """Inputs from pinned host tensors (uploaded without staging); a budget
    that holds one 256^3 frame's slot at a time still serves every request,
    and a frame that cannot fit at all is refused."""
    f, sp = mix[4]
    ref = _reference(ctx, f, sp)
    pin = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (f.points, f.normals, f.weights)]
    srv = fvr.Server(slots=3, hbm_budget=64 << 30)
    t = srv.submit(*pin, f.dims, f.bbox, vertex_normals=True)
    r = srv.drain()[0]
    _check(r, ref)
    need = srv.info()["device_bytes"]
    srv.close()
    srv = fvr.Server(slots=3, hbm_budget=int(need * 1.3))
    for _ in range(3):
        srv.submit(*pin, f.dims, f.bbox, vertex_normals=True)
    results = srv.drain()
    info = srv.info()
    print(f"[server] budget {need * 1.3 / 2**20:.0f} MiB: max in flight {info['max_in_flight']}", flush=True)
    assert info["max_in_flight"] == 1 and len(results) == 3
    for r in results:
        _check(r, ref)
    srv.close()
    tiny = fvr.Server(slots=2, hbm_budget=1 << 20)
    tiny.submit(f.points, f.normals, f.weights, f.dims, f.bbox)
    r = tiny.drain()[0]
    assert r["status"] == -3 and "budget" in r["error"]
    tiny.close()


def test_capacity_shortfall_in_one_request(ctx, mix):
    srv = fvr.Server(slots=2)
    f, sp = mix[0]
    srv.submit(f.points, f.normals, f.weights, f.dims, f.bbox, vertex_capacity=10, triangle_capacity=10)
    g, _ = mix[5]
    srv.submit(g.points, g.normals, g.weights, g.dims, g.bbox, splat="nearest")
    res = {r["ticket"]: r for r in srv.drain()}
    bad, good = res[min(res)], res[max(res)]
    ref = _reference(ctx, f, sp)
    assert bad["status"] == -4 and bad["n_vertices"] == len(ref[0]) and bad["n_triangles"] == len(ref[1])
    assert good["status"] == 0 and good["n_vertices"] > 0
    srv.close()


def test_poisson_arrivals_latency(ctx, mix):
    """Three stations at 30 Hz each (exponential inter-arrival times) for two
    seconds: every request served, latency recorded."""
    rng = np.random.default_rng(0)
    arrivals = []
    for st, (f, sp) in enumerate([mix[1], mix[3], mix[4]]):
        t = 0.0
        while True:
            t += rng.exponential(1 / 30)
            if t > 2.0:
                break
            arrivals.append((t, st, f, sp))
    arrivals.sort(key=lambda a: a[0])
    srv = fvr.Server(slots=4)
    results = []
    t0 = time.perf_counter()
    for t, st, f, sp in arrivals:
        while time.perf_counter() - t0 < t:
            results += srv.poll()
        srv.submit(f.points, f.normals, f.weights, f.dims, f.bbox, splat=sp, user=st)
    results += srv.drain()
    lat = np.array([r["latency_ms"] for r in results])
    assert len(results) == len(arrivals) and all(r["status"] == 0 for r in results)
    print(f"[server] {len(results)} requests in 2 s: latency p50 {np.percentile(lat, 50):.2f} ms, "
          f"p99 {np.percentile(lat, 99):.2f} ms", flush=True)
    srv.close()
