"""Serving form: continuous batching of mixed-resolution renders against a device-resident scene.
Each request's result must be identical alone and in the mix; admission never exceeds the arena;
an intersection overflow is re-admitted; a request larger than the arena is rejected, not stuck."""
import numpy as np
import pytest

import oracle
from paper_2411_00771_amd import scenes
from tests.helpers import FRAGILE

pytestmark = pytest.mark.gpu

RES = [(160, 120), (320, 180), (480, 270), (96, 64)]


@pytest.fixture(scope="module")
def city(cuda):
    from paper_2411_00771_amd import raster
    c = scenes.make_city(11, L=300.0, n_boxes=20)
    sc = scenes.city_scene(11, 60_000, L=300.0, city=c)
    rng = np.random.default_rng(5)
    cams = [scenes.orbit_camera(rng, c, *RES[k % len(RES)], alt=(60.0, 120.0), radius=(0.2, 0.4))
            for k in range(14)]
    return dict(sc=sc, params=raster.Params.from_scene(sc), cams=cams)


def _eq(a, b):
    return all(np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()) for k in ("rgb", "depth", "normal"))


@pytest.mark.parametrize("max_batch", [1, 3])
def test_alone_equals_mix_and_memory_admission(city, max_batch):
    """Mixed-resolution requests through 3 slots (and, with max_batch 3, same-resolution requests batched
    into one call): every result equals the request rendered alone, the budget is never exceeded, and the
    arena is whole again at the end."""
    from paper_2411_00771_amd import server
    srv = server.Server(city["params"], max_slots=3, arena_bytes=(64 if max_batch == 1 else 256) << 20, max_width=480,
                        max_height=270, max_batch=max_batch)
    mix = [srv.submit(c) for c in city["cams"]]
    peak = 0
    while srv.poll():
        peak = max(peak, srv.arena_used)
        assert srv.arena_used <= srv.arena_bytes
        assert sum(s.launch is not None for s in srv.slots) <= 3
    srv.drain()
    assert all(r.done and r.error is None for r in mix)
    assert peak > srv.fixed_bytes
    assert srv.arena.used == 0 and srv.arena.free == [(0, srv.arena.size)]
    if max_batch > 1:
        assert srv.launches < len(mix)
    ref = server.Server(city["params"], max_slots=1, arena_bytes=64 << 20, max_width=480, max_height=270)
    for r in mix:
        alone = ref.render_alone(r.cam)
        assert alone.error is None
        assert _eq(alone.result, r.result), r.rid


def test_overflow_is_readmitted(city):
    from paper_2411_00771_amd import server
    srv = server.Server(city["params"], max_slots=2, arena_bytes=256 << 20, max_width=480, max_height=270,
                        intersections_per_pixel=0.001)
    reqs = [srv.submit(c) for c in city["cams"][:4]]
    srv.drain()
    assert all(r.done and r.error is None for r in reqs)
    assert any(r.tries >= 1 for r in reqs)
    ref = server.Server(city["params"], max_slots=1, arena_bytes=256 << 20, max_width=480, max_height=270)
    for r in reqs:
        assert _eq(ref.render_alone(r.cam).result, r.result)


def test_oversize_request_rejected_not_stuck(city):
    from paper_2411_00771_amd import server
    # a budget that holds the slots' fixed buffers and 1 MiB more: no 480x270 request fits
    fixed = server.fixed_bytes(city["params"].n, max_slots=2, max_width=480, max_height=270)
    srv = server.Server(city["params"], max_slots=2, arena_bytes=fixed + (1 << 20), max_width=480, max_height=270)
    r = srv.submit(city["cams"][2])
    srv.drain()
    assert r.done and r.error is not None
    # a budget that cannot even hold the slots is refused at construction
    with pytest.raises(ValueError):
        server.Server(city["params"], max_slots=2, arena_bytes=fixed // 2, max_width=480, max_height=270)


def test_served_render_matches_oracle(city):
    from paper_2411_00771_amd import server
    cam = city["cams"][3]  # 96 x 64
    srv = server.Server(city["params"], max_slots=1, arena_bytes=64 << 20, max_width=480, max_height=270)
    r = srv.render_alone(cam)
    po, off, ids, io = oracle.forward_view(city["sc"], cam)
    ok = io["margin"] >= FRAGILE
    assert (1 - ok.mean()) <= 5e-3
    assert np.abs(r.result["rgb"].cpu().numpy() - io["rgb"])[:, ok].max() <= 1e-4
    zs = max(1.0, float(np.abs(io["depth"]).max()))
    assert np.abs(r.result["depth"].cpu().numpy() - io["depth"])[ok].max() <= 1e-4 * zs
