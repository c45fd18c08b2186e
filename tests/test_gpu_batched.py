"""GPU tests of the batched form: every view of a batch equals the plain
per-frame path for the same camera, lens and random-number key, bit for bit
(same kernels, same per-(pixel, sample, view) lens samples); the HIP-graph
replay equals the eager batch on every replay; the trace tuning does not
change results."""
import numpy as np
import pytest
import torch

import scenegen as sg
from gpu_common import print_case, upload_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_2210_04981_amd import hdof
    return hdof


@pytest.fixture(scope="module")
def ctx(hd):
    c = hd.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def room(hd, ctx):
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    yield sc
    sc.close()


def _views(hd, n=6, seed=3):
    rng = np.random.default_rng(seed)
    sizes = [(160, 90), (97, 61), (320, 180), (256, 144), (64, 64), (211, 117)]
    out = []
    for v in range(n):
        w, h = sizes[v % len(sizes)]
        cam = sg.look_camera((rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.0), rng.uniform(-10, 10), w, h)
        lens = sg.lens_fnumber(0.05, [1.4, 2.0, 2.8][v % 3], rng.uniform(0.8, 5.0))
        out.append((hd.camera_of(cam), hd.lens_of(lens), 17, 2, v + 5))
    return out


def _plain(hd, ctx, room, cfg, v):
    cam, lens, seed, frame, view = v
    return hd.hdof_frame(ctx, room, cam, None, lens, hd.light_of(cfg.light), hd.frame_params_of(cfg), seed=seed,
                         frame=frame, view=view)


def test_batched_views_equal_plain_frames(hd, ctx, room):
    print_case("batched == plain")
    cfg = sg.config_1080p()
    views = _views(hd)
    outs = hd.hdof_frame_batched(ctx, room, hd.light_of(cfg.light), hd.frame_params_of(cfg), views)
    torch.cuda.synchronize()
    ctx.sync()
    for i, v in enumerate(views):
        ref = _plain(hd, ctx, room, cfg, v)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), f"view {i} differs from the plain frame"


def test_batch_graph_replays_equal_eager(hd, ctx, room):
    print_case("batch graph replay")
    cfg = sg.config_1080p()
    views = _views(hd, n=5, seed=9)
    eager = hd.hdof_frame_batched(ctx, room, hd.light_of(cfg.light), hd.frame_params_of(cfg), views)
    torch.cuda.synchronize()
    eager = [o.clone() for o in eager]
    outs = [torch.full_like(o, -1.0) for o in eager]
    b = hd.Batch(ctx, room, hd.light_of(cfg.light), hd.frame_params_of(cfg), views, outs)
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        b.launch()
        torch.cuda.synchronize()
        for i in range(len(views)):
            assert torch.equal(outs[i], eager[i]), f"replay {rep}, view {i}"
        # eager work in between replays
        _plain(hd, ctx, room, cfg, views[rep])
        torch.cuda.synchronize()
    b.close()


def test_tuning_does_not_change_results(hd, ctx, room):
    print_case("tuning invariance")
    cfg = sg.config_1080p(256, 144)
    v = (hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), 0, 0, 0)
    base = _plain(hd, ctx, room, cfg, v).clone()
    for t in [dict(blocks_per_cu=1, refill=64, segments=1), dict(blocks_per_cu=4, refill=16, segments=3),
              dict(blocks_per_cu=32, refill=1, segments=8), dict(blocks_per_cu=10, segments=8, wave=1),
              dict(blocks_per_cu=2, segments=5, wave=1)]:
        hd.hdof_set_tuning(ctx, **t)
        out = _plain(hd, ctx, room, cfg, v)
        torch.cuda.synchronize()
        assert torch.equal(out, base), t
    hd.hdof_set_tuning(ctx)
    assert hd.hdof_get_tuning(ctx) == dict(blocks_per_cu=10, refill=64, segments=8, wave=2, overlap=1,
                                           overlap_ray_quantum=140000)
