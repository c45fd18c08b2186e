"""GPU tests of the batched form: four views of the batched workload (one
at each of its resolutions, with their own focus, f-number, eye and yaw)
run as one batch and are compared with the oracle's frame at each view's
own camera, lens, seed, frame and view index; every view of a batch equals
the plain per-frame path for the same camera, lens and random-number key,
bit for bit (same kernels, same per-(pixel, sample, view) lens samples);
the HIP-graph replay equals the eager batch on every replay; the trace
tuning does not change results."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from gpu_common import compare_frame, print_case, run_frame, upload_scene

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


def test_batched_views_match_oracle(hd, ctx, room):
    """The batch's outputs are compared with oracle.frame at every pixel
    where the G-buffer, the counts and the rays agree (the plain frame of
    the same view, with its intermediates kept, decides where that is and
    must equal the batch's output bit for bit)."""
    cfgs = sg.batched_views(seed=7)
    # 2560x1440 f/1.4 at 1.97 m, 1280x720 f/2.8 at 0.82 m, 1920x1080 f/2 at
    # 4.98 m, 640x360 f/2.8 at 1.18 m: every resolution and f-number, focus
    # across the range
    picked = [(v, cfgs[v]) for v in (2, 1, 3, 9)]
    assert len({(c.camera.width, c.camera.height) for _, c in picked}) == 4
    assert len({c.lens.aperture for _, c in picked}) == 3
    frame_index = 3
    views = [(hd.camera_of(c.camera), hd.lens_of(c.lens), c.seed, frame_index, v) for v, c in picked]
    hd.hdof_set_tuning(ctx)
    outs = hd.hdof_frame_batched(ctx, room, hd.light_of(picked[0][1].light), hd.frame_params_of(picked[0][1]), views)
    torch.cuda.synchronize()
    ctx.sync()
    scene = sg.living_room_scene(0)
    osc = oracle.Scene(scene.verts, scene.albedo)
    for (v, c), o in zip(picked, outs):
        print_case(f"batched view {v} {c.camera.width}x{c.camera.height} N={0.05 / c.lens.aperture:.1f} "
                   f"S1={c.lens.focus_distance:.2f}")
        g = run_frame(hd, ctx, room, c, frame=frame_index, view=v)
        bo = o.cpu().numpy().astype(np.float64)
        assert np.array_equal(bo, g["out"]), f"view {v}: batch differs from its plain frame"
        ref = oracle.frame(osc, c, frame_index=frame_index, view=v)
        g["out"] = bo
        info = compare_frame(g, ref, c)
        print(v, info, flush=True)
        assert info["compared"] >= 0.85, (v, info)
        assert info["traced"] > 0


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
    assert hd.hdof_get_tuning(ctx) == dict(blocks_per_cu=10, refill=64, segments=8, wave=0, overlap=1,
                                           overlap_ray_quantum=140000)


def _odd_views(hd, sizes, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for v in range(n):
        w, h = sizes[v % len(sizes)]
        cam = sg.look_camera((rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2), 0.0), rng.uniform(-10, 10), w, h)
        lens = sg.lens_fnumber(0.05, [1.4, 2.0, 2.8][v % 3], rng.uniform(0.8, 5.0))
        out.append((hd.camera_of(cam), hd.lens_of(lens), 23, 4, v))
    return out


@pytest.mark.parametrize("n", [1, 2, 11, 64])
def test_batched_ragged_views_equal_plain_frames(hd, ctx, room, n):
    """Views whose 16-pixel tile counts are not multiples of four (so a
    quad-gather block's tiles straddle two views), a 1x1 view, views far
    below one 4096-pixel block of the per-pixel passes, the largest batch
    (64 views: every step of the block-to-view search), and batches of one
    and two views (no split of the G-buffer launches, one view per chunk):
    each view equals its plain frame bit for bit."""
    sizes = [(33, 17), (1, 1), (17, 33), (50, 3), (129, 65), (7, 300), (65, 65), (31, 47)]
    if n == 64:
        sizes = [(24, 16), (33, 17), (16, 16), (17, 9), (9, 9)]
    print_case(f"{n} ragged batched views")
    cfg = sg.config_1080p()
    views = _odd_views(hd, sizes, n, seed=n)
    tiles = [((v[0].width + 15) // 16) * ((v[0].height + 15) // 16) for v in views]
    assert any(t % 4 for t in tiles) and sum(tiles) % 4
    outs = hd.hdof_frame_batched(ctx, room, hd.light_of(cfg.light), hd.frame_params_of(cfg), views)
    torch.cuda.synchronize()
    ctx.sync()
    for i, v in enumerate(views):
        ref = _plain(hd, ctx, room, cfg, v)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), f"view {i} ({v[0].width}x{v[0].height}) differs from the plain frame"


@pytest.mark.parametrize("tile", [0, 4])
def test_batched_mask_tiles_equal_plain_frames(hd, ctx, room, tile):
    """The batch with another mask tile: 4-pixel tiles (the single-launch
    masks) and the CoC-scaled tile (per-view masks); each view equals its
    plain frame bit for bit."""
    from dataclasses import replace
    print_case(f"batched views, mask tile {tile}")
    cfg = sg.config_1080p()
    cfg = replace(cfg, mask=replace(cfg.mask, tile=tile))
    views = _odd_views(hd, [(97, 61), (160, 90), (33, 17)], 5, seed=40 + tile)
    outs = hd.hdof_frame_batched(ctx, room, hd.light_of(cfg.light), hd.frame_params_of(cfg), views)
    torch.cuda.synchronize()
    ctx.sync()
    for i, v in enumerate(views):
        ref = _plain(hd, ctx, room, cfg, v)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), f"view {i} differs from the plain frame (mask tile {tile})"


def test_batched_views_with_nothing_traced(hd, ctx, room):
    """Mask thresholds no edge reaches and no history: no view traces a
    pixel, so the batch's one persistent trace runs on an empty queue; each
    view equals its plain frame bit for bit, and that frame is the
    post-filtered image composited without traced pixels."""
    from dataclasses import replace
    print_case("batched views, nothing traced")
    cfg = sg.config_1080p()
    cfg = replace(cfg, mask=replace(cfg.mask, tau_depth=1e30, tau_normal=1e30))
    views = _odd_views(hd, [(97, 61), (160, 90), (33, 17)], 4, seed=77)
    outs = hd.hdof_frame_batched(ctx, room, hd.light_of(cfg.light), hd.frame_params_of(cfg), views)
    torch.cuda.synchronize()
    ctx.sync()
    for i, v in enumerate(views):
        ref = _plain(hd, ctx, room, cfg, v)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), f"view {i} differs from the plain frame (nothing traced)"
