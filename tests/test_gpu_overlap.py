"""The overlapped frame (the post-filter gather on the context's second
stream beside the mask, trace and reconstruction; the composite after both)
against the single-stream frame: bitwise equal kept planes and outputs, for
16- and 8-pixel tiles, the specular rule, and temporal plus spatial
reconstruction along a camera path; the stage profile of an overlapped
frame times the gather on its own stream; an overlapped frame captured into
a HIP graph replays to the eager result; under capture a frame refuses a
history and its replays leave the context's history unchanged."""
import ctypes

import numpy as np
import pytest
import torch

import scenegen as sg
from gpu_common import DEV, history_numpy, print_case, to_dev, upload_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    from paper_2210_04981_amd import hdof
    return hdof


@pytest.fixture(scope="module")
def ctx(hd):
    c = hd.Context(0)
    yield c
    hd.hdof_set_tuning(c)
    c.close()


def _run(hd, ctx, sc, cfg, params, cams, lens, light, spec_y, ovl):
    """Frames along cams, single stream (ovl 0) or overlapped with ray
    quantum ovl; (out, kept planes) per frame."""
    hd.hdof_set_tuning(ctx, overlap=int(ovl > 0), overlap_ray_quantum=max(ovl, 1))
    hd.hdof_history_reset(ctx)
    hd.hdof_recon_history_reset(ctx)
    H, W = cfg.camera.height, cfg.camera.width
    res = []
    for t, cam in enumerate(cams):
        k = hd.FrameKeep.empty(H, W)
        if spec_y > 0:
            k.gb = hd.GBuffer.empty(H, W, spec=True)
        k.pp = torch.empty(3, H, W, device=DEV)
        out = torch.empty(3, H, W, device=DEV)
        hd.hdof_frame(ctx, sc, cam, cams[t - 1] if t else None, lens, light, params, frame=t, out=out, keep=k)
        res.append((out, k))
    torch.cuda.synchronize()
    ctx.sync()
    return res


def _same(hd, ctx, cfg, params, lens, a, b, ovl_b):
    """Frames a (single stream) and b (overlapped with ray quantum ovl_b):
    every kept plane and the output bitwise equal (the 16-pixel gather's
    fused composite and the separate composite kernel round alike), and b's
    output bitwise equal to the separate composite of its kept planes."""
    cam = hd.camera_of(cfg.camera)
    for t, ((oa, ka), (ob, kb)) in enumerate(zip(a, b)):
        for name in ("c_near", "c_far", "hit_ratio", "lum_m1", "lum_m2"):
            assert torch.equal(getattr(ka.rt, name), getattr(kb.rt, name)), (t, name)
        assert torch.equal(ka.spp, kb.spp) and torch.equal(ka.gb.color, kb.gb.color)
        assert torch.equal(ka.pp, kb.pp), t
        pps = None
        if params.comp.spec_y > 0:
            _, pps = hd.hdof_postfilter_specular(ctx, kb.gb.color, kb.gb.depth, kb.gb.spec, kb.spp, cam, lens,
                                                 params.pp)
        comp = hd.hdof_composite(ctx, kb.gb.color, kb.pp, kb.gb.depth, kb.spp, kb.rt, cam, lens, params.comp,
                                 pp_spec=pps)
        torch.cuda.synchronize()
        assert torch.equal(ob, comp), (t, ovl_b)
        assert torch.equal(oa, ob), (t, ovl_b, (oa - ob).abs().max().item())


@pytest.mark.parametrize("tile,spec_y", [(16, 0.0), (8, 0.0), (16, 0.3), (8, 0.3)])
def test_overlapped_frame_equals_single_stream(hd, ctx, tile, spec_y):
    print_case(f"overlap tile {tile} spec_y {spec_y}")
    W, H = 320, 180
    glossy = spec_y > 0
    scene = sg.glossy_living_room_scene(0) if glossy else sg.living_room_scene(0)
    cfg = sg.config_1080p(W, H)
    cfg.pp.tile = tile
    sc = upload_scene(hd, ctx, scene)
    if glossy:
        hd.hdof_scene_set_specular(sc, to_dev(scene.spec))
    params = hd.frame_params_of(cfg)
    params.comp.spec_y = spec_y
    cams = [hd.camera_of(cfg.camera)]
    lens, light = hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    ref = _run(hd, ctx, sc, cfg, params, cams, lens, light, spec_y, 0)
    for ovl in (140000, 1, 10 ** 9, 20000):  # default, all blocks, one per CU, in between
        _same(hd, ctx, cfg, params, lens, ref, _run(hd, ctx, sc, cfg, params, cams, lens, light, spec_y, ovl), ovl)
    assert (ref[0][0] - ref[0][1].gb.color).abs().max().item() > 0.05  # depth of field changed the image
    sc.close()


def test_overlapped_frame_with_reconstruction(hd, ctx):
    """Temporal and spatial reconstruction over four frames of a camera
    path: the overlapped frames equal the single-stream ones."""
    print_case("overlap temporal+spatial")
    W, H = 320, 180
    cfg = sg.config_temporal(W, H)
    cfg.mask.spp_max = 8
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    params = hd.frame_params_of(cfg)
    params.spatial.enable, params.spatial.n_taps, params.spatial.r_cap, params.spatial.v_clamp = 1, 24, 64.0, 0.01
    params.recon.enable, params.recon.alpha = 1, 0.2
    cams = [hd.camera_of(sg.temporal_camera(t, W, H)) for t in range(4)]
    lens, light = hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    ref = _run(hd, ctx, sc, cfg, params, cams, lens, light, 0.0, 0)
    b = _run(hd, ctx, sc, cfg, params, cams, lens, light, 0.0, 140000)
    for t, ((oa, ka), (ob, kb)) in enumerate(zip(ref, b)):
        for name in ("c_near", "c_far", "hit_ratio"):
            assert torch.equal(getattr(ka.rt, name), getattr(kb.rt, name)), (t, name)
        assert torch.equal(ka.pp, kb.pp), t
        assert torch.equal(oa, ob), (t, (oa - ob).abs().max().item())
    sc.close()


def test_overlapped_frame_profile(hd, ctx):
    """Profiled overlapped frames: every stage that ran has a positive
    duration, the gather's is its own stream's, and the frame's stream
    stages (all but the gather) fit in the frame."""
    print_case("overlap profile")
    W, H = 640, 360
    cfg = sg.config_1080p(W, H)
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    params = hd.frame_params_of(cfg)
    cam, lens, light = hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    out = torch.empty(3, H, W, device=DEV)
    hd.hdof_set_tuning(ctx)  # overlapped by default
    assert hd.hdof_get_tuning(ctx)["overlap"] == 1
    hd.hdof_history_reset(ctx)
    for _ in range(2):
        hd.hdof_frame(ctx, sc, cam, None, lens, light, params, out=out)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    hd.hdof_profile_begin(ctx)
    a.record()
    for _ in range(5):
        hd.hdof_frame(ctx, sc, cam, None, lens, light, params, out=out)
    b.record()
    st, n = hd.hdof_profile_end(ctx)
    torch.cuda.synchronize()
    frame_ms = a.elapsed_time(b) / 5
    assert n == 5
    assert all(v >= 0 for v in st.values()), st
    for k in ("gbuffer", "ray_mask", "trace", "rt_reduce", "pp_gather", "composite"):
        assert st[k] > 0, (k, st)
    main = sum(v for k, v in st.items() if k != "pp_gather")
    assert main <= frame_ms * 1.05 + 0.01, (main, frame_ms, st)
    assert st["pp_gather"] <= frame_ms * 1.05 + 0.01, (st["pp_gather"], frame_ms)
    hd.hdof_set_tuning(ctx)
    sc.close()


def test_overlapped_frame_in_a_graph(hd, ctx):
    """A frame captured into a HIP graph (torch.cuda.graph) with the overlap
    on: the fork to the context's second stream and the join are captured
    with it.  Three replays, with other eager frames and synchronisations
    between them, each equal the eager frame bitwise."""
    print_case("overlap graph capture")
    W, H = 320, 180
    cfg = sg.config_1080p(W, H)
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    params = hd.frame_params_of(cfg)
    cam, lens, light = hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    other = hd.camera_of(sg.temporal_camera(5, W, H))
    hd.hdof_set_tuning(ctx)
    assert hd.hdof_get_tuning(ctx)["overlap"] == 1
    out_e = torch.empty(3, H, W, device=DEV)
    out_g = torch.empty(3, H, W, device=DEV)
    hd.hdof_frame(ctx, sc, cam, None, lens, light, params, frame=0, out=out_e)
    hd.hdof_frame(ctx, sc, cam, None, lens, light, params, frame=0, out=out_g)  # every buffer in place
    torch.cuda.synchronize()
    ctx.sync()
    assert torch.equal(out_e, out_g)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.graph(g, stream=s):
        hd.hdof_frame(ctx, sc, cam, None, lens, light, params, frame=0, out=out_g)
    scratch = torch.empty(3, H, W, device=DEV)
    for rep in range(3):
        out_g.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_g, out_e), rep
        hd.hdof_frame(ctx, sc, other, None, lens, light, params, frame=rep + 1, out=scratch)
        torch.cuda.synchronize()
        assert not torch.equal(scratch, out_e)
    ctx.sync()
    del g
    sc.close()


def test_captured_frame_refuses_history_and_keeps_it(hd, ctx):
    """Under stream capture a frame with a previous camera (or a
    reconstruction stage) is refused before anything is recorded; a
    captured frame without one replays without touching the context's
    variance history: after eager frames, replays and another eager frame
    with a previous camera, outputs and history equal those of the same
    eager frames without the replays."""
    print_case("captured frame and the variance history")
    W, H = 320, 180
    cfg = sg.config_temporal(W, H)
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    params = hd.frame_params_of(cfg)
    lens, light = hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    cams = [hd.camera_of(sg.temporal_camera(t, W, H)) for t in range(3)]
    hd.hdof_set_tuning(ctx)
    out = torch.empty(3, H, W, device=DEV)
    hd.hdof_history_reset(ctx)
    hd.hdof_frame(ctx, sc, cams[0], None, lens, light, params, frame=0, out=out)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    rec = hd.frame_params_of(cfg)
    rec.recon.enable = 1
    hip = hd._lib  # its HIP runtime dependency, the one torch loaded
    for p_, prev in ((params, cams[0]), (rec, None)):
        graph = ctypes.c_void_p()
        assert hip.hipStreamBeginCapture(ctypes.c_void_p(s.cuda_stream), 2) == 0  # relaxed mode
        try:
            with pytest.raises(hd.HdofError):
                hd.hdof_frame(ctx, sc, cams[1], prev, lens, light, p_, frame=1, out=out, stream=s)
        finally:
            assert hip.hipStreamEndCapture(ctypes.c_void_p(s.cuda_stream), ctypes.byref(graph)) == 0
            if graph.value:
                hip.hipGraphDestroy(graph)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        hd.hdof_frame(ctx, sc, cams[2], None, lens, light, params, frame=7, out=out)
    try:
        _replays_between_frames(hd, ctx, sc, g, cams, lens, light, params, H, W)
    finally:
        torch.cuda.synchronize()
        del g
    ctx.sync()
    sc.close()


def _replays_between_frames(hd, ctx, sc, g, cams, lens, light, params, H, W):
    res = {}
    for replays in (0, 2):
        hd.hdof_history_reset(ctx)
        o = []
        for t in range(3):
            ot = torch.empty(3, H, W, device=DEV)
            hd.hdof_frame(ctx, sc, cams[t], cams[t - 1] if t else None, lens, light, params, frame=t, out=ot)
            torch.cuda.synchronize()
            for _ in range(replays):
                g.replay()
                torch.cuda.synchronize()
            o.append(ot)
        h = hd.hdof_history_save(ctx, H, W)
        torch.cuda.synchronize()
        res[replays] = (o, h)
    for t in range(3):
        assert torch.equal(res[0][0][t], res[2][0][t]), t
    for k in ("lum_m1", "lum_m2", "flags", "depth"):
        assert torch.equal(res[0][1][k], res[2][1][k]), k


@pytest.mark.parametrize("overlap", [1, 0])
def test_frame_without_kept_planes(hd, ctx, overlap):
    """Without kept trace planes (and no reconstruction) the reduction
    writes the trace planes only at traced pixels; the frame's output and
    its variance history are the same as with every plane kept, over frames
    that carry the history."""
    print_case(f"frame without kept planes, overlap {overlap}")
    W, H = 320, 180
    cfg = sg.config_1080p(W, H)
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    params = hd.frame_params_of(cfg)
    lens, light = hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    cams = [hd.camera_of(sg.temporal_camera(t, W, H)) for t in range(3)]
    hd.hdof_set_tuning(ctx, overlap=overlap)
    outs, hists = {}, {}
    for kept in (True, False):
        hd.hdof_history_reset(ctx)
        res = []
        for t, cam in enumerate(cams):
            out = torch.empty(3, H, W, device=DEV)
            k = hd.FrameKeep.empty(H, W) if kept else None
            hd.hdof_frame(ctx, sc, cam, cams[t - 1] if t else None, lens, light, params, frame=t, out=out, keep=k)
            res.append(out)
        torch.cuda.synchronize()
        ctx.sync()
        outs[kept] = res
        hists[kept] = history_numpy(hd, ctx, H, W)
    for t in range(len(cams)):
        assert torch.equal(outs[True][t], outs[False][t]), t
    for name in ("lum_m1", "lum_m2", "flags", "depth"):
        assert np.array_equal(hists[True][name], hists[False][name]), name
    hd.hdof_set_tuning(ctx)
    sc.close()


def test_overlapped_frames_alternating_cameras(hd, ctx):
    """1080p overlapped frames that alternate between two cameras, enqueued
    back to back: the gather on the second stream must wait for its own
    frame's G-buffer (a gather that started early would read the previous
    frame's packed texels, another camera's) and the composite for its own
    gather.  Each frame equals the single-stream frame of its camera bit
    for bit."""
    print_case("overlapped frames alternating cameras")
    cfg = sg.config_1080p()
    W, H = cfg.camera.width, cfg.camera.height
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    params = hd.frame_params_of(cfg)
    lens, light = hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    cams = [hd.camera_of(cfg.camera), hd.camera_of(sg.temporal_camera(30, W, H))]
    hd.hdof_set_tuning(ctx, overlap=0)
    refs = [hd.hdof_frame(ctx, sc, c, None, lens, light, params, frame=0) for c in cams]
    torch.cuda.synchronize()
    assert not torch.equal(refs[0], refs[1])
    hd.hdof_set_tuning(ctx)
    outs = [torch.empty(3, H, W, device=DEV) for _ in range(6)]
    for i, o in enumerate(outs):
        hd.hdof_frame(ctx, sc, cams[i % 2], None, lens, light, params, frame=0, out=o)
    torch.cuda.synchronize()
    ctx.sync()
    for i, o in enumerate(outs):
        assert torch.equal(o, refs[i % 2]), i
    sc.close()
