"""GPU parity of the temporal reconstruction of the traced colours (paper,
Reconstruction) against the FP64 oracle: the trace's far positions, and the
reconstruction stage over a moving-camera sequence (the temporal workload's
camera path at 480x270) fed the oracle's G-buffer, counts, traced colours,
far positions and previous history; and its place in hdof_frame.

Bars: history validity identical and colours within 1e-3 outside the
flagged reprojection bands (a rounded coordinate within 1e-5 of a pixel
boundary, a depth ratio within 1e-5 of the 1 % bound, an ambiguous ray in
the pixel or in the neighbours its far position comes from)."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from gpu_common import f32, print_case, to_dev, upload_scene

pytestmark = pytest.mark.gpu

COL_TOL = 1e-3


@pytest.fixture(scope="module")
def hd():
    from paper_2210_04981_amd import hdof
    return hdof


@pytest.fixture(scope="module")
def ctx(hd):
    c = hd.Context(0)
    yield c
    c.close()


def test_far_positions_match_oracle(hd, ctx):
    print_case("far positions")
    W, H = 320, 180
    scene, cfg = sg.living_room_scene(0), sg.config_1080p(W, H)
    osc = oracle.Scene(scene.verts, scene.albedo)
    rng = np.random.default_rng(5)
    spp = rng.integers(0, 5, (H, W)).astype(np.int32)
    ref = oracle.trace(osc, cfg.camera, cfg.lens, cfg.light, spp, seed=3, frame=1, per_ray=False)
    sc = upload_scene(hd, ctx, scene)
    offs = np.concatenate([[0], np.cumsum(spp.reshape(-1))[:-1]]).astype(np.int32)
    fp = torch.zeros(4, H, W, device="cuda")
    hd.hdof_trace_thin_lens(ctx, sc, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light), 4,
                            to_dev(spp.astype(np.uint8)), to_dev(offs), to_dev(np.array([spp.sum()], np.int32)),
                            seed=3, frame=1, far_pos=fp)
    torch.cuda.synchronize()
    ctx.sync()
    g = fp.cpu().numpy().astype(np.float64)
    r = ref["far_pos"]
    ok = ref["px_amb"] == 0
    assert np.max(np.abs(g[3] - r[3])[ok]) < 1e-4
    has = ok & (r[3] > 1e-3)
    assert has.sum() > 1000
    rel = np.abs(g[:3] - r[:3])[:, has] / np.maximum(np.linalg.norm(r[:3], axis=0)[has], 1.0)
    assert rel.max() < 1e-4, rel.max()
    assert np.all(g[:3][:, ~(r[3] > 0) & ok] == 0)
    sc.close()


def test_reconstruction_sequence_matches_oracle(hd, ctx):
    W, H = 480, 270
    scene = sg.living_room_scene(0)
    cfg = sg.config_temporal(W, H)
    cfg.mask.spp_max = 8
    osc = oracle.Scene(scene.verts, scene.albedo)
    hist = oracle.empty_recon_history(H, W)
    prev = None
    rp = hd.ReconParams(1, 0.2)
    used = 0
    for t in range(6):
        print_case(f"reconstruction frame {t}")
        cam = sg.temporal_camera(t, W, H)
        gb = oracle.gbuffer(osc, cam, cfg.lens, cfg.light)
        depth = f32(gb["depth"])
        spp = oracle.mask(depth, f32(gb["normal"]), cfg.mask, None)["spp"]
        rt = oracle.trace(osc, cam, cfg.lens, cfg.light, spp, seed=0, frame=t, per_ray=False)
        ins = {k: f32(rt[k]) for k in ("hit_ratio", "c_near", "c_far", "far_pos")}
        ref = oracle.recon(cam, depth, spp, prev, hist, ins["hit_ratio"], ins["c_near"], ins["c_far"],
                           ins["far_pos"], 0.2, rt["px_amb"])
        # GPU: the oracle's previous history, the oracle's frame inputs
        if prev is not None:
            hd.hdof_recon_history_load(ctx, to_dev(f32(hist["planes"]), torch.float32),
                                       to_dev(hist["valid"].astype(np.uint8)), to_dev(f32(hist["depth"]), torch.float32))
        else:
            hd.hdof_recon_history_reset(ctx)
        rtg = hd.RTResult(to_dev(ins["c_near"], torch.float32), to_dev(ins["c_far"], torch.float32),
                          to_dev(ins["hit_ratio"], torch.float32), torch.zeros(H, W, device="cuda"),
                          torch.zeros(H, W, device="cuda"))
        hd.hdof_rt_reconstruct(ctx, hd.camera_of(cam), hd.camera_of(prev) if prev is not None else None,
                               to_dev(depth, torch.float32), to_dev(spp.astype(np.uint8)),
                               to_dev(ins["far_pos"], torch.float32), rtg, rp)
        gh = hd.hdof_recon_history_save(ctx, H, W)
        torch.cuda.synchronize()
        ok = ref["amb"] == 0
        traced = spp > 0
        assert np.array_equal(gh["valid"].cpu().numpy().astype(np.int32), ref["history"]["valid"])
        for k in ("c_near", "c_far"):
            d = np.abs(getattr(rtg, k).cpu().numpy() - ref[k])
            assert d[:, ok].max(initial=0) < COL_TOL, (t, k, d[:, ok].max())
        hp = gh["planes"].cpu().numpy()
        d = np.abs(hp - ref["history"]["planes"])
        assert d[:, ok & traced].max(initial=0) < COL_TOL, (t, d[:, ok & traced].max())
        assert np.array_equal(gh["depth"].cpu().numpy(), depth.astype(np.float32))
        if t > 0:
            # the history was actually used somewhere (an accumulated hit ratio differs from the current one)
            used += int((np.abs(ref["history"]["planes"][3] - ins["hit_ratio"]) > 1e-6)[traced].sum())
        hist = dict(planes=f32(ref["history"]["planes"]), valid=ref["history"]["valid"],
                    depth=f32(ref["history"]["depth"]))
        prev = cam
    assert used > 1000


def test_frame_with_reconstruction(hd, ctx):
    """hdof_frame with reconstruction on: the first frame (no history)
    leaves the traced colours as they are; over a short camera path the
    frame's kept colours equal hdof_rt_reconstruct applied to the same
    frame's trace; the batched form refuses it."""
    print_case("frame + reconstruction")
    W, H = 320, 180
    scene = sg.living_room_scene(0)
    cfg = sg.config_temporal(W, H)
    cfg.mask.spp_max = 8
    sc = upload_scene(hd, ctx, scene)
    lens, light = hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    on = hd.frame_params_of(cfg)
    on.recon.enable, on.recon.alpha = 1, 0.2
    off = hd.frame_params_of(cfg)
    cams = [hd.camera_of(sg.temporal_camera(t, W, H)) for t in range(3)]
    k_on, k_off = hd.FrameKeep.empty(H, W), hd.FrameKeep.empty(H, W)
    hd.hdof_history_reset(ctx)
    hd.hdof_recon_history_reset(ctx)
    hd.hdof_frame(ctx, sc, cams[0], None, lens, light, off, frame=0, keep=k_off)
    hd.hdof_frame(ctx, sc, cams[0], None, lens, light, on, frame=0, keep=k_on)
    torch.cuda.synchronize()
    for k in ("c_near", "c_far"):
        a, b = getattr(k_on.rt, k), getattr(k_off.rt, k)
        assert torch.allclose(a, b, rtol=1e-6, atol=1e-6), k
    # frames 1, 2: manual chain (trace with far positions, then reconstruct) on a second context
    ctx2 = hd.Context(0)
    try:
        sc2 = upload_scene(hd, ctx2, scene)
        fp = torch.zeros(4, H, W, device="cuda")
        rp = hd.ReconParams(1, 0.2)
        for t in range(3):
            prev = cams[t - 1] if t else None
            if t:
                hd.hdof_frame(ctx, sc, cams[t], prev, lens, light, on, frame=t, keep=k_on)
            k = hd.FrameKeep.empty(H, W)
            hd.hdof_frame(ctx2, sc2, cams[t], prev, lens, light, off, frame=t, keep=k)
            hd.hdof_trace_thin_lens(ctx2, sc2, cams[t], lens, light, cfg.mask.spp_max, k.spp, k.offsets, k.total,
                                    seed=cfg.seed, frame=t, out=k.rt, far_pos=fp)
            hd.hdof_rt_reconstruct(ctx2, cams[t], prev, k.gb.depth, k.spp, fp, k.rt, rp)
            torch.cuda.synchronize()
            if t:
                for name in ("c_near", "c_far"):
                    assert torch.equal(getattr(k_on.rt, name), getattr(k.rt, name)), (t, name)
        sc2.close()
    finally:
        ctx2.close()
    views = [(cams[0], lens, 0, 0, 0)]
    with pytest.raises(hd.HdofError):
        hd.hdof_frame_batched(ctx, sc, light, on, views, [torch.empty(3, H, W, device="cuda")])
    sc.close()
