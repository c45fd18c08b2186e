"""GPU parity of the specular materials and the composite's specular bokeh
rule (paper, Composite) against the FP64 oracle: the G-buffer's colour and
specular luminance with a glossy scene, the traced colours, the
post-filtered specular luminance (16- and 8-pixel tiles, all pixels and
traced pixels only), the composite with the rule, and hdof_frame with it
(fused and separate composite paths) against its stages chained by hand.

Bars as for the Lambertian stages: ids equal outside the oracle's flagged
rays, colours and luminances within 1e-3 where the ids agree (the fp32
Blinn-Phong power of a cosine near 1 amplifies its rounding by the
shininess), filtered values within 1e-3."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from gpu_common import DEV, excl_cumsum, f32, print_case, to_dev, upload_scene

pytestmark = pytest.mark.gpu

TOL = 1e-3


@pytest.fixture(scope="module")
def hd():
    from paper_2210_04981_amd import hdof
    return hdof


@pytest.fixture(scope="module")
def ctx(hd):
    c = hd.Context(0)
    yield c
    c.close()


def _glossy(hd, ctx, W, H):
    scene = sg.glossy_living_room_scene(0)
    cfg = sg.config_1080p(W, H)
    sc = upload_scene(hd, ctx, scene)
    hd.hdof_scene_set_specular(sc, to_dev(scene.spec))
    osc = oracle.Scene(scene.verts, scene.albedo, scene.spec)
    return scene, cfg, sc, osc


def test_gbuffer_specular_matches_oracle(hd, ctx):
    print_case("gbuffer glossy")
    W, H = 320, 180
    scene, cfg, sc, osc = _glossy(hd, ctx, W, H)
    ref = oracle.gbuffer(osc, cfg.camera, cfg.lens, cfg.light)
    gb = hd.hdof_gbuffer(ctx, sc, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light),
                         out=hd.GBuffer.empty(H, W, spec=True))
    torch.cuda.synchronize()
    ctx.sync()
    ids, amb = gb.tri_id.cpu().numpy(), ref["amb"] != 0
    assert not ((ids != ref["tri_id"]) & ~amb).any()
    same = ids == ref["tri_id"]
    ys = gb.spec.cpu().numpy().astype(np.float64)
    assert (ref["spec"] > 0.01).sum() > 200  # highlights in view
    assert np.max(np.abs(ys - ref["spec"])[same]) < TOL
    col = gb.color.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(col - ref["color"])[:, same]) < TOL
    # the table cleared: Lambertian again, specular plane 0
    hd.hdof_scene_set_specular(sc, None)
    g0 = hd.hdof_gbuffer(ctx, sc, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light),
                         out=hd.GBuffer.empty(H, W, spec=True))
    torch.cuda.synchronize()
    assert torch.count_nonzero(g0.spec).item() == 0
    lam = oracle.gbuffer(oracle.Scene(scene.verts, scene.albedo), cfg.camera, cfg.lens, cfg.light)
    assert np.max(np.abs(g0.color.cpu().numpy() - lam["color"])[:, same]) < TOL
    sc.close()


def test_trace_specular_matches_oracle(hd, ctx):
    print_case("trace glossy")
    W, H = 240, 135
    scene, cfg, sc, osc = _glossy(hd, ctx, W, H)
    spp = np.random.default_rng(4).integers(0, 5, (H, W)).astype(np.int32)
    ref = oracle.trace(osc, cfg.camera, cfg.lens, cfg.light, spp, seed=5, frame=1, per_ray=False)
    offs = excl_cumsum(spp).astype(np.int32)
    out = hd.hdof_trace_thin_lens(ctx, sc, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light),
                                  4, to_dev(spp.astype(np.uint8)), to_dev(offs),
                                  to_dev(np.array([spp.sum()], np.int32)), seed=5, frame=1)
    torch.cuda.synchronize()
    ctx.sync()
    ok = ref["px_amb"] == 0
    h = out.hit_ratio.cpu().numpy().astype(np.float64)
    near = h * out.c_near.cpu().numpy() - ref["hit_ratio"] * ref["c_near"]
    far = (1 - h) * out.c_far.cpu().numpy() - (1 - ref["hit_ratio"]) * ref["c_far"]
    assert np.max(np.abs(near)[:, ok]) < TOL and np.max(np.abs(far)[:, ok]) < TOL
    # the highlights reach the traced colours (not a Lambertian trace)
    lam = oracle.trace(oracle.Scene(scene.verts, scene.albedo), cfg.camera, cfg.lens, cfg.light, spp, seed=5,
                       frame=1, per_ray=False)
    assert np.abs(ref["c_near"] - lam["c_near"]).max() > 0.05 or np.abs(ref["c_far"] - lam["c_far"]).max() > 0.05
    sc.close()


@pytest.mark.parametrize("tile,masked", [(16, False), (16, True), (8, False)])
def test_postfilter_specular_matches_oracle(hd, ctx, tile, masked):
    print_case(f"postfilter specular tile {tile} masked {masked}")
    W, H = 333, 187
    scene = sg.glossy_living_room_scene(0)
    cfg = sg.config_1080p(W, H)
    osc = oracle.Scene(scene.verts, scene.albedo, scene.spec)
    gb = oracle.gbuffer(osc, cfg.camera, cfg.lens, cfg.light)
    col, z, ys = f32(gb["color"]), f32(gb["depth"]), f32(gb["spec"])
    pp = sg.PPParams(tile=tile)
    spp = np.random.default_rng(6).integers(0, 3, (H, W)).astype(np.uint8)
    ref = oracle.postfilter_spec(cfg.camera, cfg.lens, ys, z, pp)
    out, so = hd.hdof_postfilter_specular(ctx, to_dev(col, torch.float32), to_dev(z, torch.float32),
                                          to_dev(ys, torch.float32), to_dev(spp) if masked else None,
                                          hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.pp_params_of(pp))
    torch.cuda.synchronize()
    ctx.sync()
    g = so.cpu().numpy().astype(np.float64)
    sel = spp > 0 if masked else np.ones((H, W), bool)
    assert np.max(np.abs(g - ref)[sel]) < TOL, np.max(np.abs(g - ref)[sel])
    if masked:
        assert np.all(g[~sel] == 0)
    assert np.abs(ref - ys).max() > 0.01  # the gather moved something
    # the colour output is the plain post-filter's
    plain = hd.hdof_postfilter(ctx, to_dev(col, torch.float32), to_dev(z, torch.float32), hd.camera_of(cfg.camera),
                               hd.lens_of(cfg.lens), hd.pp_params_of(pp))
    torch.cuda.synchronize()
    assert torch.equal(plain, out)


def test_composite_specular_matches_oracle(hd, ctx):
    print_case("composite specular")
    W, H = 200, 120
    cfg = sg.config_1080p(W, H)
    rng = np.random.default_rng(7)
    z = f32(rng.uniform(0.4, 9.0, (H, W)))
    spp = rng.integers(0, 3, (H, W)).astype(np.uint8)
    col, cpp = f32(rng.uniform(0, 1, (3, H, W))), f32(rng.uniform(0, 1, (3, H, W)))
    cn, cf = f32(rng.uniform(0, 1, (3, H, W))), f32(rng.uniform(0, 1, (3, H, W)))
    h = f32(rng.uniform(0, 1, (H, W)))
    pps = f32(rng.uniform(0, 1.2, (H, W)))
    cp = sg.CompositeParams(h_t=0.5, spec_y=0.6)
    ref = oracle.composite(cfg.camera, cfg.lens, col, cpp, z, spp.astype(np.int32), cn, cf, h, cp, pps)
    rt = hd.RTResult(to_dev(cn, torch.float32), to_dev(cf, torch.float32), to_dev(h, torch.float32),
                     torch.zeros(H, W, device=DEV), torch.zeros(H, W, device=DEV))
    got = hd.hdof_composite(ctx, to_dev(col, torch.float32), to_dev(cpp, torch.float32), to_dev(z, torch.float32),
                            to_dev(spp), rt, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens),
                            hd.composite_params_of(cp), pp_spec=to_dev(pps, torch.float32))
    torch.cuda.synchronize()
    assert np.max(np.abs(got.cpu().numpy() - ref)) < 1e-5
    base = oracle.composite(cfg.camera, cfg.lens, col, cpp, z, spp.astype(np.int32), cn, cf, h,
                            sg.CompositeParams(h_t=0.5))
    assert np.abs(ref - base).max() > 0.05  # the rule changed pixels


@pytest.mark.parametrize("tile", [16, 8])
def test_frame_with_specular_rule(hd, ctx, tile):
    """hdof_frame on the glossy scene with spec_y > 0 equals its stages
    chained by hand (G-buffer with the specular plane, mask, trace,
    hdof_postfilter_specular restricted to the traced pixels, composite with
    the rule); spec_y = 0 gives the frame without the rule; the batched form
    and the adjoint refuse the rule."""
    print_case(f"frame specular tile {tile}")
    W, H = 320, 180
    scene, cfg, sc, osc = _glossy(hd, ctx, W, H)
    cfg.pp.tile = tile
    cam, lens, light = hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    on = hd.frame_params_of(cfg)
    on.comp.spec_y = 0.3
    k = hd.FrameKeep.empty(H, W)
    k.gb = hd.GBuffer.empty(H, W, spec=True)
    out = torch.empty(3, H, W, device=DEV)
    hd.hdof_history_reset(ctx)
    hd.hdof_frame(ctx, sc, cam, None, lens, light, on, frame=0, out=out, keep=k)
    pp_col, pps = hd.hdof_postfilter_specular(ctx, k.gb.color, k.gb.depth, k.gb.spec, k.spp, cam, lens, on.pp)
    ref = hd.hdof_composite(ctx, k.gb.color, pp_col, k.gb.depth, k.spp, k.rt, cam, lens, on.comp, pp_spec=pps)
    torch.cuda.synchronize()
    d = (out - ref).abs().max().item()
    assert d < 1e-5, d
    off = hd.frame_params_of(cfg)
    out0 = torch.empty(3, H, W, device=DEV)
    hd.hdof_history_reset(ctx)
    hd.hdof_frame(ctx, sc, cam, None, lens, light, off, frame=0, out=out0)
    torch.cuda.synchronize()
    changed = ((out - out0).abs().amax(0) > 1e-3).sum().item()
    assert changed > 50, changed
    with pytest.raises(hd.HdofError):
        hd.hdof_frame_batched(ctx, sc, light, on, [(cam, lens, 0, 0, 0)], [torch.empty(3, H, W, device=DEV)])
    grad = torch.zeros(3, H, W, device=DEV)
    with pytest.raises(hd.HdofError):
        hd.hdof_postfilter_composite_backward(ctx, k.gb.color, k.gb.depth, k.spp, k.rt, cam, lens, on.pp, on.comp,
                                              torch.ones(3, H, W, device=DEV), grad)
    sc.close()
