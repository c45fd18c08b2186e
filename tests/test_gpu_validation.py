"""Argument validation with a live context: every out-of-range parameter of a
frame and of the tuning is refused with HDOF_ERR_INVALID_ARG before any
launch (the output buffer keeps its contents), the message names the
parameter, and the context still renders a valid frame afterwards."""
import math

import pytest
import torch

import scenegen as sg
from gpu_common import DEV, print_case, upload_scene

pytestmark = pytest.mark.gpu

INVALID_ARG = 1


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


@pytest.fixture(scope="module")
def room(hd, ctx):
    sc = upload_scene(hd, ctx, sg.living_room_scene(0))
    yield sc
    sc.close()


def _break(target, field, value):
    def f(cam, lens, params):
        obj = {"cam": cam, "lens": lens, "mask": params.mask, "pp": params.pp, "comp": params.comp,
               "recon": params.recon, "spatial": params.spatial}[target]
        setattr(obj, field, value)
    return f


CASES = [
    ("cam", "width", 0, "camera"),
    ("cam", "height", -5, "camera"),
    ("cam", "tan_half_fov_x", -1.0, "tan_half_fov"),
    ("lens", "focal_length", 0.0, "focal_length"),
    ("lens", "aperture", -0.01, "aperture"),
    ("lens", "focus_distance", 0.01, "focus_distance"),
    ("lens", "blades", 2, "blades"),
    ("lens", "sa", 5.0, "sa"),
    ("lens", "rotation", math.inf, "rotation"),
    ("mask", "spp_max", 0, "spp_max"),
    ("mask", "spp_max", 256, "spp_max"),
    ("mask", "tile", 12, "tile"),
    ("mask", "sigma", 3.0, "sigma"),
    ("mask", "var_alpha", 1.5, "var_alpha"),
    ("pp", "n_taps", 0, "n_taps"),
    ("pp", "n_taps", 257, "n_taps"),
    ("pp", "tile", 12, "tile"),
    ("pp", "r_cap", 300.0, "r_cap"),
    ("comp", "h_t", 0.0, "h_t"),
    ("comp", "spec_y", -1.0, "spec_y"),
    ("recon", "alpha", 0.0, "alpha"),
    ("spatial", "n_taps", 0, "n_taps"),
]


@pytest.mark.parametrize("target,field,value,word", CASES, ids=[f"{c[0]}.{c[1]}={c[2]}" for c in CASES])
def test_frame_rejects_out_of_range(hd, ctx, room, target, field, value, word):
    print_case(f"validation {target}.{field}={value}")
    W, H = 96, 64
    cfg = sg.config_1080p(W, H)
    cam, lens, light = hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    params = hd.frame_params_of(cfg)
    _break(target, field, value)(cam, lens, params)
    out = torch.full((3, H, W), -3.0, device=DEV)
    with pytest.raises(hd.HdofError) as ei:
        hd.hdof_frame(ctx, room, cam, None, lens, light, params, out=out)
    assert ei.value.status == INVALID_ARG
    assert word in str(ei.value), str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == -3.0).all())  # nothing was launched
    # the context is unharmed: a valid frame renders
    good = hd.frame_params_of(cfg)
    hd.hdof_frame(ctx, room, hd.camera_of(cfg.camera), None, hd.lens_of(cfg.lens), light, good, out=out)
    torch.cuda.synchronize()
    ctx.sync()
    assert bool(torch.isfinite(out).all()) and not bool((out == -3.0).any())


@pytest.mark.parametrize("kw", [dict(blocks_per_cu=0), dict(blocks_per_cu=33), dict(refill=0), dict(refill=65),
                                dict(segments=0), dict(segments=9), dict(wave=3), dict(overlap=2),
                                dict(overlap_ray_quantum=0)], ids=lambda kw: ",".join(f"{k}={v}" for k, v in kw.items()))
def test_tuning_rejects_out_of_range(hd, ctx, kw):
    print_case(f"tuning {kw}")
    before = hd.hdof_get_tuning(ctx)
    with pytest.raises(hd.HdofError) as ei:
        hd.hdof_set_tuning(ctx, **kw)
    assert ei.value.status == INVALID_ARG
    assert next(iter(kw)) in str(ei.value)
    assert hd.hdof_get_tuning(ctx) == before  # a refused tuning changes nothing


def test_queue_capacity_guard(hd, ctx):
    """The trace's capacity guard, forced from the host: counts of 2 rays per
    pixel against spp_max = 1 make the ray total (2N) exceed the queue's
    capacity (N entries).  The queue fill drops entries past the capacity,
    the trace clamps its total to it and raises the device flag, the
    reduction leaves the pixels whose rays lie past it untraced; hdof_sync
    reports HDOF_ERR_CAPACITY once and clears the flag.  The pixels whose
    rays fit are traced exactly as with a large enough capacity."""
    print_case("queue capacity guard")
    scene, cfg = sg.tiny_scene(0), sg.config_tiny(aperture_override=0.2)
    sc = upload_scene(hd, ctx, scene)
    H = W = 64
    N = H * W
    spp = torch.full((H, W), 2, dtype=torch.uint8, device=DEV)
    offs = (torch.arange(N, dtype=torch.int32, device=DEV) * 2).view(H, W)
    total = torch.tensor([2 * N], dtype=torch.int32, device=DEV)
    args = (hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light))
    ok = hd.hdof_trace_thin_lens(ctx, sc, *args, 2, spp, offs, total, seed=3)
    torch.cuda.synchronize()
    ctx.sync()
    ref = ok.c_near.clone(), ok.hit_ratio.clone()
    over = hd.hdof_trace_thin_lens(ctx, sc, *args, 1, spp, offs, total, seed=3)
    torch.cuda.synchronize()
    with pytest.raises(hd.HdofError) as ei:
        ctx.sync()
    assert ei.value.status == 4  # HDOF_ERR_CAPACITY
    ctx.sync()  # the flag was cleared
    fit = torch.zeros(N, dtype=torch.bool, device=DEV)
    fit[: N // 2] = True  # pixel p's rays are entries 2p, 2p + 1 < N
    fit = fit.view(H, W)
    assert torch.equal(over.c_near[:, fit], ref[0][:, fit])
    assert torch.equal(over.hit_ratio[fit], ref[1][fit])
    assert torch.all(over.hit_ratio[~fit] == 0) and torch.all(over.c_near[:, ~fit] == 0)
    sc.close()
