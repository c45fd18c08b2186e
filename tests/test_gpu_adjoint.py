"""GPU adjoint of post-filter + composite against the FP64 oracle adjoint
(colour gradient within 1e-5 of its largest magnitude, focus-distance and
aperture gradients within 1e-3 relative), through the C ABI and through the
torch.autograd.Function; and a focus-distance fit that moves towards the
target."""
import numpy as np
import pytest
import torch

import oracle as orc
import scenegen as sg
from gpu_common import DEV, f32, print_case, to_dev, upload_scene

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


def _small(seed):
    rng = np.random.default_rng(seed)
    W, H = 64, 48
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    lens = sg.Lens(0.05, float(np.float32(0.04)), 2.0)
    yy, xx = np.mgrid[0:H, 0:W]
    z = np.where(xx < W * 0.45, 0.7, 4.0) + 0.3 * np.sin(yy / 5.0)
    z[5:12, 30:40] = 2.0
    col = rng.uniform(0, 1, (3, H, W))
    spp = rng.integers(0, 3, (H, W)).astype(np.int32)
    hit = np.where(spp > 0, rng.uniform(0, 1, (H, W)), 0.0)
    cn, cf = rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (3, H, W))
    pp = sg.PPParams(n_taps=24, tile=8, r_cap=12.0, bg_ramp_px=1.0)
    g = rng.normal(size=(3, H, W))
    return cam, lens, f32(col), f32(z), spp, f32(cn), f32(cf), f32(hit), pp, sg.CompositeParams(), f32(g)


def _room(seed=0, W=256, H=144):
    scene, cfg = sg.living_room_scene(0), sg.config_1080p(W, H)
    gb = orc.gbuffer(orc.Scene(scene.verts, scene.albedo), cfg.camera, cfg.lens, cfg.light)
    rng = np.random.default_rng(seed)
    spp = rng.integers(0, 3, (H, W)).astype(np.int32)
    hit = np.where(spp > 0, rng.uniform(0, 1, (H, W)), 0.0)
    cn, cf = rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (3, H, W))
    g = rng.normal(size=(3, H, W))
    return (cfg.camera, cfg.lens, f32(gb["color"]), f32(gb["depth"]), spp, f32(cn), f32(cf), f32(hit), cfg.pp,
            cfg.comp, f32(g))


def _gpu_backward(hd, ctx, cam, lens, col, z, spp, cn, cf, hit, pp, cp, g):
    rt = hd.RTResult(to_dev(cn, torch.float32), to_dev(cf, torch.float32), to_dev(hit, torch.float32),
                     torch.zeros_like(to_dev(hit, torch.float32)), torch.zeros_like(to_dev(hit, torch.float32)))
    gc, gl = hd.hdof_postfilter_composite_backward(ctx, to_dev(col, torch.float32), to_dev(z, torch.float32),
                                                   to_dev(spp.astype(np.uint8)), rt, hd.camera_of(cam),
                                                   hd.lens_of(lens), hd.pp_params_of(pp), hd.composite_params_of(cp),
                                                   to_dev(g, torch.float32))
    torch.cuda.synchronize()
    return gc.cpu().numpy().astype(np.float64), gl.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("case", ["small0", "small1", "room", "room640", "room_t45", "room_t2"])
def test_backward_matches_oracle_adjoint(hd, ctx, case):
    """16-pixel tiles scatter through an LDS window (ceil R <= 21) or per-tap
    footprints added to global memory (larger R); room640 has both, room
    mostly the second; room_t45 and room_t2 take other tap counts (each
    block starts its transpose at tap (17 block) mod n_taps, and the texels
    are requested one tap ahead); the small cases use 8-pixel tiles (global
    atomics per pixel and tap)."""
    print_case(f"adjoint {case}")
    if case == "room":
        args = _room()
    elif case == "room640":
        args = _room(3, 640, 360)
    elif case.startswith("room_t"):
        args = list(_room(5, 320, 176))
        args[8] = sg.PPParams(n_taps=int(case[6:]), tile=16, r_cap=args[8].r_cap, bg_ramp_px=args[8].bg_ramp_px)
    else:
        args = _small(int(case[-1]))
    gc, gl = _gpu_backward(hd, ctx, *args)
    rc, rs, ra = orc.pp_composite_backward(*args)
    assert np.max(np.abs(gc - rc)) <= 1e-5 * np.max(np.abs(rc)), np.max(np.abs(gc - rc)) / np.max(np.abs(rc))
    assert abs(gl[0] - rs) <= 1e-3 * abs(rs), (gl[0], rs)
    assert abs(gl[1] - ra) <= 1e-3 * abs(ra), (gl[1], ra)


def test_autograd_function_and_focus_fit(hd, ctx):
    print_case("autograd + focus fit")
    cam, lens, col, z, spp, cn, cf, hit, pp, cp, _ = _room(1)
    H, W = z.shape
    rt = hd.RTResult(to_dev(cn, torch.float32), to_dev(cf, torch.float32), to_dev(hit, torch.float32),
                     torch.zeros(H, W, device=DEV), torch.zeros(H, W, device=DEV))
    colt = to_dev(col, torch.float32).requires_grad_(True)
    zt, st = to_dev(z, torch.float32), to_dev(spp.astype(np.uint8))
    camc, ppc, cpc = hd.camera_of(cam), hd.pp_params_of(pp), hd.composite_params_of(cp)
    f = float(lens.focal_length)

    def run(S1, A, c=colt):
        return hd.HybridDoFPost.apply(c, S1, A, zt, st, rt, camc, f, ppc, cpc, ctx)

    target = run(torch.tensor(2.0, device=DEV), torch.tensor(lens.aperture, device=DEV)).detach()
    S1 = torch.tensor(2.6, device=DEV, requires_grad=True)
    A = torch.tensor(float(lens.aperture), device=DEV, requires_grad=True)
    out = run(S1, A)
    loss = ((out - target) ** 2).sum()
    loss.backward()
    g = (2 * (out - target)).detach().cpu().numpy().astype(np.float64)
    rc, rs, ra = orc.pp_composite_backward(cam, sg.Lens(f, float(np.float32(lens.aperture)), 2.6), col, z, spp, cn,
                                           cf, hit, pp, cp, g)
    assert abs(S1.grad.item() - rs) <= 1e-3 * abs(rs)
    assert np.max(np.abs(colt.grad.cpu().numpy() - rc)) <= 1e-5 * np.max(np.abs(rc))
    # gradient descent on the focus distance alone approaches the target
    S1 = torch.tensor(2.6, device=DEV, requires_grad=True)
    opt = torch.optim.Adam([S1], lr=0.02)
    c0 = colt.detach()
    for _ in range(60):
        opt.zero_grad()
        loss = ((run(S1, torch.tensor(float(lens.aperture), device=DEV), c0) - target) ** 2).sum()
        loss.backward()
        opt.step()
    assert abs(S1.item() - 2.0) < 0.1, S1.item()
