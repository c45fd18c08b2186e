"""GPU parity of the spatial reconstruction of the traced colours (paper,
Reconstruction, last paragraph) against the FP64 oracle: the trace's
near/far CoC averages, the stage itself on seeded inputs (ragged sizes,
every level of the pyramid, 1 to 48 taps, with and without an accumulated
hit ratio and a variance plane, an empty mask, 1920x1080) and on a real
frame's trace, and its place in hdof_frame (alone and after the temporal
reconstruction).

Bars.  The level and the tap pixels are integers that floating point
decides: the oracle takes them in double and flags a pixel whose spacing
lies within relative 1e-5 of a level boundary or whose tap coordinate lies
within its rounding band of a pixel boundary; flagged pixels are left out
(a pixel's output depends on its own decisions only).  Every other traced
pixel is compared at the 1e-3 linear-colour bar, except the ill-conditioned
ones, which are counted apart: a pixel's output is a ratio of
acceptance-weighted sums, and where the taps on the acceptance ramp carry
most of the weight it accepts (cond, reported by the oracle), the
single-precision acceptance arguments' rounding (at most EPS_A = r_cap
2^-19: the texel mean radii, sums of up to 1024 radii, and the tap
distances) can move it by EPS_A * cond * range.  Pixels where that bound
exceeds half the bar are reported separately, must be under 1 % of the
traced pixels, and are held to that bound.  Untraced pixels are copied
bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from gpu_common import f32, print_case, to_dev, upload_scene

pytestmark = pytest.mark.gpu

TOL = 1e-3  # linear colour, absolute
ILL_FRAC = 0.01


def eps_a(r_cap: float) -> float:
    return r_cap * 2.0 ** -19


@pytest.fixture(scope="module")
def hd():
    from paper_2210_04981_amd import hdof
    return hdof


@pytest.fixture(scope="module")
def ctx(hd):
    c = hd.Context(0)
    yield c
    c.close()


def _run_gpu(hd, ctx, inp, n_taps, r_cap, use_hacc, use_var, v_clamp=0.01):
    H, W = inp["spp"].shape
    rt = hd.RTResult(to_dev(inp["c_near"]), to_dev(inp["c_far"]), to_dev(inp["hit_ratio"]),
                     torch.zeros(H, W, device="cuda"), torch.zeros(H, W, device="cuda"))
    sp = hd.SpatialParams(1, n_taps, r_cap, v_clamp)
    cn, cf = hd.hdof_rt_spatial(ctx, H, W, to_dev(inp["spp"]), rt,
                                to_dev(inp["hit_acc"]) if use_hacc else None, to_dev(inp["coc_nf"]),
                                to_dev(inp["variance"]) if use_var else None, sp)
    torch.cuda.synchronize()
    ctx.sync()
    return cn.cpu().numpy().astype(np.float64), cf.cpu().numpy().astype(np.float64)


def _run_oracle(inp, n_taps, r_cap, use_hacc, use_var, v_clamp=0.01):
    return oracle.spatial(inp["spp"].astype(np.int32), f32(inp["c_near"]), f32(inp["c_far"]), f32(inp["hit_ratio"]),
                          f32(inp["hit_acc"]) if use_hacc else None, f32(inp["coc_nf"]),
                          f32(inp["variance"]) if use_var else None, n_taps, r_cap, v_clamp)


def _compare(inp, g, ref, name, r_cap):
    traced = inp["spp"] > 0
    amb = ref["amb"] != 0
    stats = {}
    for i, (k, gk) in enumerate(zip(("c_near", "c_far"), g)):
        rng = float(np.max(inp[k])) if traced.any() else 0.0
        bound = eps_a(r_cap) * ref["cond"][i] * rng
        ill = traced & ~amb & (bound > 0.5 * TOL)
        well = traced & ~amb & ~ill
        d = np.abs(gk - ref[k]).max(axis=0)
        print(f"{name} {k}: traced {traced.sum()}, flagged {(traced & amb).sum()}, ill-conditioned {ill.sum()}; "
              f"max err {d[well].max(initial=0):.2e} (bar {TOL:.0e}), ill-conditioned max err "
              f"{d[ill].max(initial=0):.2e} (bound {(bound[ill] + 1e-4).max(initial=0):.2e})", flush=True)
        assert d[well].max(initial=0) <= TOL, (name, k, d[well].max())
        assert np.all(d[ill] <= bound[ill] + 1e-4), (name, k)
        assert ill.sum() <= ILL_FRAC * max(traced.sum(), 1), (name, k, ill.sum(), traced.sum())
        # untraced pixels: bit-exact copies
        assert np.array_equal(gk[:, ~traced], inp[k].astype(np.float64)[:, ~traced]), (name, k)
        stats[k] = (well.sum(), traced.sum())
    if traced.sum() >= 100:
        assert (traced & amb).sum() <= 0.25 * traced.sum(), (name, (traced & amb).sum(), traced.sum())
    return stats


CASES = [
    # name, H, W, n_taps, r_cap, coverage, coc_max, hit_acc, variance, seed
    ("ragged_197x333_n24", 197, 333, 24, 64.0, 0.3, 150.0, True, True, 1),
    ("n1_r200_levels", 130, 150, 1, 200.0, 0.5, 400.0, False, False, 2),
    ("n4_level5", 256, 320, 4, 200.0, 0.4, 300.0, True, True, 3),
    ("n48_small_coc", 96, 160, 48, 64.0, 0.6, 12.0, False, True, 4),
    ("tiny_5x7", 5, 7, 24, 64.0, 1.0, 40.0, True, True, 5),
    ("empty_mask", 40, 50, 24, 64.0, 0.0, 150.0, False, False, 6),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_spatial_stage_matches_oracle(hd, ctx, case):
    name, H, W, n_taps, r_cap, cov, cmax, use_hacc, use_var, seed = case
    print_case(f"spatial {name}")
    inp = sg.spatial_inputs(H, W, seed, cov, cmax)
    ref = _run_oracle(inp, n_taps, r_cap, use_hacc, use_var)
    g = _run_gpu(hd, ctx, inp, n_taps, r_cap, use_hacc, use_var)
    _compare(inp, g, ref, name, r_cap)
    if name == "empty_mask":
        assert not (inp["spp"] > 0).any()
    else:
        # the stage changed something (the comparison is not vacuous)
        assert np.abs(ref["c_near"] - inp["c_near"]).max() > 1e-2


def test_spatial_levels_are_all_reached(hd, ctx):
    """The seeded cases above reach every level: with 4 taps and radii up to
    150 px the spacing r sqrt(pi/4) spans 0 .. 133 px."""
    inp = sg.spatial_inputs(256, 320, 3, 0.4, 300.0)
    hacc = inp["hit_acc"].astype(np.float64)
    r = np.minimum(200.0, 0.5 * (hacc * inp["coc_nf"][0] + (1 - hacc) * inp["coc_nf"][1]))
    sp = r * np.sqrt(np.pi / 4)
    L = np.clip(np.floor(np.log2(np.maximum(sp, 1e-30))), 0, 5)[inp["spp"] > 0]
    assert set(np.unique(L).astype(int)) == {0, 1, 2, 3, 4, 5}


def test_spatial_full_size(hd, ctx):
    """1920x1080, 24 taps, r_cap 64, about 5 % of the pixels traced."""
    print_case("spatial 1920x1080")
    inp = sg.spatial_inputs(1080, 1920, 11, 0.055, 150.0)
    ref = _run_oracle(inp, 24, 64.0, True, True)
    g = _run_gpu(hd, ctx, inp, 24, 64.0, True, True)
    _compare(inp, g, ref, "1080p", 64.0)


def test_coc_averages_match_oracle(hd, ctx):
    print_case("coc averages")
    W, H = 320, 180
    scene, cfg = sg.living_room_scene(0), sg.config_1080p(W, H)
    osc = oracle.Scene(scene.verts, scene.albedo)
    rng = np.random.default_rng(8)
    spp = rng.integers(0, 5, (H, W)).astype(np.int32)
    ref = oracle.trace(osc, cfg.camera, cfg.lens, cfg.light, spp, seed=3, frame=1, per_ray=False)
    sc = upload_scene(hd, ctx, scene)
    offs = np.concatenate([[0], np.cumsum(spp.reshape(-1))[:-1]]).astype(np.int32)
    coc = torch.zeros(2, H, W, device="cuda")
    hd.hdof_trace_thin_lens(ctx, sc, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light), 4,
                            to_dev(spp.astype(np.uint8)), to_dev(offs), to_dev(np.array([spp.sum()], np.int32)),
                            seed=3, frame=1, coc_nf=coc)
    torch.cuda.synchronize()
    ctx.sync()
    g = coc.cpu().numpy().astype(np.float64)
    r = ref["coc_nf"]
    ok = ref["px_amb"] == 0
    assert (ok & (spp > 0)).sum() > 10000
    rel = np.abs(g - r)[:, ok] / np.maximum(r[:, ok], 1.0)
    assert rel.max() < 1e-4, rel.max()
    assert np.all(g[:, spp == 0] == 0)
    sc.close()


def test_spatial_on_a_real_trace(hd, ctx):
    """The oracle's own 480x270 living-room frame (G-buffer, mask, trace,
    first-frame variance) feeds both sides."""
    print_case("spatial on a traced frame")
    W, H = 480, 270
    scene, cfg = sg.living_room_scene(0), sg.config_1080p(W, H)
    osc = oracle.Scene(scene.verts, scene.albedo)
    fr = oracle.frame(osc, cfg)
    rt, spp = fr["rt"], fr["spp"]
    assert (spp > 0).sum() > 2000
    V = oracle.history_variance(fr["history"])
    inp = dict(spp=spp.astype(np.uint8), c_near=rt["c_near"].astype(np.float32), c_far=rt["c_far"].astype(np.float32),
               hit_ratio=rt["hit_ratio"].astype(np.float32), hit_acc=rt["hit_ratio"].astype(np.float32),
               coc_nf=rt["coc_nf"].astype(np.float32), variance=V.astype(np.float32))
    for n_taps in (24, 48):
        ref = _run_oracle(inp, n_taps, 64.0, False, True)
        g = _run_gpu(hd, ctx, inp, n_taps, 64.0, False, True)
        _compare(inp, g, ref, f"frame n{n_taps}", 64.0)


def _hist_variance(hd, ctx, H, W):
    h = hd.hdof_history_save(ctx, H, W)
    m1, m2, fl = h["lum_m1"], h["lum_m2"], h["flags"].to(torch.int32)
    V = torch.clamp(m2 - m1 * m1, min=0.0)
    V = torch.where((fl & 1) != 0, V, torch.zeros_like(V))
    return torch.where((fl & 2) != 0, torch.full_like(V, float("inf")), V).contiguous()


@pytest.mark.parametrize("with_recon", [False, True], ids=["spatial", "temporal+spatial"])
def test_frame_with_spatial(hd, ctx, with_recon):
    """hdof_frame with the spatial stage equals the stage chained by hand on
    a second context (trace with CoC averages, the temporal stage when on,
    then hdof_rt_spatial with the updated history's variance and the
    temporal history's accumulated hit ratio); the batched form refuses it."""
    print_case(f"frame + spatial (recon={with_recon})")
    W, H = 320, 180
    scene = sg.living_room_scene(0)
    cfg = sg.config_temporal(W, H)
    cfg.mask.spp_max = 8
    sc = upload_scene(hd, ctx, scene)
    lens, light = hd.lens_of(cfg.lens), hd.light_of(cfg.light)
    on = hd.frame_params_of(cfg)
    on.spatial.enable, on.spatial.n_taps, on.spatial.r_cap, on.spatial.v_clamp = 1, 24, 64.0, 0.01
    on.recon.enable, on.recon.alpha = int(with_recon), 0.2
    off = hd.frame_params_of(cfg)
    cams = [hd.camera_of(sg.temporal_camera(t, W, H)) for t in range(3)]
    k_on = hd.FrameKeep.empty(H, W)
    hd.hdof_history_reset(ctx)
    hd.hdof_recon_history_reset(ctx)
    ctx2 = hd.Context(0)
    try:
        sc2 = upload_scene(hd, ctx2, scene)
        hd.hdof_history_reset(ctx2)
        hd.hdof_recon_history_reset(ctx2)
        fp = torch.zeros(4, H, W, device="cuda")
        coc = torch.zeros(2, H, W, device="cuda")
        rp = hd.ReconParams(1, 0.2)
        changed = 0
        for t in range(3):
            prev = cams[t - 1] if t else None
            hd.hdof_frame(ctx, sc, cams[t], prev, lens, light, on, frame=t, keep=k_on)
            k = hd.FrameKeep.empty(H, W)
            hd.hdof_frame(ctx2, sc2, cams[t], prev, lens, light, off, frame=t, keep=k)
            hd.hdof_trace_thin_lens(ctx2, sc2, cams[t], lens, light, cfg.mask.spp_max, k.spp, k.offsets, k.total,
                                    seed=cfg.seed, frame=t, out=k.rt, far_pos=fp, coc_nf=coc)
            hacc = None
            if with_recon:
                hd.hdof_rt_reconstruct(ctx2, cams[t], prev, k.gb.depth, k.spp, fp, k.rt, rp)
                hacc = hd.hdof_recon_history_save(ctx2, H, W)["planes"][3].contiguous()
            V = _hist_variance(hd, ctx2, H, W)
            cn, cf = hd.hdof_rt_spatial(ctx2, H, W, k.spp, k.rt, hacc, coc, V,
                                        hd.SpatialParams(1, 24, 64.0, 0.01))
            torch.cuda.synchronize()
            assert torch.equal(k_on.spp, k.spp)
            for name, ref in (("c_near", cn), ("c_far", cf)):
                got = getattr(k_on.rt, name)
                if t == 0:
                    assert torch.equal(got, ref), (t, name)  # every traced pixel is new: lambda = 1
                else:
                    d = (got - ref).abs().max().item()
                    assert d < 2e-4, (t, name, d)  # V formed by torch here, by the kernel there
                changed += int(((ref - getattr(k.rt, name)).abs() > 1e-3).sum().item())
        assert changed > 1000
        sc2.close()
    finally:
        ctx2.close()
    views = [(cams[0], lens, 0, 0, 0)]
    sp_only = hd.frame_params_of(cfg)
    sp_only.spatial.enable = 1
    with pytest.raises(hd.HdofError):
        hd.hdof_frame_batched(ctx, sc, light, sp_only, views, [torch.empty(3, H, W, device="cuda")])
    sc.close()


def test_spatial_rejects_bad_arguments(hd, ctx):
    H, W = 16, 16
    inp = sg.spatial_inputs(H, W, 0, 1.0)
    rt = hd.RTResult(to_dev(inp["c_near"]), to_dev(inp["c_far"]), to_dev(inp["hit_ratio"]),
                     torch.zeros(H, W, device="cuda"), torch.zeros(H, W, device="cuda"))
    for sp in (hd.SpatialParams(1, 0, 64.0, 0.01), hd.SpatialParams(1, 24, -1.0, 0.01),
               hd.SpatialParams(1, 24, 64.0, 0.0), hd.SpatialParams(2, 24, 64.0, 0.01)):
        with pytest.raises(hd.HdofError):
            hd.hdof_rt_spatial(ctx, H, W, to_dev(inp["spp"]), rt, None, to_dev(inp["coc_nf"]), None, sp)
    with pytest.raises(hd.HdofError):  # output aliasing an input
        hd.hdof_rt_spatial(ctx, H, W, to_dev(inp["spp"]), rt, None, to_dev(inp["coc_nf"]), None,
                           hd.SpatialParams(1, 24, 64.0, 0.01), c_near_out=rt.c_near)
