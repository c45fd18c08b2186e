"""GPU parity of the temporally accumulated variance over a moving-camera
sequence (dolly 1 cm + yaw 0.2 degrees per frame, the temporal workload's
camera path) at 480x270 over 10 frames.

Per frame, the oracle produces the G-buffer, the reprojected history, the
mask, the trace and the updated history.  The GPU is given the oracle's
previous history (rounded to float32, through hdof_history_load), the
oracle's G-buffer and the oracle's traced moments, and must reproduce the
oracle's per-pixel counts (outside the flagged threshold / rounding bands)
and its updated history (exact flags, moments to fp32 rounding)."""
import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from gpu_common import chebyshev_dilate, excl_cumsum, f32, print_case, to_dev

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


def test_variance_sequence_matches_oracle(hd, ctx):
    W, H = 480, 270
    scene = sg.living_room_scene(0)
    cfg = sg.config_temporal(W, H)
    cfg.mask.spp_max = 16
    osc = oracle.Scene(scene.verts, scene.albedo)
    hist = oracle.empty_history(H, W)
    prev_cam = None
    n_checked = 0
    for t in range(10):
        print_case(f"temporal frame {t}")
        cam = sg.temporal_camera(t, W, H)
        gb = oracle.gbuffer(osc, cam, cfg.lens, cfg.light)
        depth, normal = f32(gb["depth"]), f32(gb["normal"])
        rep = None
        V = None
        if prev_cam is not None:
            rep = oracle.var_reproject(cam, depth, prev_cam, hist)
            V = rep["V"]
        mk = oracle.mask(depth, normal, cfg.mask, V)
        spp = mk["spp"]
        rt = oracle.trace(osc, cam, cfg.lens, cfg.light, spp, seed=0, frame=t, per_ray=False)
        if rep is None:
            rep_in = dict(lum_m1=np.zeros((H, W)), lum_m2=np.zeros((H, W)), flags=np.zeros((H, W), np.int32))
        else:
            rep_in = rep
        new_hist = oracle.var_update(spp, rep_in, f32(rt["lum_m1"]), f32(rt["lum_m2"]), cfg.mask.var_alpha, depth)

        # GPU: the oracle's previous history -> mask with reprojection
        if prev_cam is not None:
            hd.hdof_history_load(ctx, to_dev(f32(hist["lum_m1"]).astype(np.float32)),
                                 to_dev(f32(hist["lum_m2"]).astype(np.float32)),
                                 to_dev(hist["flags"].astype(np.uint8)), to_dev(f32(hist["depth"]).astype(np.float32)))
        else:
            hd.hdof_history_reset(ctx)
        mp = hd.mask_params_of(cfg.mask)
        g_spp, g_off, g_tot = hd.hdof_ray_mask(ctx, to_dev(depth, torch.float32), to_dev(normal, torch.float32),
                                               hd.camera_of(cam), hd.camera_of(prev_cam) if prev_cam else None,
                                               hd.lens_of(cfg.lens), mp)
        torch.cuda.synchronize()
        s = g_spp.cpu().numpy().astype(np.int64)
        # rounding / depth-test ambiguity of the reprojection spreads through the tiles
        amb = np.zeros((H, W), bool) if rep is None else rep["amb"] != 0
        from gpu_common import tile_footprint
        foot = tile_footprint(amb, cfg.mask.tile, cfg.mask.dilate)
        lo, hi = mk["spp_lo"], mk["spp_hi"]
        ok = ~foot
        assert np.all(((s >= lo) & (s <= hi))[ok]), f"frame {t}: counts outside the oracle band"
        assert np.array_equal(g_off.cpu().numpy().astype(np.int64), excl_cumsum(s))
        n_checked += int(ok.sum())
        # GPU: variance update from the oracle's counts and traced moments
        hd.hdof_variance_update(ctx, hd.camera_of(cam), mp, to_dev(spp.astype(np.uint8)), to_dev(depth, torch.float32),
                                to_dev(f32(rt["lum_m1"]), torch.float32), to_dev(f32(rt["lum_m2"]), torch.float32))
        gh = hd.hdof_history_save(ctx, H, W)
        torch.cuda.synchronize()
        gfl = gh["flags"].cpu().numpy().astype(np.int32)
        sure = ~chebyshev_dilate(amb, 0)
        assert np.array_equal(gfl[sure], new_hist["flags"][sure]), f"frame {t}: history flags differ"
        for k in ("lum_m1", "lum_m2"):
            d = np.abs(gh[k].cpu().numpy() - new_hist[k])[sure]
            assert d.max(initial=0) < 1e-5, (t, k, d.max())
        assert np.array_equal(gh["depth"].cpu().numpy(), depth.astype(np.float32))
        if t >= 1:
            assert (new_hist["flags"] & oracle.VALID).any()
        hist = dict(lum_m1=f32(new_hist["lum_m1"]), lum_m2=f32(new_hist["lum_m2"]), flags=new_hist["flags"],
                    depth=f32(new_hist["depth"]))
        prev_cam = cam
    assert n_checked > 0.6 * 10 * W * H   # tiles near a flagged reprojection are excluded
