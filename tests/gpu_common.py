"""Shared helpers of the GPU parity tests (inputs from scenegen, expected
values from the oracle, results through the C ABI binding)."""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage as ndi
import torch

import scenegen as sg

DEV = torch.device("cuda:0")


def to_dev(a, dtype=None) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def f32(a) -> np.ndarray:
    """Round to float32 (the interface precision) and widen back exactly."""
    return np.asarray(a, np.float32).astype(np.float64)


def upload_scene(hdof, ctx, scene: sg.Scene):
    return hdof.hdof_build_bvh(ctx, to_dev(scene.verts), to_dev(scene.albedo))


def chebyshev_dilate(mask: np.ndarray, r: int) -> np.ndarray:
    if r <= 0 or not mask.any():
        return mask.copy()
    return ndi.binary_dilation(mask, structure=np.ones((2 * r + 1, 2 * r + 1), bool))


def tile_footprint(mask: np.ndarray, tile: int, dil: int) -> np.ndarray:
    """Pixels whose tile lies within `dil` tiles of a tile containing a marked pixel."""
    H, W = mask.shape
    TH, TW = -(-H // tile), -(-W // tile)
    t = np.zeros((TH, TW), bool)
    ys, xs = np.nonzero(mask)
    t[ys // tile, xs // tile] = True
    t = chebyshev_dilate(t, dil)
    return np.repeat(np.repeat(t, tile, 0), tile, 1)[:H, :W]


def excl_cumsum(s: np.ndarray) -> np.ndarray:
    flat = s.reshape(-1).astype(np.int64)
    return np.concatenate([[0], np.cumsum(flat)[:-1]]).reshape(s.shape)


def print_case(name: str) -> None:
    print(f"[case] {name}", flush=True)


COL_TOL = 1e-3  # linear colour, absolute


def run_frame(hd, ctx, sc, cfg, prev=None, frame=0, view=0):
    """hdof_frame with every intermediate kept; results as float64/int64 numpy."""
    H, W = cfg.camera.height, cfg.camera.width
    keep = hd.FrameKeep.empty(H, W)
    out = hd.hdof_frame(ctx, sc, hd.camera_of(cfg.camera), hd.camera_of(prev) if prev is not None else None,
                        hd.lens_of(cfg.lens), hd.light_of(cfg.light), hd.frame_params_of(cfg), seed=cfg.seed,
                        frame=frame, view=view, keep=keep)
    torch.cuda.synchronize()
    ctx.sync()
    return frame_numpy(out, keep)


def frame_numpy(out, keep) -> dict:
    g = dict(out=out.cpu().numpy().astype(np.float64), spp=keep.spp.cpu().numpy().astype(np.int64),
             offsets=keep.offsets.cpu().numpy().astype(np.int64), total=int(keep.total.item()),
             tri_id=keep.gb.tri_id.cpu().numpy(), color=keep.gb.color.cpu().numpy().astype(np.float64),
             depth=keep.gb.depth.cpu().numpy().astype(np.float64), pp=keep.pp.cpu().numpy().astype(np.float64),
             normal=keep.gb.normal.cpu().numpy().astype(np.float64))
    for k in ("c_near", "c_far", "hit_ratio", "lum_m1", "lum_m2"):
        g[k] = getattr(keep.rt, k).cpu().numpy().astype(np.float64)
    return g


def compare_frame(g, ref, cfg, hist=None, iso=True):
    """Whole-frame parity of a GPU frame `g` (run_frame) with oracle.frame's
    `ref` on the same inputs.  Every G-buffer hit that differs must be one the
    oracle flagged; downstream stages are compared outside the stencil, tile
    and gather footprints of the pixels whose G-buffer values differ and of
    the pixels whose history reprojection the oracle flagged.  `hist`: the
    GPU's variance history after the frame (hdof_history_save, as numpy),
    compared with the oracle's updated history (flags exact, moments within
    1e-5, depth within relative 1e-5) wherever the counts, the rays and the
    reprojection agree.  Returns counts and the fraction compared at the
    full bar.  `iso`: also run the oracle's post-filter and composite on the
    GPU's own G-buffer, counts and traced planes, and compare them with the
    GPU's at every pixel (stage-isolated: no footprint is left out)."""
    gb = ref["gbuffer"]
    H, W = gb["depth"].shape
    # 1. G-buffer: differences only where the oracle flags them
    diff_id = g["tri_id"] != gb["tri_id"]
    assert not (diff_id & (gb["amb"] == 0)).any()
    same = ~diff_id
    # a legitimately different hit matters downstream only where it changes
    # the G-buffer values (neighbouring coplanar faces of one object do not)
    dz = np.abs(g["depth"] - gb["depth"]) / np.maximum(gb["depth"], 1e-6)
    dc = np.max(np.abs(g["color"] - gb["color"]), axis=0)
    diff_gb = diff_id & ((dz > 1e-5) | (dc > 2e-4))
    # neighbours of such a pixel see a different normal only if the faces differ
    diff_n = diff_id & (np.max(np.abs(g["normal"] - gb["normal"]), axis=0) > 1e-4)
    assert np.max(np.abs(g["color"] - gb["color"])[:, same], initial=0) < COL_TOL
    # 2. mask, outside the stencil + tile footprint of differing G-buffer
    #    pixels and of flagged reprojections (a pixel's variance term reads
    #    its own reprojected history only)
    mp = cfg.mask
    gr = int(math.floor(3 * mp.sigma + 0.5))
    rep = ref.get("reproj")
    rep_amb = np.zeros((H, W), bool)
    if rep is not None and "amb" in rep:
        rep_amb = rep["amb"] != 0
    seed_px = chebyshev_dilate(diff_gb | diff_n, gr + 1) | rep_amb
    tile = mp.tile if mp.tile > 0 else 16
    foot_mask = tile_footprint(seed_px, tile, mp.dilate)
    lo, hi = ref["mask"]["spp_lo"], ref["mask"]["spp_hi"]
    s = g["spp"]
    assert np.all((s >= lo) & (s <= hi) | foot_mask)
    assert np.array_equal(g["offsets"], excl_cumsum(s)) and g["total"] == s.sum()
    # 3. trace: pixels with equal counts and unambiguous rays trace the same rays
    rt = ref["rt"]
    tr_ok = (s == ref["spp"]) & (rt["px_amb"] == 0)
    h = g["hit_ratio"]
    assert np.max(np.abs(h - rt["hit_ratio"])[tr_ok], initial=0) < 1e-4
    crt_g = h * g["c_near"] + (1 - h) * g["c_far"]
    crt_r = rt["hit_ratio"] * rt["c_near"] + (1 - rt["hit_ratio"]) * rt["c_far"]
    assert np.max(np.abs(crt_g - crt_r)[:, tr_ok], initial=0) < COL_TOL
    # 4. post-filter outside the gather footprint of differing G-buffer pixels
    pp = cfg.pp
    K = math.ceil(pp.r_cap / pp.tile)
    foot_pp = chebyshev_dilate(diff_gb, int(pp.r_cap) + 2) | tile_footprint(diff_gb, pp.tile, K)
    assert np.max(np.abs(g["pp"] - ref["pp"])[:, ~foot_pp], initial=0) < COL_TOL
    # 5. composite where every input agrees
    comp_ok = same & ~foot_pp & tr_ok
    assert np.max(np.abs(g["out"] - ref["out"])[:, comp_ok], initial=0) < COL_TOL
    info = dict(diff_id=int(diff_id.sum()), diff_gb=int(diff_gb.sum()), rep_amb=int(rep_amb.sum()),
                traced=int((s > 0).sum()), compared=float(comp_ok.mean()))
    if iso:
        import oracle
        pp_iso = oracle.postfilter(cfg.camera, cfg.lens, g["color"], g["depth"], cfg.pp)
        e_pp = float(np.max(np.abs(g["pp"] - pp_iso)))
        assert e_pp < COL_TOL, e_pp
        info["pp_iso_err"] = e_pp
        if getattr(cfg.comp, "spec_y", 0.0) == 0.0:
            out_iso = oracle.composite(cfg.camera, cfg.lens, g["color"], g["pp"], g["depth"], g["spp"], g["c_near"],
                                       g["c_far"], g["hit_ratio"], cfg.comp)
            e_out = float(np.max(np.abs(g["out"] - out_iso)))
            assert e_out < COL_TOL, e_out
            info["out_iso_err"] = e_out
    # 6. the updated variance history
    if hist is not None:
        rh = ref["history"]
        h_ok = tr_ok & same & ~diff_gb & ~rep_amb
        assert np.array_equal(hist["flags"][h_ok], rh["flags"][h_ok]), "history flags differ"
        for k in ("lum_m1", "lum_m2"):
            d = np.abs(hist[k] - rh[k])[h_ok]
            assert d.max(initial=0) < 1e-5, (k, d.max())
        dzh = np.abs(hist["depth"] - rh["depth"]) / np.maximum(np.abs(rh["depth"]), 1e-6)
        assert dzh[h_ok].max(initial=0) < 1e-5
        info["history_compared"] = float(h_ok.mean())
        info["history_valid"] = int(((rh["flags"] & 1) != 0).sum())
        info["history_ema"] = int((((rh["flags"] & 1) != 0) & ((rh["flags"] & 2) == 0) & (s > 0)).sum())
        info["history_new"] = int(((rh["flags"] & 2) != 0).sum())
    return info


def history_numpy(hd, ctx, H, W) -> dict:
    """The context's variance history (the one the next frame reprojects),
    widened to float64 / int32."""
    gh = hd.hdof_history_save(ctx, H, W)
    torch.cuda.synchronize()
    return dict(lum_m1=gh["lum_m1"].cpu().numpy().astype(np.float64),
                lum_m2=gh["lum_m2"].cpu().numpy().astype(np.float64),
                flags=gh["flags"].cpu().numpy().astype(np.int32),
                depth=gh["depth"].cpu().numpy().astype(np.float64))
