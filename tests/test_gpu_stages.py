"""GPU parity of each stage against the FP64 oracle (stage-isolated: every
GPU stage and the oracle receive the same float32 inputs, produced by the
oracle or by scenegen, never by the GPU).

Bars: hit triangle ids and per-pixel ray counts identical
except where the oracle flags an edge / tie / threshold ambiguity within
1e-5; linear colour within 1e-3 absolute.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen as sg
from gpu_common import DEV, excl_cumsum, f32, print_case, to_dev, upload_scene

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


def _gpu_gbuffer(hd, ctx, scene, cfg):
    sc = upload_scene(hd, ctx, scene)
    gb = hd.hdof_gbuffer(ctx, sc, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light))
    torch.cuda.synchronize()
    ctx.sync()
    return sc, {k: getattr(gb, k).cpu().numpy() for k in ("depth", "normal", "albedo", "color", "tri_id")}


def _check_gbuffer(g, ref):
    ids, rid, amb = g["tri_id"], ref["tri_id"], ref["amb"] != 0
    bad = (ids != rid) & ~amb
    assert not bad.any(), f"{bad.sum()} unambiguous G-buffer hits differ, e.g. {np.argwhere(bad)[:5]}"
    same = ids == rid
    hit = same & (rid >= 0)
    assert np.allclose(g["depth"][hit], ref["depth"][hit], rtol=1e-5, atol=0)
    assert np.max(np.abs(g["color"] - ref["color"])[:, same], initial=0) < COL_TOL
    assert np.max(np.abs(g["normal"] - ref["normal"])[:, same], initial=0) < 1e-4
    assert np.array_equal(g["albedo"][:, same], f32(ref["albedo"])[:, same])
    return same


@pytest.mark.parametrize("which", ["tiny", "room_small"])
def test_gbuffer_matches_oracle(hd, ctx, which):
    print_case(f"gbuffer {which}")
    if which == "tiny":
        scene, cfg = sg.tiny_scene(0), sg.config_tiny()
    else:
        scene, cfg = sg.living_room_scene(0), sg.config_1080p(320, 180)
    sc, g = _gpu_gbuffer(hd, ctx, scene, cfg)
    ref = oracle.gbuffer(oracle.Scene(scene.verts, scene.albedo), cfg.camera, cfg.lens, cfg.light)
    _check_gbuffer(g, ref)
    st = sc.stats()
    assert st["max_depth"] <= 64, st
    sc.close()


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 100])
def test_gbuffer_few_triangles(hd, ctx, n):
    """BVH edge cases: a single triangle, two, ragged small counts."""
    print_case(f"gbuffer few triangles n={n}")
    rng = np.random.default_rng(n)
    xy = rng.uniform(-1.5, 1.5, (n, 3, 2))
    z = rng.uniform(1.5, 4.0, (n, 3, 1))
    verts = np.concatenate([xy, z], -1).reshape(n, 9).astype(np.float32)
    alb = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    scene = sg.Scene(verts, alb)
    cfg = sg.config_tiny()
    cfg.camera = sg.look_camera((0, 0, 0), 0.0, 48, 40)
    sc, g = _gpu_gbuffer(hd, ctx, scene, cfg)
    ref = oracle.gbuffer(oracle.Scene(verts, alb), cfg.camera, cfg.lens, cfg.light)
    _check_gbuffer(g, ref)
    sc.close()


MASK_CASES = [
    dict(sigma=1.0, tile=8, dilate=1, spp_max=8, var=False),
    dict(sigma=1.0, tile=1, dilate=0, spp_max=255, var=False),
    dict(sigma=0.7, tile=4, dilate=2, spp_max=5, var=True),
    dict(sigma=2.0, tile=16, dilate=0, spp_max=16, var=True),
    dict(sigma=1.3, tile=2, dilate=1, spp_max=1, var=True),
]


@pytest.mark.parametrize("case", range(len(MASK_CASES)))
def test_ray_mask_matches_oracle(hd, ctx, case):
    c = MASK_CASES[case]
    print_case(f"ray mask {c}")
    scene, cfg = sg.living_room_scene(0), sg.config_1080p(333, 187)   # ragged tiles on both axes
    ref_gb = oracle.gbuffer(oracle.Scene(scene.verts, scene.albedo), cfg.camera, cfg.lens, cfg.light)
    H, W = ref_gb["depth"].shape
    depth, normal = f32(ref_gb["depth"]), f32(ref_gb["normal"])
    mp = sg.MaskParams(sigma=c["sigma"], tile=c["tile"], dilate=c["dilate"], spp_max=c["spp_max"])
    hist = None
    V = None
    if c["var"]:
        # a history loaded through the ABI: static camera, random moments, some new and invalid pixels
        rng = np.random.default_rng(case)
        m1 = rng.uniform(0, 1, (H, W)).astype(np.float32)
        m2 = (m1.astype(np.float64) ** 2 + rng.exponential(0.01, (H, W))).astype(np.float32)
        flags = rng.choice([0, 1, 3], size=(H, W), p=[0.2, 0.75, 0.05]).astype(np.uint8)
        hz = (depth * rng.choice([1.0, 1.03], size=(H, W), p=[0.9, 0.1])).astype(np.float32)
        hist = dict(lum_m1=f32(m1), lum_m2=f32(m2), flags=flags.astype(np.int32), depth=f32(hz))
        rep = oracle.var_reproject(cfg.camera, depth, cfg.camera, hist)
        V = rep["V"]
        hd.hdof_history_load(ctx, to_dev(m1), to_dev(m2), to_dev(flags), to_dev(hz))
    ref = oracle.mask(depth, normal, mp, V)
    cam = hd.camera_of(cfg.camera)
    spp, offs, tot = hd.hdof_ray_mask(ctx, to_dev(depth, torch.float32), to_dev(normal, torch.float32), cam,
                                      cam if c["var"] else None, hd.lens_of(cfg.lens), hd.mask_params_of(mp))
    torch.cuda.synchronize()
    s = spp.cpu().numpy().astype(np.int64)
    amb_rep = np.zeros((H, W), bool)
    if c["var"]:
        amb_rep = rep["amb"] != 0
        assert not amb_rep.any()  # static camera: reprojection lands on pixel centres
    lo, hi = ref["spp_lo"], ref["spp_hi"]
    assert np.all((s >= lo) & (s <= hi)), f"{np.sum((s < lo) | (s > hi))} counts outside the oracle band"
    uniq = lo == hi
    assert np.array_equal(s[uniq], ref["spp"][uniq])
    assert uniq.mean() > 0.99
    assert np.array_equal(offs.cpu().numpy().astype(np.int64), excl_cumsum(s))
    assert int(tot.item()) == int(s.sum())


@pytest.mark.parametrize("f_number,tile", [(1.4, 4), (1.0, 8), (0.5, 16)])
def test_ray_mask_scaled_tile(hd, ctx, f_number, tile):
    """Mask tile 0: the tile edge is picked on the device from the frame's
    largest CoC radius (all three edges reached by the apertures), and the
    counts equal the oracle's and the GPU's own mask at that fixed edge."""
    from dataclasses import replace
    print_case(f"ray mask scaled tile f/{f_number}")
    scene, cfg = sg.living_room_scene(0), sg.config_1080p(333, 187)
    lens = sg.lens_fnumber(cfg.lens.focal_length, f_number, cfg.lens.focus_distance)
    ref_gb = oracle.gbuffer(oracle.Scene(scene.verts, scene.albedo), cfg.camera, lens, cfg.light)
    depth, normal = f32(ref_gb["depth"]), f32(ref_gb["normal"])
    t_ref, r_max = oracle.scaled_tile(cfg.camera, lens, depth)
    assert t_ref == tile
    assert min(abs(r_max - 16), abs(r_max - 32)) > 1e-3 * r_max  # clear of the band edges
    mp = sg.MaskParams(sigma=1.0, tile=0, dilate=1, spp_max=8)
    ref = oracle.mask(depth, normal, mp, None, cfg.camera, lens)
    assert ref["tile"] == tile
    cam = hd.camera_of(cfg.camera)
    d_t, n_t = to_dev(depth, torch.float32), to_dev(normal, torch.float32)
    spp, offs, tot = hd.hdof_ray_mask(ctx, d_t, n_t, cam, None, hd.lens_of(lens), hd.mask_params_of(mp))
    spp_f, offs_f, tot_f = hd.hdof_ray_mask(ctx, d_t, n_t, cam, None, hd.lens_of(lens),
                                            hd.mask_params_of(replace(mp, tile=tile)))
    torch.cuda.synchronize()
    assert torch.equal(spp, spp_f) and torch.equal(offs, offs_f) and torch.equal(tot, tot_f)
    s = spp.cpu().numpy().astype(np.int64)
    lo, hi = ref["spp_lo"], ref["spp_hi"]
    assert np.all((s >= lo) & (s <= hi))
    uniq = lo == hi
    assert np.array_equal(s[uniq], ref["spp"][uniq]) and uniq.mean() > 0.99


def test_frame_with_scaled_mask_tile(hd, ctx):
    """hdof_frame with mask tile 0 (the fused queue-filling mask reads the
    device-side choice) equals the frame with the chosen edge fixed."""
    print_case("frame with scaled mask tile")
    W, H = 320, 180
    scene, cfg = sg.living_room_scene(0), sg.config_1080p(W, H)
    sc = upload_scene(hd, ctx, scene)
    lens = sg.lens_fnumber(cfg.lens.focal_length, 1.0, cfg.lens.focus_distance)
    gb = oracle.gbuffer(oracle.Scene(scene.verts, scene.albedo), cfg.camera, lens, cfg.light)
    t, r_max = oracle.scaled_tile(cfg.camera, lens, f32(gb["depth"]))
    assert t == 8 and min(abs(r_max - 16), abs(r_max - 32)) > 1e-3 * r_max
    outs = []
    for tile in (0, t):
        p = hd.frame_params_of(cfg)
        p.mask.tile = tile
        k = hd.FrameKeep.empty(H, W)
        out = torch.empty(3, H, W, device="cuda")
        hd.hdof_history_reset(ctx)
        hd.hdof_frame(ctx, sc, hd.camera_of(cfg.camera), None, hd.lens_of(lens), hd.light_of(cfg.light), p,
                      frame=0, out=out, keep=k)
        torch.cuda.synchronize()
        outs.append((out, k))
    assert torch.equal(outs[0][1].spp, outs[1][1].spp)
    assert torch.equal(outs[0][0], outs[1][0])
    assert int(outs[0][1].total.item()) > 1000
    sc.close()


@pytest.mark.parametrize("which,wave", [("tiny", 0), ("tiny_strong", 0), ("room_small", 0), ("tiny_strong", 1),
                                        ("room_small", 1)])
def test_trace_matches_oracle(hd, ctx, which, wave):
    """Both traversal forms of the persistent trace (per-lane with refill,
    and wave-coherent batches of 64 entries) against the oracle."""
    print_case(f"trace {which} wave {wave}")
    hd.hdof_set_tuning(ctx, wave=wave)
    if which == "room_small":
        scene, cfg = sg.living_room_scene(0), sg.config_1080p(320, 180)
    else:
        scene = sg.tiny_scene(0)
        cfg = sg.config_tiny() if which == "tiny" else sg.config_tiny(aperture_override=0.2)
    osc = oracle.Scene(scene.verts, scene.albedo)
    ref_gb = oracle.gbuffer(osc, cfg.camera, cfg.lens, cfg.light)
    mk = oracle.mask(f32(ref_gb["depth"]), f32(ref_gb["normal"]), cfg.mask)
    spp = mk["spp"]
    H, W = spp.shape
    if which == "room_small":
        # every pixel traced with ragged counts, so the whole image is exercised
        spp = np.random.default_rng(3).integers(0, cfg.mask.spp_max + 1, (H, W)).astype(np.int32)
    ref = oracle.trace(osc, cfg.camera, cfg.lens, cfg.light, spp, seed=11, frame=2, view=1, per_ray=True)
    sc = upload_scene(hd, ctx, scene)
    cap = H * W * cfg.mask.spp_max
    rid = torch.full((cap,), -7, dtype=torch.int32, device=DEV)
    rz = torch.zeros(cap, dtype=torch.float32, device=DEV)
    offs = excl_cumsum(spp).astype(np.int32)
    total = np.array([spp.sum()], np.int32)
    out = hd.hdof_trace_thin_lens(ctx, sc, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens), hd.light_of(cfg.light),
                                  cfg.mask.spp_max, to_dev(spp.astype(np.uint8)), to_dev(offs), to_dev(total),
                                  seed=11, frame=2, view=1, ray_tri_id=rid, ray_depth=rz)
    torch.cuda.synchronize()
    ctx.sync()
    nr = int(total[0])
    g_id = rid.cpu().numpy()[:nr]
    g_z = rz.cpu().numpy()[:nr].astype(np.float64)
    amb = ref["ray_amb"] != 0
    bad = (g_id != ref["ray_id"]) & ~amb
    assert not bad.any(), f"{bad.sum()} of {nr} unambiguous rays hit other triangles"
    same = g_id == ref["ray_id"]
    # fp32 hit distance: relative error grows as 1/cos(incidence) on grazing hits
    rel = np.abs(g_z[same] - ref["ray_z"][same]) / ref["ray_z"][same]
    assert np.quantile(rel, 0.999) < 1e-5 and rel.max() < 1e-3, (np.quantile(rel, 0.999), rel.max())
    # per-pixel results where every ray of the pixel is unambiguous
    ok = (ref["px_amb"] == 0)
    g = {k: getattr(out, k).cpu().numpy().astype(np.float64) for k in ("c_near", "c_far", "hit_ratio", "lum_m1", "lum_m2")}
    h_ref = ref["hit_ratio"]
    assert np.max(np.abs(g["hit_ratio"] - h_ref)[ok]) < 1e-4
    near = g["hit_ratio"] * g["c_near"] - h_ref * ref["c_near"]
    far = (1 - g["hit_ratio"]) * g["c_far"] - (1 - h_ref) * ref["c_far"]
    assert np.max(np.abs(near)[:, ok]) < COL_TOL and np.max(np.abs(far)[:, ok]) < COL_TOL
    for k in ("lum_m1", "lum_m2"):
        assert np.max(np.abs(g[k] - ref[k])[ok]) < COL_TOL
    strong = ok & (h_ref > 0.05) & (h_ref < 0.95)
    assert np.max(np.abs(g["c_near"] - ref["c_near"])[:, strong], initial=0) < COL_TOL
    untraced = spp == 0
    assert np.all(g["hit_ratio"][untraced] == 0) and np.all(g["c_near"][:, untraced] == 0)
    hd.hdof_set_tuning(ctx)
    sc.close()


def _mixed_depth(H, W, cell, seed):
    """Piecewise-constant depth over square cells (0.35..9 m) with a focus-
    plane band: gather radii from 0 to the cap, sharp CoC steps."""
    rng = np.random.default_rng(seed)
    cz = rng.uniform(0.35, 9.0, ((H + cell - 1) // cell, (W + cell - 1) // cell))
    cz[rng.uniform(size=cz.shape) < 0.2] = 2.0
    return np.kron(cz, np.ones((cell, cell)))[:H, :W]


@pytest.mark.parametrize("which", ["tiny_strong", "room_small", "uniform_big_coc", "room_640",
                                   "mixed_radius_t16", "uniform_r30_t16"])
def test_postfilter_matches_oracle(hd, ctx, which):
    """Tiles of 16 stage each tap's 17x17 footprint in LDS (interior blocks
    through buffer loads, border blocks clamped to the edge); tiles of 8
    take the per-lane form."""
    print_case(f"postfilter {which}")
    if which == "tiny_strong":
        scene, cfg = sg.tiny_scene(0), sg.config_tiny(aperture_override=0.2)
    elif which in ("room_640", "mixed_radius_t16"):
        scene, cfg = sg.living_room_scene(0), sg.config_1080p(640, 360)
    else:
        scene, cfg = sg.living_room_scene(0), sg.config_1080p(320, 180)
    ref_gb = oracle.gbuffer(oracle.Scene(scene.verts, scene.albedo), cfg.camera, cfg.lens, cfg.light)
    col, z = f32(ref_gb["color"]), f32(ref_gb["depth"])
    pp = cfg.pp
    if which == "uniform_big_coc":
        z = np.full_like(z, 0.3)
        pp = sg.PPParams(n_taps=32, tile=8, r_cap=20.0, bg_ramp_px=0.5)
    elif which == "mixed_radius_t16":
        z = f32(_mixed_depth(360, 640, 12, 5))
        col = f32(np.random.default_rng(6).uniform(0, 1, (3, 360, 640)))
    elif which == "uniform_r30_t16":
        z = np.full_like(z, 0.3)
        pp = sg.PPParams(n_taps=48, tile=16, r_cap=30.0, bg_ramp_px=1.0)
    ref = oracle.postfilter(cfg.camera, cfg.lens, col, z, pp)
    got = hd.hdof_postfilter(ctx, to_dev(col, torch.float32), to_dev(z, torch.float32), hd.camera_of(cfg.camera),
                             hd.lens_of(cfg.lens), hd.pp_params_of(pp))
    torch.cuda.synchronize()
    err = np.abs(got.cpu().numpy() - ref)
    assert err.max() < COL_TOL, (err.max(), np.unravel_index(err.argmax(), err.shape))


def test_postfilter_zero_aperture_exact(hd, ctx):
    print_case("postfilter A=0")
    cfg = sg.config_tiny(aperture_override=0.0)
    rng = np.random.default_rng(4)
    col = rng.uniform(0, 1, (3, 64, 64)).astype(np.float32)
    z = rng.uniform(0.5, 8, (64, 64)).astype(np.float32)
    got = hd.hdof_postfilter(ctx, to_dev(col), to_dev(z), hd.camera_of(cfg.camera), hd.lens_of(cfg.lens),
                             hd.pp_params_of(cfg.pp))
    assert torch.equal(got.cpu(), torch.from_numpy(col))


def test_composite_matches_oracle(hd, ctx):
    print_case("composite")
    rng = np.random.default_rng(9)
    cfg = sg.config_1080p(97, 61)
    H, W = 61, 97
    z = rng.uniform(0.4, 9.0, (H, W))
    z[:10] = cfg.lens.focus_distance + rng.uniform(-0.03, 0.03, (10, W))   # focus zone and its ramp
    z = f32(z)
    spp = rng.integers(0, 3, (H, W)).astype(np.int32)
    hit = f32(np.where(spp > 0, rng.uniform(0, 1, (H, W)), 0))
    cr, cpp, cn, cf = (f32(rng.uniform(0, 2, (3, H, W))) for _ in range(4))
    for rt_override in (0, 1):
        cp = sg.CompositeParams(h_t=0.5, rt_override=rt_override)
        ref = oracle.composite(cfg.camera, cfg.lens, cr, cpp, z, spp, cn, cf, hit, cp)
        rtres = hd.RTResult(to_dev(cn, torch.float32), to_dev(cf, torch.float32), to_dev(hit, torch.float32),
                            torch.zeros(H, W, device=DEV), torch.zeros(H, W, device=DEV))
        got = hd.hdof_composite(ctx, to_dev(cr, torch.float32), to_dev(cpp, torch.float32), to_dev(z, torch.float32),
                                to_dev(spp.astype(np.uint8)), rtres, hd.camera_of(cfg.camera), hd.lens_of(cfg.lens),
                                hd.composite_params_of(cp))
        torch.cuda.synchronize()
        assert np.max(np.abs(got.cpu().numpy() - ref)) < 1e-5
