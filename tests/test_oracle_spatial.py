"""Pins of the oracle's spatial reconstruction of the traced colours (paper,
Reconstruction, last paragraph) and of the per-pixel near/far CoC averages
the trace hands it.

The spatial gather's geometry is pinned by hand-worked single-tap cases
(the first golden-angle tap of a one-tap kernel points at
sqrt(1/2) (cos g, sin g), g = pi (3 - sqrt 5) ~ 137.5 deg, i.e. up-left in
image coordinates), with distractor pixels on every other candidate the tap
could land on after a sign, axis or level slip; the texel sums against numpy
block sums over ragged images; the blend against a constant field and the
variance clamp's limits; the CoC averages against the thin-lens CoC of two
planes.
"""
import math

import numpy as np

import scenegen as sg


def _blank(W=8, H=8):
    spp = np.zeros((H, W), np.int32)
    cn = np.zeros((3, H, W))
    cf = np.zeros((3, H, W))
    h = np.zeros((H, W))
    coc = np.zeros((2, H, W))
    return spp, cn, cf, h, coc


def _put(spp, cn, cf, h, coc, x, y, s, hv, near, far=0.0, r_near=0.0, r_far=0.0):
    spp[y, x] = s
    h[y, x] = hv
    cn[:, y, x] = near
    cf[:, y, x] = far
    coc[0, y, x] = 2.0 * r_near
    coc[1, y, x] = 2.0 * r_far


def test_one_tap_level0_hand_worked(orc):
    """p = (4, 4), r_p = 1, one tap: sqrt(pi) r_p < 2 so level 0; the tap
    lands at (4.5, 4.5) + (-0.521, 0.478) -> pixel (3, 4) at distance
    sqrt(1/2).  With that neighbour's near colour 1 and an equal near weight
    the gathered near colour is 1/2; with the neighbour's CoC radius at
    distance - 1/4 it counts a quarter: 0.5 / 2.5 = 0.2."""
    g = math.pi * (3 - math.sqrt(5))
    u = math.sqrt(0.5) * np.array([math.cos(g), math.sin(g)])
    assert math.floor(4.5 + u[0]) == 3 and math.floor(4.5 + u[1]) == 4
    for r_q, expect in ((5.0, 0.5), (math.sqrt(0.5) - 0.25, 0.2)):
        spp, cn, cf, h, coc = _blank()
        _put(spp, cn, cf, h, coc, 4, 4, 2, 1.0, 0.0, far=0.7, r_near=1.0)
        _put(spp, cn, cf, h, coc, 3, 4, 2, 1.0, 1.0, r_near=r_q)
        # distractors on the cells a sign, axis swap or wrong level would reach
        for (x, y) in ((5, 4), (4, 3), (4, 5), (5, 5), (3, 3), (5, 3), (2, 4)):
            _put(spp, cn, cf, h, coc, x, y, 4, 1.0, 9.0, r_near=5.0)
        out = orc.spatial(spp, cn, cf, h, None, coc, None, n_taps=1, r_cap=64.0)
        assert abs(out["c_near"][0, 4, 4] - expect) < 1e-12, (r_q, out["c_near"][:, 4, 4])
        assert np.allclose(out["c_near"][:, 4, 4], expect, atol=1e-12)
        # no far weight anywhere (h = 1): the far colour stays
        assert np.allclose(out["c_far"][:, 4, 4], 0.7, atol=1e-15)


def test_one_tap_level1_hand_worked(orc):
    """p = (4, 4), r_p = 2, one tap: sqrt(pi) r_p = 3.54 so level 1; the tap
    at (4.5, 4.5) + (-1.043, 0.955) lies in pixel (3, 5), level-1 texel
    (1, 2) = pixels x 2..3, y 4..5, of which (2, 4) (colour 1) and (3, 5)
    (colour 3) are traced with 2 rays each and CoC radius 10: the texel sums
    to 8 over a near weight 4 and is fully accepted: (0 + 8) / (2 + 4) = 4/3
    (level 0 would give 6/4 from pixel (3, 5) alone).  The variance clamp
    then scales the step from the pixel's own colour."""
    spp, cn, cf, h, coc = _blank()
    _put(spp, cn, cf, h, coc, 4, 4, 2, 1.0, 0.0, r_near=2.0)
    _put(spp, cn, cf, h, coc, 2, 4, 2, 1.0, 1.0, r_near=10.0)
    _put(spp, cn, cf, h, coc, 3, 5, 2, 1.0, 3.0, r_near=10.0)
    for (x, y) in ((5, 4), (4, 3), (5, 5), (6, 6), (0, 0)):
        _put(spp, cn, cf, h, coc, x, y, 4, 1.0, 9.0, r_near=5.0)
    vc = 0.01
    for V, lam in ((None, 1.0), (np.inf, 1.0), (vc / 4, 0.25), (0.0, 0.0), (10 * vc, 1.0)):
        Vimg = None if V is None else np.full((8, 8), V)
        out = orc.spatial(spp, cn, cf, h, None, coc, Vimg, n_taps=1, r_cap=64.0, v_clamp=vc)
        assert np.allclose(out["c_near"][:, 4, 4], lam * 4.0 / 3.0, atol=1e-12), (V, out["c_near"][:, 4, 4])


def test_accumulated_hit_ratio_blends_the_radius(orc):
    """r_p = (H cbar_n + (1 - H) cbar_f) / 2 with H the accumulated hit ratio
    when one is given: near CoC 0, far CoC 4, H = 1/2 -> r_p = 1 (the level-0
    case above); with H = 1 (no accumulated ratio given, h = 1) r_p = 0 and
    the single tap sits at the pixel itself (only its own colour)."""
    spp, cn, cf, h, coc = _blank()
    _put(spp, cn, cf, h, coc, 4, 4, 2, 1.0, 0.0, r_near=0.0, r_far=2.0)
    _put(spp, cn, cf, h, coc, 3, 4, 2, 1.0, 1.0, r_near=5.0)
    hacc = np.full((8, 8), 0.5)
    a = orc.spatial(spp, cn, cf, h, hacc, coc, None, n_taps=1)
    b = orc.spatial(spp, cn, cf, h, None, coc, None, n_taps=1)
    assert np.allclose(a["c_near"][:, 4, 4], 0.5, atol=1e-12)
    # r_p = 0: the tap is the pixel itself, counted again (same colour)
    assert np.allclose(b["c_near"][:, 4, 4], 0.0, atol=1e-15)


def test_constant_field_is_invariant(orc):
    """Whatever the radii, weights, levels and variances, a field whose traced
    pixels share one near and one far colour is left as it is."""
    rng = np.random.default_rng(3)
    H, W = 45, 61
    spp = rng.integers(0, 6, (H, W)).astype(np.int32)
    spp[rng.uniform(size=(H, W)) < 0.4] = 0
    h = rng.uniform(0, 1, (H, W))
    h[rng.uniform(size=(H, W)) < 0.2] = 1.0
    cn = np.broadcast_to(np.array([0.3, 0.5, 0.9])[:, None, None], (3, H, W)).copy()
    cf = np.broadcast_to(np.array([1.7, 0.2, 0.4])[:, None, None], (3, H, W)).copy()
    coc = rng.uniform(0, 90, (2, H, W))
    V = rng.uniform(0, 0.03, (H, W))
    V[rng.uniform(size=(H, W)) < 0.1] = np.inf
    out = orc.spatial(spp, cn, cf, h, rng.uniform(0, 1, (H, W)), coc, V, n_taps=24)
    assert np.allclose(out["c_near"], cn, atol=1e-12)
    assert np.allclose(out["c_far"], cf, atol=1e-12)


def test_untraced_and_isolated_pixels_keep_their_colours(orc):
    rng = np.random.default_rng(4)
    H, W = 20, 30
    spp = np.zeros((H, W), np.int32)
    spp[10, 15] = 3
    cn, cf = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    h = rng.uniform(size=(H, W))
    coc = rng.uniform(0, 40, (2, H, W))
    out = orc.spatial(spp, cn, cf, h, None, coc, None, n_taps=24)
    assert np.array_equal(out["c_near"], cn) or np.allclose(out["c_near"], cn, atol=1e-14)
    assert np.allclose(out["c_far"], cf, atol=1e-14)
    # V = 0 everywhere (converged): every pixel keeps its colour exactly
    spp = rng.integers(0, 5, (H, W)).astype(np.int32)
    out = orc.spatial(spp, cn, cf, h, None, coc, np.zeros((H, W)), n_taps=24)
    assert np.array_equal(out["c_near"], cn) and np.array_equal(out["c_far"], cf)


def test_level_sums_match_numpy_block_sums(orc):
    """Texel sums of every level against numpy: pad the ragged image to a
    multiple of 2^L with untraced pixels and sum 2^L x 2^L blocks."""
    rng = np.random.default_rng(6)
    H, W = 23, 37
    spp = rng.integers(0, 4, (H, W)).astype(np.int32)
    cn, cf = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    h = rng.uniform(size=(H, W))
    hacc = rng.uniform(size=(H, W))
    coc = rng.uniform(0, 150, (2, H, W))
    r_cap = 40.0
    s = spp.astype(np.float64)
    r = np.minimum(r_cap, 0.5 * (hacc * coc[0] + (1 - hacc) * coc[1]))
    t = (spp > 0).astype(np.float64)
    planes = np.concatenate([s * h * cn, (s * h)[None], s * (1 - h) * cf, (s * (1 - h))[None],
                             (t * r)[None], t[None]])
    for L in range(orc.SP_LMAX + 1):
        b = 1 << L
        HL, WL = -(-H // b), -(-W // b)
        pad = np.zeros((10, HL * b, WL * b))
        pad[:, :H, :W] = planes
        ref = pad.reshape(10, HL, b, WL, b).sum(axis=(2, 4))
        got = orc.sp_level(spp, cn, cf, h, hacc, coc, r_cap, L)
        assert got.shape == ref.shape
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12), L


def test_coc_averages_of_two_planes(orc):
    """Half-plane occluder at z_n over a wall at z_f: a pixel's near rays all
    hit z_n and its far rays z_f, so the averages are the thin-lens CoC
    magnitudes of the two depths (the near one is negative: the average is
    of |c|); with a zero aperture both are 0."""
    z_n, z_f = 0.5, 10.0
    sc = sg.half_plane_scene(z_n, 0.0, z_f)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.2)
    cam, lens, light = cfg.camera, cfg.lens, cfg.light
    cn_, cf_ = abs(orc.coc(cam, lens, z_n)), abs(orc.coc(cam, lens, z_f))
    assert orc.coc(cam, lens, z_n) < -2 and orc.coc(cam, lens, z_f) > 2
    # thin lens: |c| = A s_px |1/S1 - 1/z| (s_px = W / (2 tan(fov/2)))
    s_px = cam.width / (2 * cam.tan_half_fov_x)
    assert abs(cn_ - lens.aperture * s_px * abs(1 / lens.focus_distance - 1 / z_n)) < 1e-4 * cn_
    xs = np.arange(20, 44)
    pix = 31 * cam.width + xs
    rt = orc.trace(S, cam, lens, light, np.full(len(xs), 64), pix=pix, seed=2, per_ray=False)
    h = rt["hit_ratio"]
    both = (h > 0) & (h < 1)
    assert both.sum() >= 4
    assert np.allclose(rt["coc_nf"][0][h > 0], cn_, rtol=1e-9)
    assert np.allclose(rt["coc_nf"][1][h < 1], cf_, rtol=1e-9)
    assert np.all(rt["coc_nf"][0][h == 0] == 0) and np.all(rt["coc_nf"][1][h == 1] == 0)
    pin = sg.config_tiny(aperture_override=0.0)
    rt0 = orc.trace(S, pin.camera, pin.lens, pin.light, np.full(len(xs), 4), pix=pix, seed=2, per_ray=False)
    assert np.all(rt0["coc_nf"] == 0)


def test_frame_applies_spatial_after_the_trace(orc):
    """oracle.frame with the spatial stage on equals the stage applied by hand
    to the same frame's trace with the updated history's variance; off, the
    traced colours pass through."""
    from dataclasses import replace
    sc = sg.tiny_scene(0)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.2)
    off = orc.frame(S, cfg)
    on = orc.frame(S, replace(cfg, spatial=sg.SpatialParams(enable=True, n_taps=16)))
    rt = off["rt"]
    assert (off["spp"] > 0).sum() > 50
    V = orc.history_variance(off["history"])
    assert np.all(np.isinf(V[off["spp"] > 0]))  # first frame: every traced pixel is new
    ref = orc.spatial(off["spp"], rt["c_near"], rt["c_far"], rt["hit_ratio"], None, rt["coc_nf"], V, n_taps=16)
    assert np.array_equal(on["rt"]["c_near"], ref["c_near"])
    assert np.array_equal(on["rt"]["c_far"], ref["c_far"])
    assert not np.array_equal(on["rt"]["c_near"], rt["c_near"])


def test_ambiguity_flags_and_conditioning(orc):
    """The oracle's flags of the integer decisions and its conditioning
    figure, on the one-tap cases worked by hand above.

    Level: with one tap the spacing is r_p sqrt(pi); r_p = 4 / sqrt(pi)
    puts it on the level-2 boundary (flag 1), 0.1 % away it is clear.
    Tap coordinate: r_p = -0.5 / u_x puts the tap's x on 4.0 (flag 2); the
    band is 1e-5 + 2^-20 (|x + 0.5| + |r_p u_x|), so an offset of 1e-4 px
    is flagged at x ~ 1000 but not at x = 4.
    Conditioning: a tap whose acceptance sits on the ramp (a = 1/4) counts
    its near weight 2 over the accepted 2 + 2/4: 0.8; a fully accepted tap
    (argument 4.8) counts nothing."""
    g = math.pi * (3 - math.sqrt(5))
    ux, uy = math.sqrt(0.5) * math.cos(g), math.sqrt(0.5) * math.sin(g)

    def one(x, y, r_p, W=8, H=8, r_q=5.0):
        spp, cn, cf, h, coc = _blank(W, H)
        _put(spp, cn, cf, h, coc, x, y, 2, 1.0, 0.0, r_near=r_p)
        tx = min(max(math.floor(x + 0.5 + r_p * ux), 0), W - 1)
        ty = min(max(math.floor(y + 0.5 + r_p * uy), 0), H - 1)
        if (tx, ty) != (x, y):
            _put(spp, cn, cf, h, coc, tx, ty, 2, 1.0, 1.0, r_near=r_q)
        return orc.spatial(spp, cn, cf, h, None, coc, None, n_taps=1, r_cap=64.0)

    r_lvl = 4.0 / math.sqrt(math.pi)
    assert one(4, 4, r_lvl)["amb"][4, 4] & 1
    assert not one(4, 4, r_lvl * 1.001)["amb"][4, 4] & 1
    r_tap = -0.5 / ux
    assert abs(4.5 + r_tap * uy - round(4.5 + r_tap * uy)) > 0.01
    assert one(4, 4, r_tap)["amb"][4, 4] & 2
    assert one(4, 4, r_tap * 1.01)["amb"][4, 4] == 0
    # 1e-4 px from a pixel boundary: flagged far from the origin, clear near it
    W = 1100
    r_far = (1000.0 - 1e-4 - 1000.5) / ux
    assert 1000.5 + r_far * ux < 1000.0 and one(1000, 4, r_far, W=W)["amb"][4, 1000] & 2
    r_near = (4.0 - 1e-4 - 4.5) / ux
    assert one(4, 4, r_near)["amb"][4, 4] == 0
    # conditioning of the near output
    out = one(4, 4, 1.0, r_q=math.sqrt(0.5) - 0.25)
    assert abs(out["cond"][0, 4, 4] - 0.8) < 1e-12 and abs(out["c_near"][0, 4, 4] - 0.2) < 1e-12
    assert one(4, 4, 1.0, r_q=5.0)["cond"][0, 4, 4] == 0.0
    # untraced pixels carry neither flags nor conditioning
    assert out["amb"][0, 0] == 0 and out["cond"][:, 0, 0].max() == 0.0
