"""Pins of the post-filter's per-tap weighting where the tap's CoC differs
from the centre's (paper, Design: the adapted gather filter; Reconstruction:
a sample whose CoC radius is below its distance is rejected).

Hand-worked cases with two taps (N = 2) on a 32x32 image: every pixel's
gather radius is then the image's largest CoC radius (the 16-px tiles all
lie within the ceil(64/16)-tile dilation).  The taps are the golden-angle
pair u_1 = 0.5 (cos g, sin g), u_2 = sqrt(3/4) (cos 2g, sin 2g),
g = pi (3 - sqrt 5): u_1 = (-0.36868, 0.33775), u_2 = (0.07571, -0.86271).
A tap at offset R u from pixel p reads the 2x2 texels from
p + floor(R u) with bilinear fractions R u - floor(R u).

The cases separate the rules a plausible slip would merge: the tap weight's
1/max(r_q, 0.5)^2 (not the centre's r_p), the background clamp's ramp over
one pixel of signed CoC (not half of one), the acceptance ramp
clamp(r_eff - d + 0.5, 0, 1), and the centre weight 1/max(r_p, 0.5)^2."""
import math

import numpy as np
import pytest

import scenegen as sg

W = H = 32
G = math.pi * (3.0 - math.sqrt(5.0))
U1 = 0.5 * np.array([math.cos(G), math.sin(G)])
U2 = math.sqrt(0.75) * np.array([math.cos(2 * G), math.sin(2 * G)])
P = (16, 16)  # the pixel under test (x, y)


def _setup():
    cfg = sg.config_tiny(aperture_override=0.2)
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    return cam, cfg.lens


def _depth_of_coc(cam, lens, c):
    """Axial depth whose signed CoC diameter is c px (thin lens with the
    interface's single-precision aperture, focus and field of view)."""
    A = float(np.float32(lens.aperture))
    S1 = float(np.float32(lens.focus_distance))
    s_px = W / (2.0 * float(np.float32(cam.tan_half_fov_x)))
    return 1.0 / (1.0 / S1 - c / (A * s_px))


def _run(orc, cmap, colour):
    cam, lens = _setup()
    depth = np.vectorize(lambda c: _depth_of_coc(cam, lens, c))(cmap)
    for c in np.unique(cmap):
        assert abs(orc.coc(cam, lens, _depth_of_coc(cam, lens, c)) - c) < 1e-9
    pp = sg.PPParams(n_taps=2, tile=16, r_cap=64.0, bg_ramp_px=1.0)
    return orc.postfilter(cam, lens, colour, depth, pp)


def test_tap_offsets_and_footprints():
    """The numbers the cases below rely on: R = 3.5 puts tap 2's footprint at
    rows y - 4, y - 3 and columns x, x + 1 (fractions 0.26500, 0.98052), tap 1's
    at rows y + 1, y + 2 and columns x - 2, x - 1."""
    o1, o2 = 3.5 * U1, 3.5 * U2
    assert np.allclose(U1, [-0.36868, 0.33775], atol=1e-5) and np.allclose(U2, [0.07571, -0.86271], atol=1e-5)
    assert tuple(np.floor(o2).astype(int)) == (0, -4) and tuple(np.floor(o1).astype(int)) == (-2, 1)
    assert np.allclose(o2 - np.floor(o2), [0.26500, 0.98052], atol=1e-5)


def test_near_tap_weighted_by_its_own_radius(orc):
    """Background pixel (c_p = 2, r_p = 1) under a near half-plane (rows
    y <= 13: c_q = -7, r_q = 3.5).  R = 3.5.  Tap 2 lies wholly in the near
    region: t = 0 (nearer), r_eff = 3.5, d = 3.5 sqrt(3/4) = 3.03109,
    a_2 = 3.5 - 3.03109 + 0.5 = 0.96891, w_2 = a_2 (R^2/2) / 3.5^2 = 0.48446.
    Tap 1 stays in the background: r_eff = 1, d = 1.75, a_1 = 0 (rejected).
    Centre w_0 = 1.  Colour 0 in the background, 1 in the near region:
    out = w_2 / (w_0 + w_2) = 0.32636.  With r_p in place of r_q in w_2 the
    answer would be 0.85589."""
    cmap = np.full((H, W), 2.0)
    cmap[: P[1] - 2, :] = -7.0
    col = np.zeros((3, H, W))
    col[:, : P[1] - 2, :] = 1.0
    out = _run(orc, cmap, col)
    d2 = 3.5 * math.sqrt(0.75)
    a2 = 3.5 - d2 + 0.5
    w2 = a2 * (3.5 ** 2 / 2) / 3.5 ** 2
    assert abs(a2 - 0.96891) < 1e-5 and abs(w2 - 0.48446) < 1e-5
    expect = w2 / (1.0 + w2)
    assert abs(expect - 0.32636) < 1e-5
    assert np.allclose(out[:, P[1], P[0]], expect, atol=1e-9), out[:, P[1], P[0]]


def test_background_clamp_mid_ramp(orc):
    """Far pixel (c_p = 6.5, r_p = 3.25) below a farther half-plane (rows
    y <= 13: c_q = 7, r_q = 3.5).  R = 3.5.  Tap 2 reads the farther region:
    t = clamp((7 - 6.5) / 1, 0, 1) = 0.5, r_eff = 3.5 - 0.5 (3.5 - 3.25) =
    3.375, a_2 = 3.375 - 3.03109 + 0.5 = 0.84391, w_2 = a_2 (6.125 / 12.25) =
    0.42196.  Tap 1 reads the pixel's own region: t = 0, r_eff = 3.25,
    d = 1.75, a_1 = 1, w_1 = 6.125 / 3.25^2 = 0.57988.  Centre
    w_0 = 1 / 3.25^2 = 0.09467.  Colours: 1 in the farther region, 0 else:
    out = w_2 / (w_0 + w_1 + w_2) = 0.38482.  A ramp of half a pixel
    (t = 1) gives 0.34763; r_p in w_2's denominator gives 0.42045."""
    cmap = np.full((H, W), 6.5)
    cmap[: P[1] - 2, :] = 7.0
    col = np.zeros((3, H, W))
    col[:, : P[1] - 2, :] = 1.0
    out = _run(orc, cmap, col)
    w0, w1 = 1 / 3.25 ** 2, 6.125 / 3.25 ** 2
    a2 = 3.375 - 3.5 * math.sqrt(0.75) + 0.5
    w2 = a2 * 6.125 / 12.25
    expect = w2 / (w0 + w1 + w2)
    assert abs(expect - 0.38482) < 1e-5
    assert np.allclose(out[:, P[1], P[0]], expect, atol=1e-9), out[:, P[1], P[0]]


def test_impulse_gives_the_tap_weight_pattern(orc):
    """Uniform CoC 7 (r = R = 3.5): every tap is accepted with a_1 = 1,
    a_2 = 0.96891, w_k = a_k / 2, centre w_0 = 1/12.25.  An impulse of 1 at
    texel i = (16, 16) reaches pixel p with weight w / W_p for every tap
    whose footprint covers i: tap 2 from p = i - (0, -4) - (dx, dy) with
    bilinear factors (1 - 0.26500, 0.26500) x (1 - 0.98052, 0.98052), tap 1
    from p = i - (-2, 1) - (dx, dy) with fractions (0.70960, 0.18211); the
    centre at p = i.  Every other pixel reads 0 exactly."""
    cmap = np.full((H, W), 7.0)
    col = np.zeros((3, H, W))
    col[:, 16, 16] = 1.0
    out = _run(orc, cmap, col)[0]
    a2 = 3.5 - 3.5 * math.sqrt(0.75) + 0.5
    w0, w1, w2 = 1 / 12.25, 0.5, a2 / 2
    Wp = w0 + w1 + w2
    expect = np.zeros((H, W))
    expect[16, 16] += w0 / Wp
    for (w, off) in ((w1, 3.5 * U1), (w2, 3.5 * U2)):
        fl = np.floor(off).astype(int)
        fx, fy = off - fl
        for dx, bx in ((0, 1 - fx), (1, fx)):
            for dy, by in ((0, 1 - fy), (1, fy)):
                px, py = 16 - fl[0] - dx, 16 - fl[1] - dy
                expect[py, px] += w * bx * by / Wp
    assert np.allclose(out, expect, atol=1e-12), np.argwhere(np.abs(out - expect) > 1e-12)
    assert np.count_nonzero(out) == 9
    # the pattern sums to the weight the impulse's texel carries over all
    # the gathers that read it, which for a uniform field is the total
    # bilinear mass of the taps (1 each) plus the centre, over W_p
    assert abs(out.sum() - (w0 + w1 + w2) / Wp) < 1e-12
