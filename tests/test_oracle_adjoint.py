"""Pins of the oracle's adjoint of post-filter + composite: the colour
gradient is the exact transpose of the (linear in colour) forward map
(dot-product test, directional differences), and the focus-distance and
aperture gradients match central finite differences of the oracle's own
forward pass."""
import numpy as np
import pytest

import oracle as orc
import scenegen as sg


def _problem(seed=0, W=48, H=40):
    rng = np.random.default_rng(seed)
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    lens = sg.Lens(0.05, 0.04, 2.0)
    yy, xx = np.mgrid[0:H, 0:W]
    z = np.where(xx < W * 0.45, 0.7, 4.0) + 0.3 * np.sin(yy / 5.0)       # near object over a far wall
    z[5:12, 30:40] = 2.0                                                  # an in-focus patch
    col = rng.uniform(0, 1, (3, H, W))
    spp = rng.integers(0, 3, (H, W)).astype(np.int32)
    hit = np.where(spp > 0, rng.uniform(0, 1, (H, W)), 0.0)
    cn, cf = rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (3, H, W))
    pp = sg.PPParams(n_taps=24, tile=8, r_cap=12.0, bg_ramp_px=1.0)
    cp = sg.CompositeParams()
    return cam, lens, col, z, spp, cn, cf, hit, pp, cp, rng


def _fwd(cam, lens, col, z, spp, cn, cf, hit, pp, cp):
    return orc.pp_composite_forward(cam, lens, col, z, spp, cn, cf, hit, pp, cp)


def test_colour_gradient_is_transpose():
    cam, lens, col, z, spp, cn, cf, hit, pp, cp, rng = _problem()
    x = rng.normal(size=col.shape)
    y = rng.normal(size=col.shape)
    base = _fwd(cam, lens, np.zeros_like(col), z, spp, cn, cf, hit, pp, cp)
    Mx = _fwd(cam, lens, x, z, spp, cn, cf, hit, pp, cp) - base
    MTy, _, _ = orc.pp_composite_backward(cam, lens, col, z, spp, cn, cf, hit, pp, cp, y)
    lhs, rhs = np.sum(Mx * y), np.sum(x * MTy)
    assert abs(lhs - rhs) < 1e-9 * max(1.0, abs(lhs))


def test_colour_gradient_directional_difference():
    cam, lens, col, z, spp, cn, cf, hit, pp, cp, rng = _problem(1)
    g = rng.normal(size=col.shape)
    v = rng.normal(size=col.shape)
    gc, _, _ = orc.pp_composite_backward(cam, lens, col, z, spp, cn, cf, hit, pp, cp, g)
    h = 1e-4
    Lp = np.sum(g * _fwd(cam, lens, col + h * v, z, spp, cn, cf, hit, pp, cp))
    Lm = np.sum(g * _fwd(cam, lens, col - h * v, z, spp, cn, cf, hit, pp, cp))
    assert abs((Lp - Lm) / (2 * h) - np.sum(gc * v)) < 1e-8 * max(1.0, abs(np.sum(gc * v)))


@pytest.mark.parametrize("seed", [0, 2, 3])
def test_lens_gradients_match_central_differences(seed):
    cam, lens, col, z, spp, cn, cf, hit, pp, cp, rng = _problem(seed)
    g = rng.normal(size=col.shape)
    _, gs, ga = orc.pp_composite_backward(cam, lens, col, z, spp, cn, cf, hit, pp, cp, g)
    def L(S1, A):
        return np.sum(g * _fwd(cam, sg.Lens(lens.focal_length, A, S1), col, z, spp, cn, cf, hit, pp, cp))
    # the interface carries float32 lens values: step between representable values
    S1, A = np.float32(lens.focus_distance), np.float32(lens.aperture)
    Sp, Sm = np.float32(S1 + 1e-4), np.float32(S1 - 1e-4)
    Ap, Am = np.float32(A + 1e-5), np.float32(A - 1e-5)
    fs = (L(float(Sp), float(A)) - L(float(Sm), float(A))) / (float(Sp) - float(Sm))
    fa = (L(float(S1), float(Ap)) - L(float(S1), float(Am))) / (float(Ap) - float(Am))
    assert abs(gs - fs) <= 1e-5 * abs(fs), (gs, fs)
    assert abs(ga - fa) <= 1e-5 * abs(fa), (ga, fa)
