"""Pins of the oracle's specular materials and the composite's specular
bokeh rule (paper, Composite: near traced pixels favour the post-process
colour by the post-filtered specular intensity).

The highlight is pinned at the mirror point of a floor, where the half
vector equals the normal and the lobe takes its peak k_s I / d^2 whatever
the shininess; the composite rule by its limits and one interior value."""

import numpy as np

import scenegen as sg


def _floor_scene(ks, shin, albedo=(0.4, 0.5, 0.6)):
    big = 50.0
    floor = np.array([[-big, -1.0, -big, big, -1.0, big, big, -1.0, -big],
                      [-big, -1.0, -big, -big, -1.0, big, big, -1.0, big]])
    return floor, np.array([albedo] * 2), np.array([[ks, shin]] * 2)


def _mirror_camera():
    """33x33 camera at the origin whose centre pixel looks at the floor's
    mirror point of a light at (0, 1, 4): P = (0, -1, 4/3)."""
    fwd = np.array([0.0, -0.6, 0.8])
    return sg.Camera(np.zeros(3, np.float32), np.array([1, 0, 0], np.float32), np.array([0, 0.8, 0.6], np.float32),
                     fwd.astype(np.float32), 0.3, 33, 33)


def test_highlight_at_the_mirror_point(orc):
    verts, alb, spec = _floor_scene(0.7, 50.0)
    light = sg.Light(np.array([0, 1, 4], np.float32), np.array([3.0, 2.0, 1.0], np.float32),
                     np.array([0.05, 0.05, 0.05], np.float32))
    cam = _mirror_camera()
    lens = sg.Lens(0.05, 0.0, 2.0)
    S = orc.Scene(verts, alb, spec)
    gb = orc.gbuffer(S, cam, lens, light)
    # P = (0, -1, 4/3): |L - P|^2 = 4 + (8/3)^2 = 100/9, n.l = 0.6, n.h = 1
    d2 = 100.0 / 9.0
    I = light.intensity.astype(np.float64)
    Ls = 0.7 * I / d2
    Ld = np.array(alb[0]) * (light.ambient.astype(np.float64) + I * 0.6 / d2)
    c = gb["color"][:, 16, 16]
    assert np.allclose(c, Ld + Ls, rtol=1e-5), (c, Ld + Ls)
    ys = 0.2126 * Ls[0] + 0.7152 * Ls[1] + 0.0722 * Ls[2]
    assert abs(gb["spec"][16, 16] - ys) < 1e-5 * ys
    # n.h = 1 there: the value does not depend on the shininess (it does elsewhere)
    g5 = orc.gbuffer(orc.Scene(verts, alb, _floor_scene(0.7, 5.0)[2]), cam, lens, light)
    assert abs(g5["spec"][16, 16] - gb["spec"][16, 16]) < 1e-9 * ys
    assert abs(g5["spec"][10, 16] - gb["spec"][10, 16]) > 1e-3 * ys
    # Lambertian scene: no specular plane, colour = the diffuse part
    gl = orc.gbuffer(orc.Scene(verts, alb), cam, lens, light)
    assert np.all(gl["spec"] == 0)
    assert np.allclose(gl["color"][:, 16, 16], Ld, rtol=1e-5)
    # k_s = 0 gives the Lambertian image exactly
    g0 = orc.gbuffer(orc.Scene(verts, alb, _floor_scene(0.0, 50.0)[2]), cam, lens, light)
    assert np.array_equal(g0["color"], gl["color"]) and np.all(g0["spec"] == 0)


def test_no_highlight_from_behind(orc):
    """A light below the floor lights its other side: the viewer's side gets
    the ambient term only, no diffuse and no specular part."""
    verts, alb, spec = _floor_scene(0.9, 8.0)
    light = sg.Light(np.array([0, -3, 4], np.float32), np.array([3.0, 3.0, 3.0], np.float32),
                     np.array([0.05, 0.05, 0.05], np.float32))
    gb = orc.gbuffer(orc.Scene(verts, alb, spec), _mirror_camera(), sg.Lens(0.05, 0.0, 2.0), light)
    hit = gb["tri_id"] >= 0
    assert hit.sum() > 500
    assert np.all(gb["spec"][hit] == 0)
    assert np.allclose(gb["color"][:, hit], (np.array(alb[0]) * 0.05)[:, None], rtol=1e-12)


def test_traced_colours_carry_the_highlight(orc):
    """A pinhole lens: every lens ray is the pixel's pinhole ray, so the
    traced colour equals the G-buffer colour, highlight included."""
    verts, alb, spec = _floor_scene(0.7, 50.0)
    light = sg.Light(np.array([0, 1, 4], np.float32), np.array([3.0, 2.0, 1.0], np.float32),
                     np.array([0.05, 0.05, 0.05], np.float32))
    cam, lens = _mirror_camera(), sg.Lens(0.05, 0.0, 2.0)
    S = orc.Scene(verts, alb, spec)
    gb = orc.gbuffer(S, cam, lens, light)
    rt = orc.trace(S, cam, lens, light, np.full((33, 33), 2), seed=1, per_ray=False)
    crt = rt["hit_ratio"] * rt["c_near"] + (1 - rt["hit_ratio"]) * rt["c_far"]
    assert np.allclose(crt, gb["color"], atol=1e-12)


def test_composite_specular_rule(orc):
    """Near traced pixels blend from the traced to the post-process colour
    by sigma = clamp(Y_s,pp / spec_y, 0, 1); far and untraced pixels do not
    see it; spec_y = 0 switches it off."""
    cfg = sg.config_tiny(aperture_override=0.2)
    cam, lens = cfg.camera, cfg.lens
    H, W = cam.height, cam.width
    z = np.full((H, W), 0.3)          # far in front of the 2 m focus: CoC << -sqrt 2, near, phi = 1
    z[:, W // 2:] = 50.0              # behind it: far
    assert orc.coc(cam, lens, 0.3) < -3 and orc.coc(cam, lens, 50.0) > 3
    spp = np.ones((H, W), np.int32)
    spp[: H // 2] = 0
    col = np.zeros((3, H, W))
    cpp = np.full((3, H, W), 0.8)
    cn = np.full((3, H, W), 0.2)
    cf = np.full((3, H, W), 0.4)
    h = np.full((H, W), 1.0)
    spec_y = 0.5
    for ys, sig in ((0.0, 0.0), (0.125, 0.25), (0.5, 1.0), (3.0, 1.0)):
        pps = np.full((H, W), ys)
        cp = sg.CompositeParams(h_t=0.5, rt_override=0, spec_y=spec_y)
        out = orc.composite(cam, lens, col, cpp, z, spp, cn, cf, h, cp, pps)
        near_tr = out[:, H // 2:, : W // 2]
        assert np.allclose(near_tr, 0.2 + sig * (0.8 - 0.2), atol=1e-12), (ys, near_tr.min(), near_tr.max())
        assert np.allclose(out[:, : H // 2, : W // 2], 0.8)  # untraced near: post-process
        base = orc.composite(cam, lens, col, cpp, z, spp, cn, cf, h, sg.CompositeParams(h_t=0.5))
        assert np.array_equal(out[:, :, W // 2:], base[:, :, W // 2:])  # far side unchanged
    off = orc.composite(cam, lens, col, cpp, z, spp, cn, cf, h, sg.CompositeParams(h_t=0.5, spec_y=0.0),
                        np.full((H, W), 9.0))
    assert np.array_equal(off, orc.composite(cam, lens, col, cpp, z, spp, cn, cf, h, sg.CompositeParams(h_t=0.5)))


def test_postfilter_spec_is_the_gather_of_the_specular_plane(orc):
    """A constant specular plane filters to itself (normalised weights); in
    general it is channel for channel the colour gather."""
    cfg = sg.config_tiny(aperture_override=0.2)
    sc = sg.tiny_scene(0)
    gb = orc.gbuffer(orc.Scene(sc.verts, sc.albedo), cfg.camera, cfg.lens, cfg.light)
    c = orc.postfilter_spec(cfg.camera, cfg.lens, np.full((64, 64), 0.37), gb["depth"], cfg.pp)
    assert np.allclose(c, 0.37, atol=1e-12)
    ys = np.random.default_rng(2).uniform(0, 2, (64, 64))
    a = orc.postfilter_spec(cfg.camera, cfg.lens, ys, gb["depth"], cfg.pp)
    b = orc.postfilter(cfg.camera, cfg.lens, np.stack([ys, 0 * ys, ys]), gb["depth"], cfg.pp)
    assert np.array_equal(a, b[0]) and np.array_equal(a, b[2])
    assert not np.allclose(a, ys)
