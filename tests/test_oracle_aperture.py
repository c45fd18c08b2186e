"""Pins of the oracle's aperture silhouettes and spherical aberration (the
paper's Discussion: bokeh shapes other than the disk through the shape of the
sampling kernel, and the relative weight of its samples).

The polygon sampler is pinned by an independent point-in-polygon test, its
area uniformity and the polar moment of a regular polygon; the traced hit
ratio against the area of the polygon left of a half-plane's shadow line
(clipped by hand); the post-filter's taps by the shape of the blur of one
bright pixel."""
import math

import numpy as np

import scenegen as sg


def _lens_points(orc, cam, lens, n, x=20, y=20, seed=3):
    """Lens-plane coordinates (right, up) and weights of n samples of one pixel."""
    pts, ws = [], []
    for j in range(n):
        O, _, w = orc.lens_ray(cam, lens, x, y, j, seed=seed, weight=True)
        l = O - cam.eye.astype(np.float64)
        pts.append((l @ cam.right.astype(np.float64), l @ cam.up.astype(np.float64)))
        ws.append(w)
    return np.array(pts), np.array(ws)


def _gauge(pts, B, theta, a):
    """Gauge of points w.r.t. the regular B-gon of circumradius a (1 on its
    boundary), from its edge half-planes."""
    g = np.zeros(len(pts))
    for i in range(B):
        mid = theta + (2 * i + 1) * math.pi / B  # outward normal of edge i
        nrm = np.array([math.cos(mid), math.sin(mid)])
        g = np.maximum(g, pts @ nrm / (a * math.cos(math.pi / B)))
    return g


def test_polygon_samples_fill_the_polygon_uniformly(orc):
    cfg = sg.config_tiny(aperture_override=0.2)
    a = cfg.lens.aperture / 2
    for B, theta in ((5, 0.3), (6, 0.0), (3, 1.0)):
        lens = sg.Lens(cfg.lens.focal_length, cfg.lens.aperture, cfg.lens.focus_distance, B, theta, 0.0)
        pts, w = _lens_points(orc, cfg.camera, lens, 4000)
        g = _gauge(pts, B, theta, a)
        assert g.max() <= 1 + 1e-6, (B, g.max())
        assert g.max() > 0.97  # reaches the boundary
        n = len(pts)
        f = (g <= 0.5).mean()  # the half-scale polygon holds a quarter of the area
        assert abs(f - 0.25) < 4 * math.sqrt(0.25 * 0.75 / n), (B, f)
        sect = np.floor(((np.arctan2(pts[:, 1], pts[:, 0]) - theta) % (2 * math.pi)) / (2 * math.pi / B))
        frac = np.bincount(sect.astype(int), minlength=B) / n
        assert np.all(np.abs(frac - 1 / B) < 4 * math.sqrt((1 / B) * (1 - 1 / B) / n)), (B, frac)
        assert np.all(w == 1.0)


def test_aberration_weight_mean_is_the_polar_moment(orc):
    """E[1 + s (2 rho^2 - 1)] with E[rho^2] = 1/2 on the disk and
    (1 + 2 cos^2(pi/B)) / 6 on the regular B-gon of circumradius 1."""
    cfg = sg.config_tiny(aperture_override=0.2)
    for B, s in ((0, 0.8), (0, -0.6), (6, 0.7), (5, -0.9)):
        lens = sg.Lens(cfg.lens.focal_length, cfg.lens.aperture, cfg.lens.focus_distance, B, 0.2, s)
        pts, w = _lens_points(orc, cfg.camera, lens, 6000, seed=8)
        m2 = 0.5 if B == 0 else (1 + 2 * math.cos(math.pi / B) ** 2) / 6
        expect = 1 + s * (2 * m2 - 1)
        sd = w.std() / math.sqrt(len(w))
        assert abs(w.mean() - expect) < 4 * sd + 1e-12, (B, s, w.mean(), expect)
        rho = np.hypot(pts[:, 0], pts[:, 1]) / (cfg.lens.aperture / 2)
        assert np.all(w >= 0) and np.corrcoef(rho, w)[0, 1] * np.sign(s) > 0.9  # rises with rho when s > 0


def _clip_left(poly, lam):
    """The part of a convex polygon (list of (x, y)) with x < lam."""
    out = []
    for i in range(len(poly)):
        p, q = poly[i], poly[(i + 1) % len(poly)]
        pin, qin = p[0] < lam, q[0] < lam
        if pin:
            out.append(p)
        if pin != qin:
            t = (lam - p[0]) / (q[0] - p[0])
            out.append((lam, p[1] + t * (q[1] - p[1])))
    return out


def _area(poly):
    if len(poly) < 3:
        return 0.0
    x = np.array([p[0] for p in poly])
    y = np.array([p[1] for p in poly])
    return 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def test_half_plane_hit_ratio_with_a_polygon(orc):
    """Near occluder over x < 0: a lens point (lx, ly) reaches it iff
    lx < lambda (the disk pin's shadow line), so the hit ratio is the share
    of the polygon's area left of lambda; with aberration, the share of its
    weight (integrated on a fine grid)."""
    z_n, z_f = 0.5, 10.0
    sc = sg.half_plane_scene(z_n, 0.0, z_f)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.2)
    cam, S1 = cfg.camera, cfg.lens.focus_distance
    a = cfg.lens.aperture / 2
    xs = np.arange(20, 44, 3)
    pix = 31 * cam.width + xs
    n_s = 4096
    B, theta = 6, 0.4
    verts = [(a * math.cos(theta + 2 * math.pi * i / B), a * math.sin(theta + 2 * math.pi * i / B)) for i in range(B)]
    area = _area(verts)
    gx, gy = np.meshgrid(np.linspace(-a, a, 1601), np.linspace(-a, a, 1601))
    gp = np.stack([gx.ravel(), gy.ravel()], 1)
    inside = _gauge(gp, B, theta, a) <= 1
    for s in (0.0, 0.8):
        lens = sg.Lens(cfg.lens.focal_length, cfg.lens.aperture, S1, B, theta, s)
        rt = orc.trace(S, cam, lens, cfg.light, np.full(len(xs), n_s), pix=pix, seed=1, per_ray=False)
        wgrid = np.maximum(0, 1 + s * (2 * (gp[:, 0] ** 2 + gp[:, 1] ** 2) / a ** 2 - 1)) * inside
        for k, x in enumerate(xs):
            u = (2 * (x + 0.5) / cam.width - 1) * cam.tan_half_fov_x
            lam = (0.0 - u * z_n) / (1 - z_n / S1)
            if s == 0.0:
                F = _area(_clip_left(verts, lam)) / area
                tol = 0.0
            else:
                F = wgrid[gp[:, 0] < lam].sum() / wgrid.sum()
                tol = 2e-3  # the grid's own error
            h = rt["hit_ratio"][k]
            sd = math.sqrt(max(F * (1 - F), 1e-12) / n_s) * (1.5 if s else 1.0)
            assert abs(h - F) <= 4 * sd + tol, (s, x, h, F)


def test_postfilter_blur_of_a_point_takes_the_polygon(orc):
    """One bright pixel on a black near plane (every CoC radius 40 px): the
    pixels it reaches through the gather's taps are the tap set mirrored
    through it.  With a hexagonal aperture they stay inside the mirrored
    hexagon of circumradius 40 (plus the bilinear footprint) and reach its
    corners; with the disk they bulge past its edges (by 40 (1 - cos 30 deg)
    = 5.4 px at the edge midpoints).  A constant image stays constant
    whatever the shape and aberration."""
    cam = sg.look_camera((0, 0, 0), 0.0, 128, 128)
    H, W = cam.height, cam.width
    base = sg.Lens(0.05, 0.2, 2.0)
    c = -80.0  # in front of the focus plane
    s_px = W / (2 * cam.tan_half_fov_x)
    z = 1.0 / (1.0 / base.focus_distance - c / (base.aperture * s_px))
    assert z > 0 and abs(orc.coc(cam, base, z) - c) < 1e-5
    depth = np.full((H, W), z)
    img = np.zeros((3, H, W))
    img[:, 64, 64] = 1.0
    pp = sg.PPParams(n_taps=256, tile=16, r_cap=64.0)
    B, theta, R = 6, 0.25, 40.0
    g = {}
    for shape in ("disk", "hexagon"):
        lens = base if shape == "disk" else sg.Lens(base.focal_length, base.aperture, base.focus_distance, B, theta)
        out = orc.postfilter(cam, lens, img, depth, pp)[0]
        ys, xs = np.nonzero(out > 1e-9)
        d = np.stack([xs - 64.0, ys - 64.0], 1)
        g[shape] = _gauge(d, B, theta + math.pi, 1.0)  # the mirrored hexagon, in circumradius units
    assert g["hexagon"].max() <= R + 2.0, g["hexagon"].max()
    assert g["hexagon"].max() >= R - 3.0, g["hexagon"].max()
    assert g["disk"].max() > R + 3.0, g["disk"].max()
    for s in (-0.8, 0.9):
        lens = sg.Lens(base.focal_length, base.aperture, base.focus_distance, 5, 0.1, s)
        const = orc.postfilter(cam, lens, np.full((3, H, W), 0.42), depth, sg.PPParams())
        assert np.allclose(const, 0.42, atol=1e-12)


def test_postfilter_aberration_weights_the_rim(orc):
    """The blur of one bright pixel under spherical aberration: the taps at
    the rim of the kernel (|d| > 0.8 R) carry weight 1 + s (2 rho^2 - 1)
    against the inner ones (|d| < 0.4 R), so the rim of the bokeh is brighter
    than its centre for s > 0 and dimmer for s < 0 (even for s = 0)."""
    cam = sg.look_camera((0, 0, 0), 0.0, 128, 128)
    H, W = cam.height, cam.width
    base = sg.Lens(0.05, 0.2, 2.0)
    s_px = W / (2 * cam.tan_half_fov_x)
    z = 1.0 / (1.0 / base.focus_distance + 60.0 / (base.aperture * s_px))  # CoC -60: radius 30
    depth = np.full((H, W), z)
    img = np.zeros((3, H, W))
    img[:, 64, 64] = 1.0
    pp = sg.PPParams(n_taps=256, tile=16, r_cap=64.0)
    for s, lo, hi in ((0.0, 0.8, 1.25), (0.9, 2.0, 1e9), (-0.9, 0.0, 0.5)):
        out = orc.postfilter(cam, sg.Lens(base.focal_length, base.aperture, base.focus_distance, 0, 0.0, s),
                             img, depth, pp)[0]
        ys, xs = np.nonzero(out > 1e-9)
        r = np.hypot(xs - 64.0, ys - 64.0)
        v = out[ys, xs]
        ratio = v[r > 24].mean() / v[r < 12].mean()
        assert lo < ratio < hi, (s, ratio)
