"""Pins of the FP64 oracle against things other than itself.

Each test ties one oracle function to a library routine, a closed form of the
thin-lens model, brute force on a tiny input, or an invariant the paper's
method fixes, chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a swapped operand) fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.special as sps

import scenegen as sg

SQ2 = math.sqrt(2.0)


# ----------------------------------------------------------------------------
# counter-based generator: bit-exact against numpy's Philox4x64-10
# ----------------------------------------------------------------------------

def _numpy_philox(ctr, key):
    """numpy.random.Philox increments its 256-bit counter before each block,
    so the block for counter C is the first output after setting C - 1."""
    C = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    K = sum(int(k) << (64 * i) for i, k in enumerate(key))
    bg = np.random.Philox(counter=(C - 1) % (1 << 256), key=K)
    return bg.random_raw(4).astype(np.uint64)


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(123)
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 0, 0, 0], [0, 0]),
             ([2**64 - 1] * 4, [2**64 - 1] * 2), ([5, 3, 7, 0], [11, 13])]
    for _ in range(200):
        cases.append((rng.integers(0, 2**63, 4, dtype=np.uint64).tolist(),
                      rng.integers(0, 2**63, 2, dtype=np.uint64).tolist()))
    for ctr, key in cases:
        if all(int(c) == 0 for c in ctr):
            continue  # numpy cannot be positioned before counter 0 without wrap
        got = orc.philox4x64_10(ctr, key)
        exp = _numpy_philox(ctr, key)
        assert np.array_equal(got, exp), (ctr, key, got, exp)


def test_lens_uniforms_uniform_disk(orc):
    """Lens points are uniform on the disk of radius A/2: radial CDF r^2/a^2
    and uniform angle (Kolmogorov-Smirnov bounds at 4096 samples)."""
    cfg = sg.config_tiny(aperture_override=0.2)
    a = cfg.lens.aperture / 2
    e = cfg.camera.eye.astype(np.float64)
    r2, th = [], []
    for j in range(4096):
        O, _ = orc.lens_ray(cfg.camera, cfg.lens, 10, 20, j, seed=3, frame=1)
        l = O - e
        lx = l @ cfg.camera.right.astype(np.float64)
        ly = l @ cfg.camera.up.astype(np.float64)
        r2.append((lx * lx + ly * ly) / (a * a))
        th.append((math.atan2(ly, lx) / (2 * math.pi)) % 1.0)
    for v in (np.sort(r2), np.sort(th)):
        ecdf = np.arange(1, len(v) + 1) / len(v)
        assert np.max(np.abs(ecdf - v)) < 1.63 / math.sqrt(len(v)) * 1.5
    assert max(r2) <= 1.0 + 1e-12


# ----------------------------------------------------------------------------
# thin lens: Potmesil CoC, pinhole limit, focus plane
# ----------------------------------------------------------------------------

def test_coc_matches_potmesil(orc):
    """Potmesil & Chakravarty: image-plane CoC diameter A f |z - S1| / (z (S1 - f))
    at image distance f S1 / (S1 - f); in pixels of a sensor of half-width
    tan_half_fov_x * image distance spanning W pixels."""
    cfg = sg.config_1080p()
    f, A, S1 = cfg.lens.focal_length, cfg.lens.aperture, cfg.lens.focus_distance
    W, tx = cfg.camera.width, cfg.camera.tan_half_fov_x
    vi = f * S1 / (S1 - f)
    for z in [0.5, 0.6, 1.0, 1.94, 2.0, 2.06, 2.5, 6.0, 1e4]:
        c_sensor = A * f * abs(z - S1) / (z * (S1 - f))
        c_px = c_sensor * W / (2 * tx * vi)
        got = orc.coc(cfg.camera, cfg.lens, z)
        assert abs(abs(got) - c_px) < 1e-9 * max(1, c_px)
        assert (got < 0) == (z < S1) or z == S1


def test_lens_ray_spread_is_coc(orc):
    """Lens rays of one pixel meet the plane at depth z in points whose pinhole
    images spread over a disk of diameter |c(z)| pixels; at z = S1 they meet
    in one point."""
    cfg = sg.config_tiny(aperture_override=0.2)
    cam = cfg.camera
    w, r, u = (cam.fwd.astype(np.float64), cam.right.astype(np.float64), cam.up.astype(np.float64))
    e = cam.eye.astype(np.float64)
    spx = cam.width / (2 * cam.tan_half_fov_x)
    for z in [0.7, 2.0, 5.0]:
        pts = []
        for j in range(2048):
            O, D = orc.lens_ray(cam, cfg.lens, 40, 17, j, seed=9)
            t = (z - (O - e) @ w) / (D @ w)
            P = O + t * D - e
            pts.append([spx * (P @ r) / (P @ w), spx * (P @ u) / (P @ w)])
        pts = np.array(pts)
        # the disk is centred on the pixel's own pinhole image
        ctr = np.array([(2 * 40.5 / cam.width - 1) * cam.tan_half_fov_x,
                        (1 - 2 * 17.5 / cam.height) * cam.tan_half_fov_x * cam.height / cam.width]) * spx
        spread = np.max(np.linalg.norm(pts - ctr, axis=1)) * 2
        c = abs(orc.coc(cam, cfg.lens, z))
        if z == 2.0:
            assert spread < 1e-9
        else:
            assert 0.97 * c < spread <= c * (1 + 1e-9)


def test_zero_aperture_is_pinhole(orc):
    cfg = sg.config_tiny(aperture_override=0.0)
    cam = cfg.camera
    for (x, y, j) in [(0, 0, 0), (13, 51, 3), (63, 63, 7)]:
        O, D = orc.lens_ray(cam, cfg.lens, x, y, j, seed=5)
        Op, Dp = orc.lens_ray(cam, cfg.lens, x, y, 0, pinhole=True)
        assert np.array_equal(O, Op) and np.array_equal(D, Dp)
        assert np.array_equal(O, cam.eye.astype(np.float64))
        # D = S1 v with v the pixel's pinhole direction (unit forward component)
        assert abs(D @ cam.fwd.astype(np.float64) - cfg.lens.focus_distance) < 1e-12


# ----------------------------------------------------------------------------
# closest hit
# ----------------------------------------------------------------------------

def _brute_numpy(verts, O, D):
    """Closest hit by solving [-D, e1, e2] (t, b1, b2) = O - v0 for every pair
    (textbook barycentric system via numpy.linalg.solve)."""
    v0, v1, v2 = verts[:, 0:3], verts[:, 3:6], verts[:, 6:9]
    e1, e2 = v1 - v0, v2 - v0
    n_r, n_t = O.shape[0], verts.shape[0]
    M = np.empty((n_r, n_t, 3, 3))
    M[..., 0] = -D[:, None, :]
    M[..., 1] = e1[None]
    M[..., 2] = e2[None]
    rhs = O[:, None, :] - v0[None]
    det = np.linalg.det(M)
    ok = np.abs(det) > 1e-14
    M[~ok] = np.eye(3)
    sol = np.linalg.solve(M, rhs[..., None])[..., 0]
    t, b1, b2 = sol[..., 0], sol[..., 1], sol[..., 2]
    hit = ok & (t > 0) & (b1 >= 0) & (b2 >= 0) & (b1 + b2 <= 1)
    tt = np.where(hit, t, np.inf)
    idx = np.argmin(tt, axis=1)
    tmin = tt[np.arange(n_r), idx]
    idx = np.where(np.isinf(tmin), -1, idx)
    return tmin, idx


def test_closest_hit_matches_brute_force(orc):
    sc = sg.tiny_scene(0)
    S = orc.Scene(sc.verts, sc.albedo)
    rng = np.random.default_rng(0)
    n = 600
    O = np.concatenate([rng.uniform(-0.3, 0.3, (n, 2)), rng.uniform(-0.5, 0.2, (n, 1))], 1)
    D = np.concatenate([rng.uniform(-0.6, 0.6, (n, 2)), np.ones((n, 1)) * rng.uniform(0.5, 2, (n, 1))], 1)
    t, i, a = S.cast(O, D)
    tb, ib, ab = S.cast(O, D, brute=True)
    assert np.array_equal(i, ib) and np.array_equal(a, ab)
    tn, inp = _brute_numpy(sc.verts.astype(np.float64), O, D)
    ok = a == 0
    assert ok.mean() > 0.95
    assert np.array_equal(i[ok], inp[ok])
    assert np.allclose(t[ok], tn[ok], rtol=1e-9, atol=0)


def test_watertight_shared_edges_and_vertices(orc):
    """Rays aimed exactly at shared edges and vertices of a closed tessellated
    box hit the box (never the room behind it)."""
    box = sg.grid_box((0.0, 0.0, 3.0), 0.5, 4)
    room = sg.room_box((-5, -5, -5), (5, 5, 10))
    verts = np.concatenate([box, room]).astype(np.float32).astype(np.float64)
    S = orc.Scene(verts, np.full((verts.shape[0], 3), 0.5))
    targets = []
    front = [t.reshape(3, 3) for t in box if np.all(t.reshape(3, 3)[:, 2] == 2.5)]
    assert len(front) == 32
    for v in front:
        for p in [v[0], v[1], v[2], 0.5 * (v[0] + v[1]), 0.5 * (v[1] + v[2]), 0.5 * (v[0] + v[2])]:
            if abs(p[0]) < 0.5 and abs(p[1]) < 0.5:   # interior of the visible face
                targets.append(p)
    T = np.array(targets)
    assert len(T) > 50
    O = np.zeros_like(T)
    t, i, a = S.cast(O, T - O)
    assert np.all((i >= 0) & (i < box.shape[0]))


# ----------------------------------------------------------------------------
# shading, G-buffer
# ----------------------------------------------------------------------------

def test_shading_closed_form(orc):
    """Single square facing the camera at z = 2, light at the eye: the centre
    pixel of an odd-sized image sees n.l = 1 at distance 2, so
    C = albedo (ambient + I / 4); depth 2; normal faces the camera."""
    quad = np.array([[-1, -1, 2, 1, -1, 2, 1, 1, 2], [-1, -1, 2, 1, 1, 2, -1, 1, 2]], np.float64)
    alb = np.array([[0.25, 0.5, 0.75]] * 2)
    S = orc.Scene(quad, alb)
    cam = sg.look_camera((0, 0, 0), 0.0, 65, 65)
    lens = sg.lens_fnumber(0.05, 2.0, 3.0)
    light = sg.Light(np.zeros(3, np.float32), np.array([4, 8, 2], np.float32),
                     np.array([0.05, 0.1, 0.0], np.float32))
    gb = orc.gbuffer(S, cam, lens, light)
    c = gb["color"][:, 32, 32]
    ka = light.ambient.astype(np.float64)   # the interface carries float32 values
    expect = np.array([0.25 * (ka[0] + 1.0), 0.5 * (ka[1] + 2.0), 0.75 * (ka[2] + 0.5)])
    assert np.allclose(c, expect, rtol=0, atol=1e-12)
    assert abs(gb["depth"][32, 32] - 2.0) < 1e-12
    assert np.allclose(gb["normal"][:, 32, 32], [0, 0, -1])
    # off-centre pixel: cosine and inverse square by hand
    x, y = 50, 10
    sx = (2 * (x + 0.5) / 65 - 1) * float(np.float32(0.36))
    sy = (1 - 2 * (y + 0.5) / 65) * float(np.float32(0.36))
    P = np.array([sx * 2, sy * 2, 2.0])
    d2 = P @ P
    cosv = 2.0 / math.sqrt(d2)
    expect = np.array([0.25 * (ka[0] + 4 * cosv / d2), 0.5 * (ka[1] + 8 * cosv / d2), 0.75 * (2 * cosv / d2)])
    assert np.allclose(gb["color"][:, y, x], expect, atol=1e-6)  # camera basis is float32


# ----------------------------------------------------------------------------
# ray trace: half-plane partial occlusion, focus plane, identity
# ----------------------------------------------------------------------------

def _disk_fraction(tau):
    tau = np.clip(tau, -1, 1)
    return 0.5 + (tau * np.sqrt(1 - tau * tau) + np.arcsin(tau)) / math.pi


def test_half_plane_hit_ratio(orc):
    """Near occluder covering x < 0 at depth z_n over a far wall: the fraction
    of lens rays that hit the occluder is the area of the lens disk left of
    lambda = (x_e - u z_n) / (1 - z_n / S1), u the pixel's tan-x."""
    z_n, z_f = 0.5, 10.0
    sc = sg.half_plane_scene(z_n, 0.0, z_f)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.2)
    cam, lens, light = cfg.camera, cfg.lens, cfg.light
    S1 = lens.focus_distance
    a = lens.aperture / 2
    assert orc.coc(cam, lens, z_n) <= -SQ2 and orc.coc(cam, lens, z_f) >= SQ2
    xs = np.arange(16, 48)
    pix = 31 * cam.width + xs
    n_s = 4096
    rt = orc.trace(S, cam, lens, light, np.full(len(xs), n_s), pix=pix, seed=1, per_ray=True)
    for k, x in enumerate(xs):
        u = (2 * (x + 0.5) / cam.width - 1) * cam.tan_half_fov_x
        lam = (0.0 - u * z_n) / (1 - z_n / S1)
        F = _disk_fraction(lam / a)
        h = rt["hit_ratio"][k]
        sd = math.sqrt(max(F * (1 - F), 1e-12) / n_s)
        assert abs(h - F) <= 4 * sd + 1e-12, (x, h, F)
    # identity h C_tn + (1-h) C_tf = mean L
    L = rt["ray_L"].reshape(3, len(xs), n_s).mean(-1)
    mix = rt["hit_ratio"] * rt["c_near"] + (1 - rt["hit_ratio"]) * rt["c_far"]
    assert np.allclose(mix, L, atol=1e-12)
    assert np.all((rt["hit_ratio"] >= 0) & (rt["hit_ratio"] <= 1))


def test_focus_plane_rays_agree(orc):
    """A wall at exactly the focus distance: every lens ray of a pixel hits the
    point its pinhole ray hits, so the traced colour equals the G-buffer."""
    S1 = 2.0
    wall = np.array([[-9, -9, S1, 9, -9, S1, 9, 9, S1], [-9, -9, S1, 9, 9, S1, -9, 9, S1]])
    S = orc.Scene(wall, np.array([[0.3, 0.6, 0.9]] * 2))
    cfg = sg.config_tiny(aperture_override=0.2)
    gb = orc.gbuffer(S, cfg.camera, cfg.lens, cfg.light)
    rt = orc.trace(S, cfg.camera, cfg.lens, cfg.light, np.full((64, 64), 16), seed=2, per_ray=False)
    crt = rt["hit_ratio"] * rt["c_near"] + (1 - rt["hit_ratio"]) * rt["c_far"]
    assert np.max(np.abs(crt - gb["color"])) < 1e-6


def test_zero_aperture_trace_equals_gbuffer(orc):
    sc = sg.tiny_scene(0)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.0)
    gb = orc.gbuffer(S, cfg.camera, cfg.lens, cfg.light)
    rt = orc.trace(S, cfg.camera, cfg.lens, cfg.light, np.full((64, 64), 3), seed=4, per_ray=True)
    ids = rt["ray_id"].reshape(64, 64, 3)
    assert np.array_equal(ids, np.repeat(gb["tri_id"][..., None], 3, -1))
    crt = rt["hit_ratio"] * rt["c_near"] + (1 - rt["hit_ratio"]) * rt["c_far"]
    assert np.max(np.abs(crt - gb["color"])) < 1e-12


# ----------------------------------------------------------------------------
# mask
# ----------------------------------------------------------------------------

def test_mask_gaussian_and_sobel_match_scipy(orc):
    rng = np.random.default_rng(5)
    H, W = 37, 53
    z = ndi.uniform_filter(rng.uniform(0.5, 6.0, (H, W)), 3)
    n = rng.normal(size=(3, H, W))
    n /= np.linalg.norm(n, axis=0)
    mp = sg.MaskParams(sigma=1.0, spp_max=8, tile=8, dilate=1)
    for sigma in (1.0, 0.7, 1.6):
        mp.sigma = sigma
        out = orc.mask(z, n, mp)
        ref = [ndi.gaussian_filter(ch, sigma, mode="nearest", truncate=3.0) for ch in [z, *n]]
        for c in range(4):
            assert np.allclose(out["blur"][c], ref[c], atol=1e-12)
        def mag(b):
            return np.hypot(ndi.sobel(b, axis=1, mode="nearest"), ndi.sobel(b, axis=0, mode="nearest"))
        gz = mag(ref[0]) / (8 * np.maximum(ref[0], 1e-3))
        gn = np.sqrt(sum(mag(b) ** 2 for b in ref[1:])) / 8
        assert np.allclose(out["g_z"], gz, atol=1e-12)
        assert np.allclose(out["g_n"], gn, atol=1e-12)
        m = np.maximum(gz / mp.tau_depth, gn / mp.tau_normal)
        assert np.allclose(out["score"], m, rtol=1e-12)


def test_mask_counts_tiles_and_scan(orc):
    rng = np.random.default_rng(6)
    H, W = 45, 70
    z = np.where(rng.random((H, W)) < 0.03, 1.0, 4.0) * np.ones((H, W))
    n = np.zeros((3, H, W))
    n[2] = 1.0
    V = np.where(rng.random((H, W)) < 0.01, rng.uniform(0, 0.05, (H, W)), 0.0)
    V[3, 4] = np.inf
    for tile, dil, spp_max in [(8, 1, 8), (4, 0, 5), (1, 0, 16), (16, 2, 3)]:
        mp = sg.MaskParams(spp_max=spp_max, tile=tile, dilate=dil)
        out = orc.mask(z, n, mp, V)
        m = out["score"]
        raw = np.where(m >= 1, np.minimum(spp_max, np.ceil(np.where(np.isinf(m), spp_max, m))), 0)
        # brute force: max of raw over all pixels whose tile is within `dil` tiles
        ty, tx = np.arange(H) // tile, np.arange(W) // tile
        exp = np.zeros((H, W), np.int64)
        for y in range(H):
            rows = np.abs(ty - ty[y]) <= dil
            for x in range(W):
                cols = np.abs(tx - tx[x]) <= dil
                exp[y, x] = raw[np.ix_(rows, cols)].max()
        assert np.array_equal(out["spp"], exp)
        flat = out["spp"].reshape(-1).astype(np.int64)
        assert np.array_equal(out["offsets"].reshape(-1), np.concatenate([[0], np.cumsum(flat)[:-1]]))
        assert out["total"] == flat.sum()
        assert np.all(out["spp_lo"] <= out["spp"]) and np.all(out["spp"] <= out["spp_hi"])
    # constant image: zero gradient, no rays
    out = orc.mask(np.full((20, 30), 3.0), n[:, :20, :30], sg.MaskParams())
    assert out["total"] == 0 and np.all(out["g_z"] == 0) and np.all(out["g_n"] == 0)


def test_mask_threshold_ambiguity_band(orc):
    """A score exactly at an integer threshold is flagged (s_lo != s_hi)."""
    H, W = 16, 16
    z = np.full((H, W), 2.0)
    n = np.zeros((3, H, W))
    n[2] = 1
    V = np.zeros((H, W))
    V[8, 8] = 0.03  # V / tau_v = 3 exactly -> ceil = 3, but 3(1+eps) -> 4
    out = orc.mask(z, n, sg.MaskParams(tile=1, dilate=0, spp_max=8), V)
    assert out["spp"][8, 8] == 3 and out["spp_lo"][8, 8] == 3 and out["spp_hi"][8, 8] == 4


# ----------------------------------------------------------------------------
# variance history
# ----------------------------------------------------------------------------

def test_variance_static_camera_ema_closed_form(orc):
    rng = np.random.default_rng(8)
    H, W = 12, 10
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    z = rng.uniform(1, 5, (H, W))
    hist = orc.empty_history(H, W)
    alpha = 0.2
    xs = rng.uniform(0, 1, (6, H, W))
    spp = np.ones((H, W), np.int32)
    for k in range(6):
        rep = orc.var_reproject(cam, z, cam, hist)
        if k > 0:
            for key in ("lum_m1", "lum_m2", "flags"):
                assert np.array_equal(rep[key], hist[key])
            if k == 1:
                assert np.all(np.isinf(rep["V"]))   # newly traced last frame
        hist = orc.var_update(spp, rep, xs[k], xs[k] ** 2, alpha, z)
    # mu_n = (1-a)^(n) x_0 + a sum_{k=1..n} (1-a)^(n-k) x_k  (first frame restarts at x_0)
    n = 5
    mu = (1 - alpha) ** n * xs[0] + alpha * sum((1 - alpha) ** (n - k) * xs[k] for k in range(1, n + 1))
    assert np.allclose(hist["lum_m1"], mu, atol=1e-12)
    assert np.all(hist["flags"] == 1)
    rep = orc.var_reproject(cam, z, cam, hist)
    assert np.allclose(rep["V"], np.maximum(0, hist["lum_m2"] - hist["lum_m1"] ** 2), atol=1e-15)


def test_variance_pure_yaw_reprojection(orc):
    """Points far away under a pure yaw psi: the previous camera (yaw 0) sees
    the current pixel's direction at tan-x tan(psi + atan sx) and tan-y
    sy / (cos psi - sx sin psi); the axial depth scales by cos psi - sx sin psi."""
    H, W = 200, 320
    deg = 0.6
    psi = math.radians(deg)
    prev = sg.look_camera((0, 0, 0), 0.0, W, H)
    cur = sg.look_camera((0, 0, 0), deg, W, H)
    z = np.full((H, W), orc.ZMAX)
    hist = orc.empty_history(H, W)
    hist["lum_m1"] = np.arange(H * W, dtype=np.float64).reshape(H, W)
    hist["flags"][:] = 1
    hist["depth"][:] = orc.ZMAX
    rep = orc.var_reproject(cur, z, prev, hist)
    tx = float(prev.tan_half_fov_x)
    ty = tx * H / W
    ctx = float(cur.tan_half_fov_x)
    cty = ctx * H / W
    n_in = 0
    for y in range(0, H, 7):
        for x in range(0, W, 5):
            sx = (2 * (x + 0.5) / W - 1) * ctx
            sy = (1 - 2 * (y + 0.5) / H) * cty
            k = math.cos(psi) - sx * math.sin(psi)
            sxp = math.tan(psi + math.atan(sx))
            syp = sy / k
            fx = (sxp / tx + 1) * W / 2
            fy = (1 - syp / ty) * H / 2
            if rep["amb"][y, x]:
                continue
            depth_ok = abs(orc.ZMAX - orc.ZMAX * k) / (orc.ZMAX * k) <= 0.01
            if 0 <= fx < W and 0 <= fy < H and depth_ok:
                n_in += 1
                assert rep["flags"][y, x] == 1
                assert rep["lum_m1"][y, x] == int(fy) * W + int(fx)
            else:
                assert rep["flags"][y, x] == 0 and rep["V"][y, x] == 0
    assert n_in > 1000


def test_variance_depth_test_rejects(orc):
    H, W = 8, 8
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    z = np.full((H, W), 2.0)
    hist = orc.empty_history(H, W)
    hist["flags"][:] = 1
    hist["depth"][:] = 2.0
    hist["depth"][2, 3] = 2.0 * 1.02   # 2 % off: rejected
    hist["depth"][4, 4] = 2.0 * 1.005  # 0.5 % off: kept
    rep = orc.var_reproject(cam, z, cam, hist)
    assert rep["flags"][2, 3] == 0 and rep["flags"][4, 4] == 1 and rep["flags"][0, 0] == 1


# ----------------------------------------------------------------------------
# post-process gather filter
# ----------------------------------------------------------------------------

def test_postfilter_zero_aperture_and_constant(orc):
    cfg = sg.config_tiny(aperture_override=0.0)
    rng = np.random.default_rng(1)
    col = rng.uniform(0, 1, (3, 64, 64))
    z = rng.uniform(0.5, 8, (64, 64))
    out = orc.postfilter(cfg.camera, cfg.lens, col, z, cfg.pp)
    assert np.array_equal(out, col)
    cfg = sg.config_tiny(aperture_override=0.2)
    const = np.ones((3, 64, 64)) * np.array([0.2, 0.4, 0.9])[:, None, None]
    out = orc.postfilter(cfg.camera, cfg.lens, const, z, cfg.pp)
    assert np.allclose(out, const, atol=1e-13)
    out = orc.postfilter(cfg.camera, cfg.lens, col, z, cfg.pp)
    assert np.all(out >= col.min() - 1e-12) and np.all(out <= col.max() + 1e-12)


def test_postfilter_radius_tiles_brute_force(orc):
    rng = np.random.default_rng(2)
    H, W = 70, 90
    c = rng.normal(0, 20, (H, W))
    for tile, rcap in [(16, 64.0), (8, 10.0), (4, 5.0)]:
        R = orc.pp_radius(c, rcap, tile)
        K = math.ceil(rcap / tile)
        ty, tx = np.arange(H) // tile, np.arange(W) // tile
        for y in range(0, H, 3):
            for x in range(0, W, 4):
                sel = (np.abs(ty - ty[y])[:, None] <= K) & (np.abs(tx - tx[x])[None, :] <= K)
                assert R[y, x] == min(rcap, 0.5 * np.abs(c[sel]).max())


def test_postfilter_uniform_depth_is_disk_average(orc):
    """Uniform depth with CoC radius >= 96 px and R_cap = 64: every tap is
    accepted with equal weight, so the filter is a 48-point quadrature of the
    disk average of radius 64.  For cos(k x) the disk average is
    2 J1(kR)/(kR) cos(k x) (Bessel), which the golden-angle points reproduce
    to a few percent."""
    W = H = 256
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    spx = W / (2 * cam.tan_half_fov_x)
    S1, zz = 2.0, 8.0
    A = 2 * 100.0 / (spx * (1 / S1 - 1 / zz))  # |c| = 200 px -> r = 100
    lens = sg.Lens(0.05, float(np.float32(A)), S1)
    pp = sg.PPParams(r_cap=64.0)
    k = 2.5 / 64.0
    xs = np.arange(W) + 0.5
    col = np.broadcast_to(0.5 + 0.4 * np.cos(k * xs)[None, None, :], (3, H, W)).copy()
    z = np.full((H, W), zz)
    pix = np.array([128 * W + x for x in range(96, 160, 3)])
    out = orc.postfilter(cam, lens, col, z, pp, pix=pix)
    avg = 2 * sps.j1(2.5) / 2.5
    w0 = 1.0 / 100.0**2
    wt = 64.0**2 / 100.0**2
    for i, p in enumerate(pix):
        x = p % W
        disk = 0.5 + 0.4 * avg * math.cos(k * (x + 0.5))
        exp = (w0 * col[0, 128, x] + wt * disk) / (w0 + wt)
        assert abs(out[0, i] - exp) < 0.03
    assert np.allclose(out[0], out[1]) and np.allclose(out[1], out[2])


def test_postfilter_sharp_foreground_over_blurred_background(orc):
    """An in-focus object in front of a far background stays exactly sharp
    (background taps are clamped to its zero radius and rejected), while a
    blurred near object spreads over an in-focus background."""
    W = H = 96
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    lens = sg.lens_fnumber(0.05, 1.0, 0.5)
    pp = sg.PPParams()
    assert orc.coc(cam, lens, 20.0) > 10.0   # every tap lies beyond the 0.5-px ramp
    col = np.zeros((3, H, W))
    z = np.full((H, W), 20.0)                  # blurred far background
    z[30:60, 30:60] = 0.5                      # in-focus square
    col[0] = 1.0
    col[:, 30:60, 30:60] = np.array([0, 1, 0])[:, None, None]
    out = orc.postfilter(cam, lens, col, z, pp)
    assert np.array_equal(out[:, 30:60, 30:60], col[:, 30:60, 30:60])
    # blurred near square over an in-focus background bleeds outward
    z2 = np.full((H, W), 0.5)
    z2[30:60, 30:60] = 0.25
    out2 = orc.postfilter(cam, lens, col, z2, pp)
    assert out2[1, 45, 62] > 0.05           # green spreads past the edge
    assert np.array_equal(out2[:, 5, 5], col[:, 5, 5])  # far from it: untouched


# ----------------------------------------------------------------------------
# composite
# ----------------------------------------------------------------------------

def test_composite_rules(orc):
    W, H = 8, 1
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    lens = sg.lens_fnumber(0.05, 1.4, 2.0)
    spx = W / (2 * cam.tan_half_fov_x)
    A, S1 = lens.aperture, lens.focus_distance
    def z_of_c(c):
        return 1.0 / (1.0 / S1 - c / (A * spx))
    cs = [0.0, -10.0, -10.0, 10.0, 10.0, 10.0, SQ2 + 0.5, 10.0]
    spp = np.array([[4, 4, 0, 4, 4, 4, 0, 4]], np.int32)
    hit = np.array([[0.3, 0.3, 0.0, 0.0, 0.75, 0.25, 0.0, 0.5]])
    z = np.array([[z_of_c(c) for c in cs]])
    Cr = np.ones((3, H, W)) * 0.1
    Cpp = np.ones((3, H, W)) * 0.2
    Cn = np.ones((3, H, W)) * 0.6
    Cf = np.ones((3, H, W)) * 0.4
    out = orc.composite(cam, lens, Cr, Cpp, z, spp, Cn, Cf, hit, sg.CompositeParams())[0, 0]
    crt = hit[0] * 0.6 + (1 - hit[0]) * 0.4
    exp = [0.1,              # focus zone: raster
           crt[1],           # near, traced: ray trace
           0.2,              # near, untraced: post-process
           crt[3],           # far, h = 0: ray trace
           0.2,              # far, h >= h_t: post-process
           0.5 * crt[5] + 0.5 * 0.2,  # far, h = h_t / 2: half and half
           0.5 * 0.1 + 0.5 * 0.2,     # |c| = sqrt2 + 0.5, untraced: phi = 0.5
           0.2]              # far, h = h_t: post-process
    assert np.allclose(out, exp, atol=1e-12)
    ov = orc.composite(cam, lens, Cr, Cpp, z, spp, Cn, Cf, hit, sg.CompositeParams(rt_override=1))[0, 0]
    assert np.allclose(ov[spp[0] > 0], crt[spp[0] > 0], atol=1e-15)


# ----------------------------------------------------------------------------
# whole frame invariants
# ----------------------------------------------------------------------------

def test_frame_zero_aperture_is_raster(orc):
    sc = sg.tiny_scene(0)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.0)
    fr = orc.frame(S, cfg)
    assert np.array_equal(fr["out"], fr["gbuffer"]["color"])


def test_frame_full_mask_override_is_full_rt(orc):
    sc = sg.tiny_scene(0)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.2)
    fr = orc.frame(S, cfg, rt_full_spp=5)
    rt = orc.trace(S, cfg.camera, cfg.lens, cfg.light, np.full((64, 64), 5), seed=cfg.seed, per_ray=True)
    mean_L = rt["ray_L"].reshape(3, 64, 64, 5).mean(-1)
    assert np.allclose(fr["out"], mean_L, atol=1e-12)


def test_frame_new_regions_get_max_rays(orc):
    """Regions traced in one frame are 'new' in the next and get spp_max."""
    sc = sg.tiny_scene(0)
    S = orc.Scene(sc.verts, sc.albedo)
    cfg = sg.config_tiny(aperture_override=0.1)
    cfg.mask.tile, cfg.mask.dilate = 1, 0
    cfg.mask.tau_depth, cfg.mask.tau_normal = 0.2, 0.4
    f0 = orc.frame(S, cfg)
    f1 = orc.frame(S, cfg, prev_camera=cfg.camera, history=f0["history"], frame_index=1)
    traced0 = f0["spp"] > 0
    assert traced0.any() and not traced0.all()
    assert np.all(f1["spp"][traced0] == cfg.mask.spp_max)


# ----------------------------------------------------------------------------
# mask resolution scaled by the maximum CoC
# ----------------------------------------------------------------------------

def test_scaled_tile_of_a_wall(orc):
    """A wall filling the view at depth z: every pixel's CoC radius is the
    thin-lens |c|/2 = A s_px |1/S1 - 1/z| / 2 (s_px = W / (2 tan(fov/2))),
    and the tile edge follows the bands R < 16 -> 4, R < 32 -> 8, else 16."""
    z = 0.3
    wall = np.array([[-9, -9, z, 9, -9, z, 9, 9, z], [-9, -9, z, 9, 9, z, -9, 9, z]])
    S = orc.Scene(wall, np.array([[0.5, 0.5, 0.5]] * 2))
    cfg = sg.config_tiny()
    cam = cfg.camera
    gb = orc.gbuffer(S, cam, cfg.lens, cfg.light)
    assert np.allclose(gb["depth"], z, rtol=1e-9)
    s_px = cam.width / (2 * cam.tan_half_fov_x)
    seen = set()
    for A in (0.02, 0.1, 0.2, 0.3, 0.4):
        lens = sg.Lens(cfg.lens.focal_length, A, cfg.lens.focus_distance)
        R = A * s_px * abs(1 / lens.focus_distance - 1 / z) / 2
        t, r = orc.scaled_tile(cam, lens, gb["depth"])
        assert abs(r - R) < 1e-6 * max(R, 1), (A, r, R)
        assert t == (4 if R < 16 else (8 if R < 32 else 16)), (A, R, t)
        seen.add(t)
    assert seen == {4, 8, 16}


def test_scaled_tile_mask_equals_the_fixed_tile(orc):
    """tile = 0 is the mask with the tile edge the maximum CoC picks."""
    from dataclasses import replace
    sc = sg.living_room_scene(0)
    cfg = sg.config_1080p(160, 90)
    gb = orc.gbuffer(orc.Scene(sc.verts, sc.albedo), cfg.camera, cfg.lens, cfg.light)
    for N in (2.8, 0.5, 0.25):
        lens = sg.lens_fnumber(cfg.lens.focal_length, N, cfg.lens.focus_distance)
        a = orc.mask(gb["depth"], gb["normal"], replace(cfg.mask, tile=0), None, cfg.camera, lens)
        b = orc.mask(gb["depth"], gb["normal"], replace(cfg.mask, tile=a["tile"]), None)
        assert np.array_equal(a["spp"], b["spp"]) and a["total"] == b["total"]
    # a larger aperture never picks a finer mask
    tiles = [orc.scaled_tile(cfg.camera, sg.lens_fnumber(cfg.lens.focal_length, N, cfg.lens.focus_distance),
                             gb["depth"])[0] for N in (8, 2.8, 1.4, 0.5, 0.25)]
    assert tiles == sorted(tiles) and len(set(tiles)) >= 2
