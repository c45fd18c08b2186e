"""Pins of the oracle's temporal reconstruction of the traced colours
(paper, Reconstruction): the exponential moving average in closed form on a
static camera, the exact history source under a camera translation over a
fronto-parallel wall (near path through the G-buffer surface, far path
through the far-hit position, with the neighbour fallback), the depth test
and the treatment of untraced pixels.  Wall points, shifts and the EMA sums
are computed here from the camera definition, not by the oracle."""
import numpy as np
import pytest

import scenegen as sg

ALPHA = 0.2


def _wall_points(cam, Z):
    """World points at axial depth Z through every pixel centre: X = e + Z v,
    v = w + sx r + sy u (tan-space pixel coordinates)."""
    H, W = cam.height, cam.width
    tx = float(cam.tan_half_fov_x)
    ty = tx * H / W
    xs = (2 * (np.arange(W) + 0.5) / W - 1) * tx
    ys = (1 - 2 * (np.arange(H) + 0.5) / H) * ty
    sx, sy = np.meshgrid(xs, ys)
    e, r, u, w = (np.asarray(a, np.float64) for a in (cam.eye, cam.right, cam.up, cam.fwd))
    X = e[:, None, None] + Z * (w[:, None, None] + sx * r[:, None, None] + sy * u[:, None, None])
    return X


def _far_pos(X, weight=1.0):
    H, W = X.shape[1:]
    return np.concatenate([X, np.full((1, H, W), weight)], axis=0)


def test_static_camera_is_the_closed_form_ema(orc):
    """Static camera, every pixel traced: after K frames the near output is
    sum_i a_i h_i C_i / sum_i a_i h_i with a_0 = (1-alpha)^K and
    a_i = alpha (1-alpha)^(K-i); the far output uses (1-h_i) weights for the
    colour and 1 - (the same EMA of h) as its normaliser."""
    W, H, Z, K = 24, 16, 3.0, 6
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    z = np.full((H, W), Z)
    spp = np.full((H, W), 4, np.int32)
    X = _wall_points(cam, Z)
    rng = np.random.default_rng(1)
    hs = rng.uniform(0.05, 0.95, (K + 1, H, W))
    Cn = rng.uniform(0, 1, (K + 1, 3, H, W))
    Cf = rng.uniform(0, 1, (K + 1, 3, H, W))
    hist = orc.empty_recon_history(H, W)
    prev = None
    for t in range(K + 1):
        r = orc.recon(cam, z, spp, prev, hist, hs[t], Cn[t], Cf[t], _far_pos(X), ALPHA)
        assert not r["amb"].any()
        hist, prev = r["history"], cam
    a = np.array([(1 - ALPHA) ** K] + [ALPHA * (1 - ALPHA) ** (K - i) for i in range(1, K + 1)])
    hn = np.tensordot(a, hs, 1)
    near = np.tensordot(a, hs[:, None] * Cn, 1) / hn
    far = np.tensordot(a, (1 - hs)[:, None] * Cf, 1) / (1 - hn)
    assert np.allclose(r["c_near"], near, rtol=1e-12, atol=1e-12)
    assert np.allclose(r["c_far"], far, rtol=1e-12, atol=1e-12)
    assert np.allclose(r["history"]["planes"][3], hn) and np.allclose(r["history"]["planes"][7], hn)


def test_translation_takes_history_three_pixels_over(orc):
    """The camera moves along its right axis by 3 Z (2 tan_x / W): a wall
    point seen at pixel x was at x + 3 in the previous frame.  Both paths
    (G-buffer surface, far position) take the history of pixel (x + 3, y);
    pixels whose source falls outside start afresh."""
    W, H, Z = 32, 12, 2.5
    prev = sg.look_camera((0, 0, 0), 0.0, W, H)
    dx = 3 * Z * 2 * prev.tan_half_fov_x / W
    cur = sg.look_camera((float(np.float32(dx)), 0, 0), 0.0, W, H)
    # float32 eye: recompute the exact shift the cameras imply
    shift = (float(cur.eye[0]) - float(prev.eye[0])) / Z * W / (2 * prev.tan_half_fov_x)
    assert abs(shift - 3) < 1e-5
    z = np.full((H, W), Z)
    spp = np.full((H, W), 2, np.int32)
    rng = np.random.default_rng(2)
    hist = dict(planes=rng.uniform(0.1, 0.9, (8, H, W)), valid=np.ones((H, W), np.int32), depth=np.full((H, W), Z))
    h = rng.uniform(0.1, 0.9, (H, W))
    Cn, Cf = rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (3, H, W))
    X = _wall_points(cur, Z)
    r = orc.recon(cur, z, spp, prev, hist, h, Cn, Cf, _far_pos(X), ALPHA)
    P = hist["planes"]
    for y in range(H):
        for x in range(W):
            if x + 3 < W:
                N = (1 - ALPHA) * P[0:3, y, x + 3] + ALPHA * h[y, x] * Cn[:, y, x]
                Hn = (1 - ALPHA) * P[3, y, x + 3] + ALPHA * h[y, x]
                F = (1 - ALPHA) * P[4:7, y, x + 3] + ALPHA * (1 - h[y, x]) * Cf[:, y, x]
                Hf = (1 - ALPHA) * P[7, y, x + 3] + ALPHA * h[y, x]
            else:
                N, Hn = h[y, x] * Cn[:, y, x], h[y, x]
                F, Hf = (1 - h[y, x]) * Cf[:, y, x], h[y, x]
            assert np.allclose(r["c_near"][:, y, x], N / Hn, rtol=1e-12)
            assert np.allclose(r["c_far"][:, y, x], F / (1 - Hf), rtol=1e-12)


def test_far_position_falls_back_to_the_neighbours(orc):
    """A pixel with no far hit takes the mean far position of its 8
    neighbours: on a plane that is its own wall point, so under the same
    translation it still reads the history 3 pixels over.  The near path is
    cut (depth test fails) so only the far path carries history; a pixel
    with no far hit around it starts afresh."""
    W, H, Z = 32, 12, 2.5
    prev = sg.look_camera((0, 0, 0), 0.0, W, H)
    dx = float(np.float32(3 * Z * 2 * prev.tan_half_fov_x / W))
    cur = sg.look_camera((dx, 0, 0), 0.0, W, H)
    z = np.full((H, W), Z)
    spp = np.full((H, W), 1, np.int32)
    rng = np.random.default_rng(3)
    hist = dict(planes=rng.uniform(0.1, 0.9, (8, H, W)), valid=np.ones((H, W), np.int32),
                depth=np.full((H, W), 2 * Z))   # previous depth 100 % off: near path rejected
    h = rng.uniform(0.1, 0.9, (H, W))
    Cn, Cf = rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (3, H, W))
    fp = _far_pos(_wall_points(cur, Z))
    fp[3, 5, 10] = 0.0                      # no far hit: neighbours' mean = own wall point
    fp[3, 8:11, 19:22] = 0.0                # no far hit anywhere around (9, 20)
    r = orc.recon(cur, z, spp, prev, hist, h, Cn, Cf, fp, ALPHA)
    P = hist["planes"]
    y, x = 5, 10
    F = (1 - ALPHA) * P[4:7, y, x + 3] + ALPHA * (1 - h[y, x]) * Cf[:, y, x]
    Hf = (1 - ALPHA) * P[7, y, x + 3] + ALPHA * h[y, x]
    assert np.allclose(r["c_far"][:, y, x], F / (1 - Hf), rtol=1e-9)
    y, x = 9, 20
    assert np.allclose(r["c_far"][:, y, x], Cf[:, y, x], rtol=1e-12)
    # near path everywhere restarted: output = current near colour
    assert np.allclose(r["c_near"], Cn, rtol=1e-12)


def test_depth_test_and_untraced_pixels(orc):
    """Near history is used only when the previous depth agrees within 1 %;
    untraced pixels pass their colours through and leave no history."""
    W, H, Z = 16, 8, 2.0
    cam = sg.look_camera((0, 0, 0), 0.0, W, H)
    z = np.full((H, W), Z)
    spp = np.full((H, W), 3, np.int32)
    spp[:, :4] = 0
    rng = np.random.default_rng(4)
    pz = np.full((H, W), Z)
    pz[:, 8:12] = Z * 1.02    # 2 % off: rejected
    pz[:, 12:] = Z * 1.005    # 0.5 % off: accepted
    hist = dict(planes=rng.uniform(0.1, 0.9, (8, H, W)), valid=np.ones((H, W), np.int32), depth=pz)
    h = rng.uniform(0.1, 0.9, (H, W))
    Cn, Cf = rng.uniform(0, 1, (3, H, W)), rng.uniform(0, 1, (3, H, W))
    X = _wall_points(cam, Z)
    r = orc.recon(cam, z, spp, cam, hist, h, Cn, Cf, _far_pos(X, 0.0), ALPHA)  # no far hits at all
    P = hist["planes"]
    N = (1 - ALPHA) * P[0:3] + ALPHA * h * Cn
    Hn = (1 - ALPHA) * P[3] + ALPHA * h
    acc = N / Hn
    assert np.allclose(r["c_near"][:, :, 4:8], acc[:, :, 4:8])
    assert np.allclose(r["c_near"][:, :, 8:12], Cn[:, :, 8:12])
    assert np.allclose(r["c_near"][:, :, 12:], acc[:, :, 12:])
    assert np.allclose(r["c_near"][:, :, :4], Cn[:, :, :4]) and np.allclose(r["c_far"][:, :, :4], Cf[:, :, :4])
    assert not r["history"]["valid"][:, :4].any() and r["history"]["valid"][:, 4:].all()
    assert np.all(r["history"]["planes"][:, :, :4] == 0)
