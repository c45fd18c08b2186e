"""FP64 CPU oracle of the hybrid depth-of-field hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are its only users.  The GPU library
(``paper_2210_04981_amd``) never imports it, and it never imports the GPU
library: the two share no code.  Only ``scenegen`` (seeded inputs, none of
the method's arithmetic) feeds both.

The arithmetic lives in ``hdof_oracle.c`` (plain C, double precision,
OpenMP over pixels); this module marshals numpy arrays and strings the
per-stage functions into a frame.  Each wrapper names the paper section it
follows; the readings of the paper the C code takes are stated there.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hdof_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# HDOF_ORACLE_SANITIZED=1: the AddressSanitizer + UndefinedBehaviorSanitizer
# build (its runtime must be preloaded; see tests/test_oracle_sanitized.py)
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
_SANITIZED = os.environ.get("HDOF_ORACLE_SANITIZED") == "1"

ZMAX = 1.0e4
VALID, NEW = 1, 2


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle shared library with gcc (-O2, OpenMP); sanitize:
    the checking build (-O1, AddressSanitizer and UndefinedBehaviorSanitizer,
    any report fatal)."""
    out = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        checks = ",".join(("address", "undefined"))  # host code (gcc), the oracle only
        opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + checks,
               "-fno-sanitize-recover=all"] if sanitize else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB_SAN if _SANITIZED else _LIB
        if not os.path.exists(path):
            build(force=True, sanitize=_SANITIZED)
        L = C.CDLL(path)
        P = C.c_void_p
        i32, i64, u64, f64 = C.c_int, C.c_int64, C.c_uint64, C.c_double
        L.or_scene_create.restype = P
        L.or_scene_create.argtypes = [P, P, i32]
        L.or_scene_destroy.argtypes = [P]
        L.or_scene_nodes.restype = i32
        L.or_scene_nodes.argtypes = [P]
        L.or_num_threads.restype = i32
        L.or_set_threads.argtypes = [i32]
        L.or_philox4x64_10.argtypes = [P, P, P]
        L.or_coc.restype = f64
        L.or_coc.argtypes = [P, i32, i32, P, f64]
        L.or_lens_ray.argtypes = [P, i32, i32, P, i32, i32, u64, u64, u64, u64, i32, P, P, P]
        L.or_cast_rays.argtypes = [P, i32, P, P, i32, P, P, P]
        L.or_gbuffer.argtypes = [P, P, i32, i32, P, P, P, i64, P, P, P, P, P, P, P]
        L.or_scene_set_spec.argtypes = [P, P]
        L.or_gauss_taps.argtypes = [f64, P, P]
        L.or_mask_scaled_tile.restype = i32
        L.or_mask_scaled_tile.argtypes = [P, i32, i32, P, P, P]
        L.or_mask.restype = i32
        L.or_mask.argtypes = [i32, i32, P, P, P, f64, f64, f64, f64, i32, i32, i32,
                              P, P, P, P, P, P, P, P, P]
        L.or_trace.argtypes = [P, P, i32, i32, P, P, P, P, i64, P, u64, u64, u64,
                               P, P, P, P, i64, P, P, P, P, P, P, P, P]
        L.or_sp_level.argtypes = [i32, i32, P, P, P, P, P, P, f64, i32, P]
        L.or_spatial.argtypes = [i32, i32, P, P, P, P, P, P, P, i32, f64, f64, P, P, P, P]
        L.or_recon.argtypes = [P, i32, i32, P, P, P, P, P, P, P, P, P, P, P, f64, P, P, P, P, P, P]
        L.or_var_reproject.argtypes = [P, i32, i32, P, P, i32, i32, P, P, P, P, P, P, P, P, P]
        L.or_var_update.argtypes = [i32, i32, P, P, P, P, P, P, f64, P, P, P, P, P]
        L.or_pp_radius.argtypes = [i32, i32, P, f64, i32, P]
        L.or_postfilter.argtypes = [P, i32, i32, P, P, P, P, P, i64, P]
        L.or_composite.argtypes = [P, i32, i32, P, P, P, P, P, P, P, P, f64, i32, P, f64, P]
        L.or_pp_radius_arg.argtypes = [i32, i32, P, f64, i32, P, P]
        L.or_pp_composite_backward.argtypes = [P, i32, i32, P, P, P, P, P, P, P, P, f64, i32, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


# ----------------------------------------------------------------------------
# counter-based generator
# ----------------------------------------------------------------------------

def philox4x64_10(ctr, key) -> np.ndarray:
    """Philox4x64-10 block (Salmon et al., SC'11) for one counter/key."""
    c = np.ascontiguousarray(np.asarray(ctr, np.uint64))
    k = np.ascontiguousarray(np.asarray(key, np.uint64))
    o = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(_p(c), _p(k), _p(o))
    return o


# ----------------------------------------------------------------------------
# scene
# ----------------------------------------------------------------------------

class Scene:
    """Triangle soup + the oracle's own median-split BVH (double precision)."""

    def __init__(self, verts, albedo, spec=None):
        """spec: per-triangle (k_s, shininess) of the specular lobe, or None
        (Lambertian)."""
        self.verts = _f64(verts).reshape(-1, 9)
        self.albedo = _f64(albedo).reshape(-1, 3)
        self.n = self.verts.shape[0]
        self._h = lib().or_scene_create(_p(self.verts), _p(self.albedo), self.n)
        self.spec = None if spec is None else _f64(spec).reshape(-1, 2)
        if self.spec is not None:
            lib().or_scene_set_spec(self._h, _p(self.spec))

    @property
    def handle(self):
        return self._h

    @property
    def n_nodes(self) -> int:
        return lib().or_scene_nodes(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_scene_destroy(h)
            self._h = None

    def cast(self, O, D, brute: bool = False):
        """Closest hits of rays (n,3) origins/directions: t (inf on miss),
        triangle id (-1 on miss), ambiguity flag."""
        O = _f64(O).reshape(-1, 3)
        D = _f64(D).reshape(-1, 3)
        n = O.shape[0]
        t = np.zeros(n)
        i = np.zeros(n, np.int32)
        a = np.zeros(n, np.int32)
        lib().or_cast_rays(self._h, n, _p(O), _p(D), int(brute), _p(t), _p(i), _p(a))
        return t, i, a


def cam_args(camera):
    """(cam[13] float64, W, H) from a scenegen.Camera (float32 widened exactly)."""
    return _f64(camera.as_floats()), int(camera.width), int(camera.height)


def coc(camera, lens, z) -> float:
    """Signed CoC diameter (px) of axial depth z under the thin-lens model."""
    cam, W, H = cam_args(camera)
    return lib().or_coc(_p(cam), W, H, _p(_f64(lens.as_floats())), float(z))


def lens_ray(camera, lens, x, y, j, seed=0, frame=0, view=0, pinhole=False, weight=False):
    """Thin-lens ray (O, D) of sample j of pixel (x, y); with weight=True
    also the sample's spherical-aberration weight."""
    cam, W, H = cam_args(camera)
    O = np.zeros(3)
    D = np.zeros(3)
    w = np.zeros(1)
    lib().or_lens_ray(_p(cam), W, H, _p(_f64(lens.as_floats())), int(x), int(y), int(j),
                      int(seed), int(frame), int(view), int(pinhole), _p(O), _p(D), _p(w))
    return (O, D, float(w[0])) if weight else (O, D)


# ----------------------------------------------------------------------------
# stages
# ----------------------------------------------------------------------------

def gbuffer(scene: Scene, camera, lens, light, pix=None) -> dict:
    """Pinhole G-buffer (paper, Design): depth, normal, albedo, shaded colour,
    triangle id, ambiguity and specular luminance for every pixel (or for the
    listed linear pixel indices)."""
    cam, W, H = cam_args(camera)
    pixa = None if pix is None else _i64(pix)
    n = W * H if pix is None else pixa.shape[0]
    z = np.zeros(n)
    nrm = np.zeros((3, n))
    alb = np.zeros((3, n))
    col = np.zeros((3, n))
    tid = np.zeros(n, np.int32)
    amb = np.zeros(n, np.int32)
    ys = np.zeros(n)
    lib().or_gbuffer(scene.handle, _p(cam), W, H, _p(_f64(lens.as_floats())),
                     _p(_f64(light.as_floats())), _p(pixa), n,
                     _p(z), _p(nrm), _p(alb), _p(col), _p(tid), _p(amb), _p(ys))
    out = dict(depth=z, normal=nrm, albedo=alb, color=col, tri_id=tid, amb=amb, spec=ys)
    if pix is None:
        out = {k: (v.reshape(-1, H, W) if v.ndim == 2 else v.reshape(H, W)) for k, v in out.items()}
    return out


def gauss_taps(sigma: float):
    r = C.c_int(0)
    taps = np.zeros(32)
    lib().or_gauss_taps(float(sigma), C.byref(r), _p(taps))
    return taps[: 2 * r.value + 1].copy()


def scaled_tile(camera, lens, depth):
    """Mask tile edge scaled by the frame's maximum CoC radius R (paper,
    Discussion): (tile, R)."""
    cam, W, H = cam_args(camera)
    r = np.zeros(1)
    t = lib().or_mask_scaled_tile(_p(cam), W, H, _p(_f64(lens.as_floats())), _p(_f64(depth).reshape(H, W)), _p(r))
    return int(t), float(r[0])


def mask(depth, normal, mp, V=None, camera=None, lens=None) -> dict:
    """Adaptive ray mask (paper, Ray Trace): Gaussian + Sobel on depth and
    normal, variance score, tile max + dilation, exclusive scan.  Returns the
    per-pixel count s with its ambiguity bounds s_lo/s_hi, offsets, total,
    the tile edge used and the intermediate blurred channels and scores.
    mp.tile == 0: the tile edge is scaled by the frame's maximum CoC
    (needs the camera and lens)."""
    depth = _f64(depth)
    H, W = depth.shape
    tile, r_max = int(mp.tile), None
    if tile == 0:
        if camera is None or lens is None:
            raise ValueError("oracle mask: tile 0 needs the camera and lens")
        tile, r_max = scaled_tile(camera, lens, depth)
    normal = _f64(normal).reshape(3, H, W)
    Va = None if V is None else _f64(V).reshape(H, W)
    N = W * H
    blur = np.zeros((4, H, W))
    gz = np.zeros((H, W))
    gn = np.zeros((H, W))
    m = np.zeros((H, W))
    s = np.zeros((H, W), np.int32)
    slo = np.zeros((H, W), np.int32)
    shi = np.zeros((H, W), np.int32)
    off = np.zeros((H, W), np.int64)
    tot = np.zeros(1, np.int64)
    rc = lib().or_mask(W, H, _p(depth), _p(normal), _p(Va), float(mp.sigma), float(mp.tau_depth),
                       float(mp.tau_normal), float(mp.tau_var), int(mp.spp_max), tile,
                       int(mp.dilate), _p(blur), _p(gz), _p(gn), _p(m), _p(s), _p(slo), _p(shi),
                       _p(off), _p(tot))
    if rc != 0:
        raise ValueError("oracle mask: bad parameters")
    return dict(blur=blur, g_z=gz, g_n=gn, score=m, spp=s, spp_lo=slo, spp_hi=shi,
                offsets=off, total=int(tot[0]), tile=tile, r_max=r_max)


def trace(scene: Scene, camera, lens, light, spp, pix=None, seed=0, frame=0, view=0,
          per_ray: bool = True) -> dict:
    """Thin-lens distributed ray trace + per-pixel reduction (paper, Ray
    Trace).  `spp` is the per-pixel count (full image (H,W) when pix is None,
    else one count per listed pixel).  `far_pos` (4 planes): far-weighted
    mean hit point of the rays that hit, and its weight.  `coc_nf` (2
    planes): mean |CoC| of the near rays and of the far rays."""
    cam, W, H = cam_args(camera)
    sp = _i32(spp).reshape(-1)
    pixa = None if pix is None else _i64(pix)
    n = sp.shape[0]
    base = np.zeros(n, np.int64)
    if n > 1:
        base[1:] = np.cumsum(sp[:-1].astype(np.int64))
    nr = int(sp.astype(np.int64).sum())
    rid = np.zeros(nr, np.int32) if per_ray else None
    rz = np.zeros(nr) if per_ray else None
    rL = np.zeros((3, nr)) if per_ray else None
    ra = np.zeros(nr, np.int32) if per_ray else None
    cn = np.zeros((3, n))
    cf = np.zeros((3, n))
    h = np.zeros(n)
    m1 = np.zeros(n)
    m2 = np.zeros(n)
    pa = np.zeros(n, np.int32)
    fp = np.zeros((4, n))
    cc = np.zeros((2, n))
    lib().or_trace(scene.handle, _p(cam), W, H, _p(_f64(lens.as_floats())),
                   _p(_f64(light.as_floats())), _p(pixa), _p(sp), n,
                   _p(base) if per_ray else None, int(seed), int(frame), int(view),
                   _p(rid), _p(rz), _p(rL), _p(ra), nr,
                   _p(cn), _p(cf), _p(h), _p(m1), _p(m2), _p(pa), _p(fp), _p(cc))
    out = dict(c_near=cn, c_far=cf, hit_ratio=h, lum_m1=m1, lum_m2=m2, px_amb=pa,
               ray_base=base, ray_id=rid, ray_z=rz, ray_L=rL, ray_amb=ra, far_pos=fp, coc_nf=cc)
    if pix is None:
        out["far_pos"] = fp.reshape(4, H, W)
        out["coc_nf"] = cc.reshape(2, H, W)
        for k in ("c_near", "c_far"):
            out[k] = out[k].reshape(3, H, W)
        for k in ("hit_ratio", "lum_m1", "lum_m2", "px_amb"):
            out[k] = out[k].reshape(H, W)
    return out


def var_reproject(camera, depth, prev_camera, hist: dict) -> dict:
    """Reproject the previous frame's luminance-moment history into the
    current frame and form the variance score V."""
    cam, W, H = cam_args(camera)
    pcam, PW, PH = cam_args(prev_camera)
    z = _f64(depth).reshape(H, W)
    rm1 = np.zeros((H, W))
    rm2 = np.zeros((H, W))
    rfl = np.zeros((H, W), np.int32)
    V = np.zeros((H, W))
    amb = np.zeros((H, W), np.int32)
    lib().or_var_reproject(_p(cam), W, H, _p(z), _p(pcam), PW, PH,
                           _p(_f64(hist["lum_m1"])), _p(_f64(hist["lum_m2"])),
                           _p(_i32(hist["flags"])), _p(_f64(hist["depth"])),
                           _p(rm1), _p(rm2), _p(rfl), _p(V), _p(amb))
    return dict(lum_m1=rm1, lum_m2=rm2, flags=rfl, V=V, amb=amb)


def empty_history(H: int, W: int) -> dict:
    return dict(lum_m1=np.zeros((H, W)), lum_m2=np.zeros((H, W)),
                flags=np.zeros((H, W), np.int32), depth=np.full((H, W), ZMAX))


def var_update(spp, rep: dict, ybar, y2bar, alpha, depth) -> dict:
    """EMA update of the luminance moments after the trace."""
    sp = _i32(spp)
    H, W = sp.shape
    m1 = np.zeros((H, W))
    m2 = np.zeros((H, W))
    fl = np.zeros((H, W), np.int32)
    zh = np.zeros((H, W))
    lib().or_var_update(W, H, _p(sp), _p(_f64(rep["lum_m1"])), _p(_f64(rep["lum_m2"])),
                        _p(_i32(rep["flags"])), _p(_f64(ybar)), _p(_f64(y2bar)), float(alpha),
                        _p(_f64(depth)), _p(m1), _p(m2), _p(fl), _p(zh))
    return dict(lum_m1=m1, lum_m2=m2, flags=fl, depth=zh)


def pp_radius(coc_img, r_cap: float, tile: int):
    c = _f64(coc_img)
    H, W = c.shape
    R = np.zeros((H, W))
    lib().or_pp_radius(W, H, _p(c), float(r_cap), int(tile), _p(R))
    return R


def postfilter(camera, lens, color, depth, pp, pix=None):
    """Post-process gather DoF filter; output (3,H,W) or (3,n) for `pix`."""
    cam, W, H = cam_args(camera)
    col = _f64(color).reshape(3, H, W)
    z = _f64(depth).reshape(H, W)
    ppa = _f64([pp.n_taps, pp.tile, pp.r_cap, pp.bg_ramp_px])
    pixa = None if pix is None else _i64(pix)
    n = W * H if pix is None else pixa.shape[0]
    out = np.zeros((3, n))
    lib().or_postfilter(_p(cam), W, H, _p(_f64(lens.as_floats())), _p(col), _p(z), _p(ppa),
                        _p(pixa), n, _p(out))
    return out.reshape(3, H, W) if pix is None else out


def composite(camera, lens, color, cpp, depth, spp, c_near, c_far, hit, cp, pp_spec=None):
    """Composite (paper, Composite); with `pp_spec` (the post-filtered
    specular luminance) and cp.spec_y > 0 the near traced pixels favour the
    post-process colour by clamp(pp_spec / spec_y, 0, 1)."""
    cam, W, H = cam_args(camera)
    out = np.zeros((3, H, W))
    spec_y = float(getattr(cp, "spec_y", 0.0))
    lib().or_composite(_p(cam), W, H, _p(_f64(lens.as_floats())), _p(_f64(color)), _p(_f64(cpp)),
                       _p(_f64(depth)), _p(_i32(spp)), _p(_f64(c_near)), _p(_f64(c_far)),
                       _p(_f64(hit)), float(cp.h_t), int(cp.rt_override),
                       _p(None if pp_spec is None else _f64(pp_spec)), spec_y, _p(out))
    return out


def postfilter_spec(camera, lens, spec, depth, pp, pix=None):
    """The post-filtered specular luminance: the post-filter's gather (same
    radius, taps and weights) applied to the G-buffer's specular luminance."""
    ys = _f64(spec)
    out = postfilter(camera, lens, np.broadcast_to(ys.reshape(1, *ys.shape[-2:]), (3,) + ys.shape[-2:]),
                     depth, pp, pix)
    return out[0]


def frame(scene: Scene, cfg, prev_camera=None, history=None, frame_index=0, view=0,
          rt_full_spp: int | None = None, recon_history=None) -> dict:
    """One frame of the hot path in the paper's stage order:
    G-buffer -> ray mask (with reprojected variance when a history is given)
    -> thin-lens trace -> variance update -> temporal reconstruction of the
    traced colours (when cfg.recon.enable; its history is `recon_history`,
    used when prev_camera is given) -> spatial reconstruction (when
    cfg.spatial.enable; variance from the updated history) -> post-process
    -> composite.
    `rt_full_spp` forces a full mask of that many samples (full ray-traced
    reference: every pixel traced, composite overridden)."""
    cam, lens, light = cfg.camera, cfg.lens, cfg.light
    H, W = cam.height, cam.width
    gb = gbuffer(scene, cam, lens, light)
    depth = gb["depth"]
    rep = None
    V = None
    if prev_camera is not None and history is not None:
        rep = var_reproject(cam, depth, prev_camera, history)
        V = rep["V"]
    mk = mask(depth, gb["normal"], cfg.mask, V, cam, lens)
    spp = mk["spp"] if rt_full_spp is None else np.full((H, W), rt_full_spp, np.int32)
    rt = trace(scene, cam, lens, light, spp, seed=cfg.seed, frame=frame_index, view=view,
               per_ray=False)
    if rep is None:
        rep = dict(lum_m1=np.zeros((H, W)), lum_m2=np.zeros((H, W)),
                   flags=np.zeros((H, W), np.int32))
    hist = var_update(spp, rep, rt["lum_m1"], rt["lum_m2"], cfg.mask.var_alpha, depth)
    rc = None
    rcfg = getattr(cfg, "recon", None)
    if rcfg is not None and rcfg.enable:
        rh = recon_history if recon_history is not None else empty_recon_history(H, W)
        rc = recon(cam, depth, spp, prev_camera, rh, rt["hit_ratio"], rt["c_near"], rt["c_far"], rt["far_pos"],
                   rcfg.alpha, rt["px_amb"])
        rt = dict(rt, c_near=rc["c_near"], c_far=rc["c_far"])
    scfg = getattr(cfg, "spatial", None)
    sc = None
    if scfg is not None and scfg.enable:
        hacc = rc["history"]["planes"][3] if rc is not None else None
        sc = spatial(spp, rt["c_near"], rt["c_far"], rt["hit_ratio"], hacc, rt["coc_nf"], history_variance(hist),
                     scfg.n_taps, scfg.r_cap, scfg.v_clamp)
        rt = dict(rt, c_near=sc["c_near"], c_far=sc["c_far"])
    cpp = postfilter(cam, lens, gb["color"], depth, cfg.pp)
    comp = cfg.comp
    if rt_full_spp is not None:
        from dataclasses import replace
        comp = replace(comp, rt_override=1)
    pps = None
    if getattr(comp, "spec_y", 0.0) > 0.0:
        pps = postfilter_spec(cam, lens, gb["spec"], depth, cfg.pp)
    out = composite(cam, lens, gb["color"], cpp, depth, spp, rt["c_near"], rt["c_far"],
                    rt["hit_ratio"], comp, pps)
    return dict(gbuffer=gb, mask=mk, spp=spp, rt=rt, history=hist, reproj=rep, pp=cpp, out=out,
                recon=rc, spatial=sc, pp_spec=pps)


def empty_recon_history(H: int, W: int) -> dict:
    return dict(planes=np.zeros((8, H, W)), valid=np.zeros((H, W), np.int32), depth=np.zeros((H, W)))


def recon(camera, depth, spp, prev_camera, hist: dict, hit, c_near, c_far, far_pos, alpha=0.2,
          px_amb=None) -> dict:
    """Temporal reconstruction of the near and far traced colours (paper,
    Reconstruction): returns the reconstructed c_near, c_far, the new
    history and the ambiguity flags.  `prev_camera` None: no history."""
    cam, W, H = cam_args(camera)
    pc = None if prev_camera is None else cam_args(prev_camera)[0]
    cno, cfo = np.zeros((3, H, W)), np.zeros((3, H, W))
    ho, vo, zo = np.zeros((8, H, W)), np.zeros((H, W), np.int32), np.zeros((H, W))
    am = np.zeros((H, W), np.int32)
    lib().or_recon(_p(cam), W, H, _p(_f64(depth)), _p(_i32(spp)), _p(pc), _p(_f64(hist["planes"])),
                   _p(_i32(hist["valid"])), _p(_f64(hist["depth"])), _p(_f64(hit)), _p(_f64(c_near)),
                   _p(_f64(c_far)), _p(_f64(far_pos)), _p(None if px_amb is None else _i32(px_amb)), float(alpha),
                   _p(cno), _p(cfo), _p(ho), _p(vo), _p(zo), _p(am))
    return dict(c_near=cno, c_far=cfo, history=dict(planes=ho, valid=vo, depth=zo), amb=am)


SP_LMAX = 5


def sp_level(spp, c_near, c_far, hit, hit_acc, coc_nf, r_cap: float, level: int) -> np.ndarray:
    """The level-`level` texel sums of the spatial reconstruction, (10, HL, WL):
    near sums (3), near weight, far sums (3), far weight, radius sum, count."""
    sp = _i32(spp)
    H, W = sp.shape
    WL, HL = -(-W // (1 << level)), -(-H // (1 << level))
    out = np.zeros((10, HL, WL))
    lib().or_sp_level(W, H, _p(sp), _p(_f64(c_near)), _p(_f64(c_far)), _p(_f64(hit)),
                      _p(None if hit_acc is None else _f64(hit_acc)), _p(_f64(coc_nf)), float(r_cap),
                      int(level), _p(out))
    return out


def spatial(spp, c_near, c_far, hit, hit_acc, coc_nf, V, n_taps=24, r_cap=64.0, v_clamp=0.01) -> dict:
    """Spatial reconstruction of the near and far traced colours (paper,
    Reconstruction, last paragraph): returns c_near, c_far, `amb` (per
    pixel: 1 = level decision within relative 1e-5 of a level boundary,
    2 = a tap coordinate within its rounding band of a pixel boundary) and
    `cond`, the sensitivity of each output (near, far) to errors in the
    acceptances of the taps on or near the acceptance ramp.
    `hit_acc` None: the latest hit ratio stands for the accumulated one; `V`
    None: no variance estimate (full weight)."""
    sp = _i32(spp)
    H, W = sp.shape
    cno, cfo = np.zeros((3, H, W)), np.zeros((3, H, W))
    cond = np.zeros((2, H, W))
    amb = np.zeros((H, W), np.int32)
    lib().or_spatial(W, H, _p(sp), _p(_f64(c_near)), _p(_f64(c_far)), _p(_f64(hit)),
                     _p(None if hit_acc is None else _f64(hit_acc)), _p(_f64(coc_nf)),
                     _p(None if V is None else _f64(V)), int(n_taps), float(r_cap), float(v_clamp),
                     _p(cno), _p(cfo), _p(amb), _p(cond))
    return dict(c_near=cno, c_far=cfo, amb=amb, cond=cond)


def history_variance(hist: dict) -> np.ndarray:
    """The variance estimate a variance history holds: +inf where new,
    max(0, m2 - m1^2) where valid, 0 elsewhere."""
    fl = _i32(hist["flags"])
    V = np.maximum(0.0, _f64(hist["lum_m2"]) - _f64(hist["lum_m1"]) ** 2)
    V = np.where(fl & VALID, V, 0.0)
    return np.where(fl & NEW, np.inf, V)


def pp_composite_backward(camera, lens, color, depth, spp, c_near, c_far, hit, pp, cp, grad_out):
    """Adjoint of post-filter + composite: (dL/dC_r (3,H,W), dL/dS1, dL/dA)
    for dL/dout = grad_out, with depth, counts and traced colours fixed."""
    cam, W, H = cam_args(camera)
    gcol = np.zeros((3, H, W))
    gl = np.zeros(2)
    ppa = _f64([pp.n_taps, pp.tile, pp.r_cap, pp.bg_ramp_px])
    lib().or_pp_composite_backward(_p(cam), W, H, _p(_f64(lens.as_floats())), _p(_f64(color)), _p(_f64(depth)),
                                   _p(_i32(spp)), _p(_f64(c_near)), _p(_f64(c_far)), _p(_f64(hit)), _p(ppa),
                                   float(cp.h_t), int(cp.rt_override), _p(_f64(grad_out)), _p(gcol), _p(gl))
    return gcol, float(gl[0]), float(gl[1])


def pp_composite_forward(camera, lens, color, depth, spp, c_near, c_far, hit, pp, cp):
    """out(C_r, S1, A) of the differentiable form (post-filter then composite)."""
    cpp = postfilter(camera, lens, color, depth, pp)
    return composite(camera, lens, color, cpp, depth, spp, c_near, c_far, hit, cp)
