"""Thin Python binding of libhdof.so (the C ABI in include/hdof.h).

Argument marshalling only: every step of the hybrid depth-of-field path runs
in the library's HIP kernels.  PyTorch supplies device memory (tensors are
passed as raw ``data_ptr()`` values) and the stream (torch's current stream
unless one is given).  Each wrapper checks tensor device, dtype, contiguity
and size against what the kernels assume before anything is enqueued, and
raises ``HdofError`` on a non-OK status.  There is no fallback: if the
library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdof.so")
# a build variant (same ABI, other compile-time tuning) may be named by path
LIB_PATH = os.environ.get("HDOF_LIBRARY", LIB_PATH)

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2210_04981_amd.build` "
                      "(hipcc, gfx950).  There is no fallback path.")

_lib = C.CDLL(LIB_PATH)

F3 = C.c_float * 3


class Camera(C.Structure):
    _fields_ = [("eye", F3), ("right", F3), ("up", F3), ("fwd", F3),
                ("tan_half_fov_x", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class Lens(C.Structure):
    _fields_ = [("focal_length", C.c_float), ("aperture", C.c_float), ("focus_distance", C.c_float),
                ("blades", C.c_int32), ("rotation", C.c_float), ("sa", C.c_float)]


class Light(C.Structure):
    _fields_ = [("pos", F3), ("intensity", F3), ("ambient", F3)]


class MaskParams(C.Structure):
    _fields_ = [("sigma", C.c_float), ("tau_depth", C.c_float), ("tau_normal", C.c_float),
                ("tau_var", C.c_float), ("var_alpha", C.c_float), ("spp_max", C.c_int32),
                ("tile", C.c_int32), ("dilate", C.c_int32)]


class PPParams(C.Structure):
    _fields_ = [("n_taps", C.c_int32), ("tile", C.c_int32), ("r_cap", C.c_float),
                ("bg_ramp_px", C.c_float)]


class CompositeParams(C.Structure):
    _fields_ = [("h_t", C.c_float), ("rt_override", C.c_int32), ("spec_y", C.c_float)]


class ReconParams(C.Structure):
    _fields_ = [("enable", C.c_int32), ("alpha", C.c_float)]


class SpatialParams(C.Structure):
    _fields_ = [("enable", C.c_int32), ("n_taps", C.c_int32), ("r_cap", C.c_float), ("v_clamp", C.c_float)]


class FrameParams(C.Structure):
    _fields_ = [("mask", MaskParams), ("pp", PPParams), ("comp", CompositeParams), ("recon", ReconParams),
                ("spatial", SpatialParams)]


P = C.c_void_p


class GBufferBufs(C.Structure):
    _fields_ = [("depth", P), ("normal", P), ("albedo", P), ("color", P), ("tri_id", P), ("spec", P)]


class RTBufs(C.Structure):
    _fields_ = [("c_near", P), ("c_far", P), ("hit_ratio", P), ("lum_m1", P), ("lum_m2", P)]


class FrameBufs(C.Structure):
    _fields_ = [("gb", GBufferBufs), ("spp", P), ("offsets", P), ("total", P), ("rt", RTBufs),
                ("pp", P)]


class View(C.Structure):
    _fields_ = [("cam", Camera), ("lens", Lens), ("seed", C.c_uint32), ("frame", C.c_uint32),
                ("view", C.c_uint32), ("d_out", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("refill", C.c_int32), ("segments", C.c_int32), ("wave", C.c_int32),
                ("overlap", C.c_int32), ("overlap_ray_quantum", C.c_int32)]


class AutotuneReport(C.Structure):
    _fields_ = [("key", C.c_char * 256), ("best_ms", C.c_float), ("default_ms", C.c_float),
                ("candidates", C.c_int32), ("from_cache", C.c_int32)]


MAX_VIEWS = 64
POSTFILTER_NOALLOC_MAX_PX = 3686400  # HDOF_POSTFILTER_NOALLOC_MAX_PX


class SceneInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int32), ("n_nodes", C.c_int32), ("max_depth", C.c_int32),
                ("leaf_size", C.c_int32), ("device_bytes", C.c_int64)]


_S = C.c_int
_u32, _i32 = C.c_uint32, C.c_int32
_PROTOS = {
    "hdof_create": (_S, [C.c_int, C.POINTER(P)]),
    "hdof_destroy": (None, [P]),
    "hdof_status_str": (C.c_char_p, [_S]),
    "hdof_last_error": (C.c_char_p, []),
    "hdof_sync": (_S, [P, P]),
    "hdof_build_bvh": (_S, [P, P, P, _i32, C.POINTER(P), P]),
    "hdof_scene_destroy": (None, [P]),
    "hdof_scene_stats": (_S, [P, C.POINTER(SceneInfo)]),
    "hdof_gbuffer": (_S, [P, P, C.POINTER(Camera), C.POINTER(Lens), C.POINTER(Light), GBufferBufs, P]),
    "hdof_ray_mask": (_S, [P, C.POINTER(GBufferBufs), C.POINTER(Camera), C.POINTER(Camera),
                           C.POINTER(Lens), C.POINTER(MaskParams), P, P, P, P]),
    "hdof_trace_thin_lens": (_S, [P, P, C.POINTER(Camera), C.POINTER(Lens), C.POINTER(Light), _i32,
                                  P, P, P, _u32, _u32, _u32, RTBufs, P, P, P, P, P]),
    "hdof_rt_spatial": (_S, [P, _i32, _i32, P, RTBufs, P, P, P, C.POINTER(SpatialParams), P, P, P]),
    "hdof_rt_reconstruct": (_S, [P, C.POINTER(Camera), C.POINTER(Camera), P, P, P, RTBufs,
                                 C.POINTER(ReconParams), P]),
    "hdof_recon_history_load": (_S, [P, _i32, _i32, P, P, P, P]),
    "hdof_recon_history_save": (_S, [P, P, P, P, P]),
    "hdof_recon_history_reset": (_S, [P]),
    "hdof_variance_update": (_S, [P, C.POINTER(Camera), C.POINTER(MaskParams), P, P, P, P, P]),
    "hdof_history_load": (_S, [P, _i32, _i32, P, P, P, P, P]),
    "hdof_history_save": (_S, [P, P, P, P, P, P]),
    "hdof_history_reset": (_S, [P]),
    "hdof_postfilter": (_S, [P, P, P, C.POINTER(Camera), C.POINTER(Lens), C.POINTER(PPParams), P, P]),
    "hdof_postfilter_noalloc": (_S, [P, P, P, C.POINTER(Camera), C.POINTER(Lens), C.POINTER(PPParams), P, P]),
    "hdof_composite": (_S, [P, P, P, P, P, RTBufs, C.POINTER(Camera), C.POINTER(Lens),
                            C.POINTER(CompositeParams), P, P, P]),
    "hdof_postfilter_specular": (_S, [P, P, P, P, P, C.POINTER(Camera), C.POINTER(Lens), C.POINTER(PPParams),
                                      P, P, P]),
    "hdof_scene_set_specular": (_S, [P, P, P]),
    "hdof_frame": (_S, [P, P, C.POINTER(Camera), C.POINTER(Camera), C.POINTER(Lens), C.POINTER(Light),
                        C.POINTER(FrameParams), _u32, _u32, _u32, P, C.POINTER(FrameBufs), P]),
    "hdof_profile_begin": (_S, [P]),
    "hdof_profile_end": (_S, [P, C.POINTER(C.c_float), C.POINTER(_i32)]),
    "hdof_frame_batched": (_S, [P, P, C.POINTER(Light), C.POINTER(FrameParams), _i32, C.POINTER(View), P]),
    "hdof_batch_create": (_S, [P, P, C.POINTER(Light), C.POINTER(FrameParams), _i32, C.POINTER(View),
                               C.POINTER(P)]),
    "hdof_batch_launch": (_S, [P, P]),
    "hdof_batch_destroy": (None, [P]),
    "hdof_set_tuning": (_S, [P, C.POINTER(Tuning)]),
    "hdof_get_tuning": (_S, [P, C.POINTER(Tuning)]),
    "hdof_autotune": (_S, [P, P, C.POINTER(Light), C.POINTER(FrameParams), _i32, C.POINTER(View), C.POINTER(Camera),
                           C.c_char_p, _i32,
                           C.POINTER(Tuning), C.POINTER(AutotuneReport), P]),
    "hdof_postfilter_composite_backward": (_S, [P, P, P, P, RTBufs, C.POINTER(Camera), C.POINTER(Lens),
                                                C.POINTER(PPParams), C.POINTER(CompositeParams), P, P, P, P]),
    "hdof_counters_begin": (_S, [P]),
    "hdof_counters_end": (_S, [P, C.POINTER(C.c_int64)]),
}

PROFILE_STAGES = ("gbuffer", "ray_mask", "queue_fill", "trace", "rt_reduce", "var_update", "recon", "pp_prep",
                  "pp_gather", "composite")
for _name, (_res, _args) in _PROTOS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_PROTOS)


class HdofError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.hdof_last_error().decode()
        super().__init__(f"{where}: {_lib.hdof_status_str(status).decode()}: {msg}")


def _check(status: int, where: str) -> None:
    if status != 0:
        raise HdofError(status, where)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t: torch.Tensor | None, dtype, numel: int | None, name: str) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name}: expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")
    return t.data_ptr()


def camera(eye, right, up, fwd, tan_half_fov_x, width, height) -> Camera:
    return Camera(F3(*eye), F3(*right), F3(*up), F3(*fwd), float(tan_half_fov_x), int(width), int(height))


def lens(focal_length, aperture, focus_distance, blades=0, rotation=0.0, sa=0.0) -> Lens:
    return Lens(float(focal_length), float(aperture), float(focus_distance), int(blades), float(rotation), float(sa))


def light(pos, intensity, ambient) -> Light:
    return Light(F3(*pos), F3(*intensity), F3(*ambient))


def mask_params(sigma=1.0, tau_depth=0.05, tau_normal=0.1, tau_var=0.01, var_alpha=0.2, spp_max=8,
                tile=8, dilate=1) -> MaskParams:
    return MaskParams(sigma, tau_depth, tau_normal, tau_var, var_alpha, spp_max, tile, dilate)


def pp_params(n_taps=48, tile=16, r_cap=64.0, bg_ramp_px=1.0) -> PPParams:
    return PPParams(n_taps, tile, r_cap, bg_ramp_px)


def composite_params(h_t=0.5, rt_override=0, spec_y=0.0) -> CompositeParams:
    return CompositeParams(h_t, rt_override, spec_y)


# ----------------------------------------------------------------------------
# context and scene
# ----------------------------------------------------------------------------

class Context:
    """Owns an hdof_ctx (device, scratch, variance history)."""

    def __init__(self, device: int = 0):
        h = P()
        _check(_lib.hdof_create(int(device), C.byref(h)), "hdof_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _lib.hdof_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self, stream=None):
        _check(_lib.hdof_sync(self.handle, _stream(stream)), "hdof_sync")


class Scene:
    """Owns an hdof_scene (BVH + triangles + albedo on the device)."""

    def __init__(self, handle, ctx: Context, n_tris: int):
        self.handle = handle
        self.ctx = ctx
        self.n_tris = n_tris

    def stats(self) -> dict:
        s = SceneInfo()
        _check(_lib.hdof_scene_stats(self.handle, C.byref(s)), "hdof_scene_stats")
        return dict(n_tris=s.n_tris, n_nodes=s.n_nodes, max_depth=s.max_depth,
                    device_bytes=s.device_bytes)

    def close(self):
        if self.handle:
            _lib.hdof_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hdof_create(device: int = 0) -> Context:
    return Context(device)


def hdof_scene_set_specular(scene: "Scene", spec: torch.Tensor | None, stream=None) -> None:
    """Per-triangle (k_s, shininess) specular table (n, 2), or None (Lambertian)."""
    _check(_lib.hdof_scene_set_specular(scene.handle, _ptr(spec, torch.float32, 2 * scene.n_tris, "spec"),
                                        _stream(stream)), "hdof_scene_set_specular")


def hdof_build_bvh(ctx: Context, verts: torch.Tensor, albedo: torch.Tensor, stream=None) -> Scene:
    n = verts.shape[0]
    pv = _ptr(verts, torch.float32, 9 * n, "verts")
    pa = _ptr(albedo, torch.float32, 3 * n, "albedo")
    if verts.numel() != 9 * n or albedo.numel() != 3 * n:
        raise ValueError("verts must be (n, 9) and albedo (n, 3)")
    h = P()
    _check(_lib.hdof_build_bvh(ctx.handle, pv, pa, int(n), C.byref(h), _stream(stream)), "hdof_build_bvh")
    return Scene(h, ctx, n)


# ----------------------------------------------------------------------------
# stages
# ----------------------------------------------------------------------------

@dataclass
class GBuffer:
    depth: torch.Tensor
    normal: torch.Tensor
    albedo: torch.Tensor
    color: torch.Tensor
    tri_id: torch.Tensor
    spec: torch.Tensor | None = None  # specular luminance (optional)

    @staticmethod
    def empty(H: int, W: int, device="cuda", spec: bool = False) -> "GBuffer":
        f = dict(dtype=torch.float32, device=device)
        return GBuffer(torch.empty(H, W, **f), torch.empty(3, H, W, **f), torch.empty(3, H, W, **f),
                       torch.empty(3, H, W, **f), torch.empty(H, W, dtype=torch.int32, device=device),
                       torch.empty(H, W, **f) if spec else None)

    def bufs(self) -> GBufferBufs:
        n = self.depth.numel()
        return GBufferBufs(_ptr(self.depth, torch.float32, n, "depth"),
                           _ptr(self.normal, torch.float32, 3 * n, "normal"),
                           _ptr(self.albedo, torch.float32, 3 * n, "albedo"),
                           _ptr(self.color, torch.float32, 3 * n, "color"),
                           _ptr(self.tri_id, torch.int32, n, "tri_id"),
                           _ptr(self.spec, torch.float32, n, "spec"))


@dataclass
class RTResult:
    c_near: torch.Tensor
    c_far: torch.Tensor
    hit_ratio: torch.Tensor
    lum_m1: torch.Tensor
    lum_m2: torch.Tensor

    @staticmethod
    def empty(H: int, W: int, device="cuda") -> "RTResult":
        f = dict(dtype=torch.float32, device=device)
        return RTResult(torch.empty(3, H, W, **f), torch.empty(3, H, W, **f), torch.empty(H, W, **f),
                        torch.empty(H, W, **f), torch.empty(H, W, **f))

    def bufs(self, n: int) -> RTBufs:
        return RTBufs(_ptr(self.c_near, torch.float32, 3 * n, "c_near"),
                      _ptr(self.c_far, torch.float32, 3 * n, "c_far"),
                      _ptr(self.hit_ratio, torch.float32, n, "hit_ratio"),
                      _ptr(self.lum_m1, torch.float32, n, "lum_m1"),
                      _ptr(self.lum_m2, torch.float32, n, "lum_m2"))


def _npx(cam: Camera) -> int:
    return int(cam.width) * int(cam.height)


def hdof_gbuffer(ctx: Context, scene: Scene, cam: Camera, lns: Lens, lit: Light, out: GBuffer | None = None,
                 stream=None) -> GBuffer:
    if out is None:
        out = GBuffer.empty(cam.height, cam.width)
    if out.depth.numel() < _npx(cam):
        raise ValueError("G-buffer smaller than the camera image")
    _check(_lib.hdof_gbuffer(ctx.handle, scene.handle, C.byref(cam), C.byref(lns), C.byref(lit), out.bufs(),
                             _stream(stream)), "hdof_gbuffer")
    return out


def hdof_ray_mask(ctx: Context, depth: torch.Tensor, normal: torch.Tensor, cam: Camera, prev: Camera | None,
                  lns: Lens, mp: MaskParams, spp=None, offsets=None, total=None, stream=None):
    n = _npx(cam)
    dev = depth.device
    spp = torch.empty(cam.height, cam.width, dtype=torch.uint8, device=dev) if spp is None else spp
    offsets = torch.empty(cam.height, cam.width, dtype=torch.int32, device=dev) if offsets is None else offsets
    total = torch.empty(1, dtype=torch.int32, device=dev) if total is None else total
    gb = GBufferBufs(_ptr(depth, torch.float32, n, "depth"), _ptr(normal, torch.float32, 3 * n, "normal"),
                     None, None, None)
    _check(_lib.hdof_ray_mask(ctx.handle, C.byref(gb), C.byref(cam), C.byref(prev) if prev is not None else None,
                              C.byref(lns), C.byref(mp), _ptr(spp, torch.uint8, n, "spp"),
                              _ptr(offsets, torch.int32, n, "offsets"), _ptr(total, torch.int32, 1, "total"),
                              _stream(stream)), "hdof_ray_mask")
    return spp, offsets, total


def hdof_trace_thin_lens(ctx: Context, scene: Scene, cam: Camera, lns: Lens, lit: Light, spp_max: int,
                         spp: torch.Tensor, offsets: torch.Tensor, total: torch.Tensor, seed=0, frame=0, view=0,
                         out: RTResult | None = None, ray_tri_id: torch.Tensor | None = None,
                         ray_depth: torch.Tensor | None = None, far_pos: torch.Tensor | None = None,
                         coc_nf: torch.Tensor | None = None, stream=None) -> RTResult:
    n = _npx(cam)
    out = RTResult.empty(cam.height, cam.width) if out is None else out
    cap = n * int(spp_max)
    _check(_lib.hdof_trace_thin_lens(ctx.handle, scene.handle, C.byref(cam), C.byref(lns), C.byref(lit),
                                     int(spp_max), _ptr(spp, torch.uint8, n, "spp"),
                                     _ptr(offsets, torch.int32, n, "offsets"), _ptr(total, torch.int32, 1, "total"),
                                     int(seed), int(frame), int(view), out.bufs(n),
                                     _ptr(ray_tri_id, torch.int32, cap, "ray_tri_id"),
                                     _ptr(ray_depth, torch.float32, cap, "ray_depth"),
                                     _ptr(far_pos, torch.float32, 4 * n, "far_pos"),
                                     _ptr(coc_nf, torch.float32, 2 * n, "coc_nf"), _stream(stream)),
           "hdof_trace_thin_lens")
    return out


def hdof_rt_spatial(ctx: Context, H: int, W: int, spp, rt: RTResult, hit_acc, coc_nf, variance,
                    sp: "SpatialParams", c_near_out=None, c_far_out=None, stream=None):
    """Spatial reconstruction of rt.c_near / rt.c_far into new planes
    (returned as (c_near, c_far)); hit_acc and variance may be None."""
    n = H * W
    cno = torch.empty(3, H, W, device="cuda") if c_near_out is None else c_near_out
    cfo = torch.empty(3, H, W, device="cuda") if c_far_out is None else c_far_out
    _check(_lib.hdof_rt_spatial(ctx.handle, int(W), int(H), _ptr(spp, torch.uint8, n, "spp"), rt.bufs(n),
                                _ptr(hit_acc, torch.float32, n, "hit_acc"), _ptr(coc_nf, torch.float32, 2 * n, "coc_nf"),
                                _ptr(variance, torch.float32, n, "variance"), C.byref(sp),
                                _ptr(cno, torch.float32, 3 * n, "c_near_out"), _ptr(cfo, torch.float32, 3 * n, "c_far_out"),
                                _stream(stream)), "hdof_rt_spatial")
    return cno, cfo


def hdof_rt_reconstruct(ctx: Context, cam: Camera, prev: Camera | None, depth, spp, far_pos, rt: RTResult,
                        rp: "ReconParams", stream=None) -> RTResult:
    """Temporal reconstruction: rt.c_near and rt.c_far are updated in place."""
    n = _npx(cam)
    _check(_lib.hdof_rt_reconstruct(ctx.handle, C.byref(cam), C.byref(prev) if prev is not None else None,
                                    _ptr(depth, torch.float32, n, "depth"), _ptr(spp, torch.uint8, n, "spp"),
                                    _ptr(far_pos, torch.float32, 4 * n, "far_pos"), rt.bufs(n), C.byref(rp),
                                    _stream(stream)), "hdof_rt_reconstruct")
    return rt


def hdof_recon_history_load(ctx: Context, planes, valid, depth, stream=None):
    H, W = depth.shape
    n = H * W
    _check(_lib.hdof_recon_history_load(ctx.handle, W, H, _ptr(planes, torch.float32, 8 * n, "planes"),
                                        _ptr(valid, torch.uint8, n, "valid"), _ptr(depth, torch.float32, n, "depth"),
                                        _stream(stream)), "hdof_recon_history_load")


def hdof_recon_history_save(ctx: Context, H: int, W: int, stream=None) -> dict:
    out = dict(planes=torch.empty(8, H, W, dtype=torch.float32, device="cuda"),
               valid=torch.empty(H, W, dtype=torch.uint8, device="cuda"),
               depth=torch.empty(H, W, dtype=torch.float32, device="cuda"))
    _check(_lib.hdof_recon_history_save(ctx.handle, out["planes"].data_ptr(), out["valid"].data_ptr(),
                                        out["depth"].data_ptr(), _stream(stream)), "hdof_recon_history_save")
    return out


def hdof_recon_history_reset(ctx: Context):
    _check(_lib.hdof_recon_history_reset(ctx.handle), "hdof_recon_history_reset")


def hdof_variance_update(ctx: Context, cam: Camera, mp: MaskParams, spp, depth, lum_m1, lum_m2, stream=None):
    n = _npx(cam)
    _check(_lib.hdof_variance_update(ctx.handle, C.byref(cam), C.byref(mp), _ptr(spp, torch.uint8, n, "spp"),
                                     _ptr(depth, torch.float32, n, "depth"),
                                     _ptr(lum_m1, torch.float32, n, "lum_m1"),
                                     _ptr(lum_m2, torch.float32, n, "lum_m2"), _stream(stream)),
           "hdof_variance_update")


def hdof_history_load(ctx: Context, lum_m1, lum_m2, flags, depth, stream=None):
    H, W = depth.shape
    n = H * W
    _check(_lib.hdof_history_load(ctx.handle, W, H, _ptr(lum_m1, torch.float32, n, "lum_m1"),
                                  _ptr(lum_m2, torch.float32, n, "lum_m2"), _ptr(flags, torch.uint8, n, "flags"),
                                  _ptr(depth, torch.float32, n, "depth"), _stream(stream)), "hdof_history_load")


def hdof_history_save(ctx: Context, H: int, W: int, stream=None) -> dict:
    f = dict(dtype=torch.float32, device="cuda")
    out = dict(lum_m1=torch.empty(H, W, **f), lum_m2=torch.empty(H, W, **f),
               flags=torch.empty(H, W, dtype=torch.uint8, device="cuda"), depth=torch.empty(H, W, **f))
    _check(_lib.hdof_history_save(ctx.handle, out["lum_m1"].data_ptr(), out["lum_m2"].data_ptr(),
                                  out["flags"].data_ptr(), out["depth"].data_ptr(), _stream(stream)),
           "hdof_history_save")
    return out


def hdof_history_reset(ctx: Context):
    _check(_lib.hdof_history_reset(ctx.handle), "hdof_history_reset")


def hdof_postfilter(ctx: Context, color, depth, cam: Camera, lns: Lens, pp: PPParams, out=None, stream=None):
    n = _npx(cam)
    out = torch.empty(3, cam.height, cam.width, dtype=torch.float32, device=color.device) if out is None else out
    _check(_lib.hdof_postfilter(ctx.handle, _ptr(color, torch.float32, 3 * n, "color"),
                                _ptr(depth, torch.float32, n, "depth"), C.byref(cam), C.byref(lns), C.byref(pp),
                                _ptr(out, torch.float32, 3 * n, "out"), _stream(stream)), "hdof_postfilter")
    return out


def hdof_postfilter_noalloc(ctx: Context, color, depth, cam: Camera, lns: Lens, pp: PPParams, out,
                            stream=None):
    """hdof_postfilter with the library's fixed device scratch (no device
    allocation in the call); `out` is required."""
    n = _npx(cam)
    _check(_lib.hdof_postfilter_noalloc(ctx.handle, _ptr(color, torch.float32, 3 * n, "color"),
                                        _ptr(depth, torch.float32, n, "depth"), C.byref(cam), C.byref(lns),
                                        C.byref(pp), _ptr(out, torch.float32, 3 * n, "out"), _stream(stream)),
           "hdof_postfilter_noalloc")
    return out


def hdof_composite(ctx: Context, color, pp_col, depth, spp, rt: RTResult, cam: Camera, lns: Lens,
                   cp: CompositeParams, out=None, stream=None, pp_spec=None):
    n = _npx(cam)
    out = torch.empty(3, cam.height, cam.width, dtype=torch.float32, device=color.device) if out is None else out
    _check(_lib.hdof_composite(ctx.handle, _ptr(color, torch.float32, 3 * n, "color"),
                               _ptr(pp_col, torch.float32, 3 * n, "pp"), _ptr(depth, torch.float32, n, "depth"),
                               _ptr(spp, torch.uint8, n, "spp"), rt.bufs(n), C.byref(cam), C.byref(lns),
                               C.byref(cp), _ptr(pp_spec, torch.float32, n, "pp_spec"),
                               _ptr(out, torch.float32, 3 * n, "out"), _stream(stream)),
           "hdof_composite")
    return out


def hdof_postfilter_specular(ctx: Context, color, depth, spec, spp, cam: Camera, lns: Lens, pp: PPParams,
                             out=None, spec_out=None, stream=None):
    """The post-filter plus the post-filtered specular luminance: (out, spec_out)."""
    n = _npx(cam)
    out = torch.empty(3, cam.height, cam.width, dtype=torch.float32, device=color.device) if out is None else out
    spec_out = torch.empty(cam.height, cam.width, dtype=torch.float32, device=color.device) \
        if spec_out is None else spec_out
    _check(_lib.hdof_postfilter_specular(ctx.handle, _ptr(color, torch.float32, 3 * n, "color"),
                                         _ptr(depth, torch.float32, n, "depth"), _ptr(spec, torch.float32, n, "spec"),
                                         _ptr(spp, torch.uint8, n, "spp"), C.byref(cam), C.byref(lns), C.byref(pp),
                                         _ptr(out, torch.float32, 3 * n, "out"),
                                         _ptr(spec_out, torch.float32, n, "spec_out"), _stream(stream)),
           "hdof_postfilter_specular")
    return out, spec_out


@dataclass
class FrameKeep:
    """Caller-owned intermediates of hdof_frame (all optional)."""
    gb: GBuffer | None = None
    spp: torch.Tensor | None = None
    offsets: torch.Tensor | None = None
    total: torch.Tensor | None = None
    rt: RTResult | None = None
    pp: torch.Tensor | None = None

    @staticmethod
    def empty(H: int, W: int, device="cuda") -> "FrameKeep":
        return FrameKeep(GBuffer.empty(H, W, device), torch.empty(H, W, dtype=torch.uint8, device=device),
                         torch.empty(H, W, dtype=torch.int32, device=device),
                         torch.empty(1, dtype=torch.int32, device=device), RTResult.empty(H, W, device),
                         torch.empty(3, H, W, dtype=torch.float32, device=device))

    def bufs(self, n: int) -> FrameBufs:
        fb = FrameBufs()
        if self.gb is not None:
            fb.gb = self.gb.bufs()
        if self.rt is not None:
            fb.rt = self.rt.bufs(n)
        fb.spp = _ptr(self.spp, torch.uint8, n, "spp")
        fb.offsets = _ptr(self.offsets, torch.int32, n, "offsets")
        fb.total = _ptr(self.total, torch.int32, 1, "total")
        fb.pp = _ptr(self.pp, torch.float32, 3 * n, "pp")
        return fb


def hdof_frame(ctx: Context, scene: Scene, cam: Camera, prev: Camera | None, lns: Lens, lit: Light,
               params: FrameParams, seed=0, frame=0, view=0, out=None, keep: FrameKeep | None = None,
               stream=None):
    n = _npx(cam)
    out = torch.empty(3, cam.height, cam.width, dtype=torch.float32, device="cuda") if out is None else out
    fb = keep.bufs(n) if keep is not None else None
    _check(_lib.hdof_frame(ctx.handle, scene.handle, C.byref(cam), C.byref(prev) if prev is not None else None,
                           C.byref(lns), C.byref(lit), C.byref(params), int(seed), int(frame), int(view),
                           _ptr(out, torch.float32, 3 * n, "out"), C.byref(fb) if fb is not None else None,
                           _stream(stream)), "hdof_frame")
    return out


# ----------------------------------------------------------------------------
# duck-typed constructors (objects with the same field names)
# ----------------------------------------------------------------------------

def camera_of(c) -> Camera:
    return camera(c.eye, c.right, c.up, c.fwd, c.tan_half_fov_x, c.width, c.height)


def lens_of(l) -> Lens:
    return lens(l.focal_length, l.aperture, l.focus_distance, getattr(l, "blades", 0), getattr(l, "rotation", 0.0),
                getattr(l, "sa", 0.0))


def light_of(l) -> Light:
    return light(l.pos, l.intensity, l.ambient)


def mask_params_of(m) -> MaskParams:
    return mask_params(m.sigma, m.tau_depth, m.tau_normal, m.tau_var, m.var_alpha, m.spp_max, m.tile, m.dilate)


def pp_params_of(p) -> PPParams:
    return pp_params(p.n_taps, p.tile, p.r_cap, p.bg_ramp_px)


def composite_params_of(c) -> CompositeParams:
    return composite_params(c.h_t, c.rt_override, float(getattr(c, "spec_y", 0.0)))


def recon_params_of(r) -> ReconParams:
    return ReconParams(int(bool(r.enable)), float(r.alpha))


def spatial_params_of(sp) -> SpatialParams:
    return SpatialParams(int(bool(sp.enable)), int(sp.n_taps), float(sp.r_cap), float(sp.v_clamp))


def frame_params_of(cfg) -> FrameParams:
    rc = getattr(cfg, "recon", None)
    sc = getattr(cfg, "spatial", None)
    return FrameParams(mask_params_of(cfg.mask), pp_params_of(cfg.pp), composite_params_of(cfg.comp),
                       recon_params_of(rc) if rc is not None else ReconParams(0, 0.2),
                       spatial_params_of(sc) if sc is not None else SpatialParams(0, 24, 64.0, 0.01))


def hdof_profile_begin(ctx: Context) -> None:
    _check(_lib.hdof_profile_begin(ctx.handle), "hdof_profile_begin")


def hdof_profile_end(ctx: Context) -> tuple[dict, int]:
    """Mean ms per stage over the frames recorded since hdof_profile_begin."""
    ms = (C.c_float * len(PROFILE_STAGES))()
    n = C.c_int32(0)
    _check(_lib.hdof_profile_end(ctx.handle, ms, C.byref(n)), "hdof_profile_end")
    return {k: float(v) for k, v in zip(PROFILE_STAGES, ms)}, int(n.value)


def hdof_counters_begin(ctx: Context) -> None:
    _check(_lib.hdof_counters_begin(ctx.handle), "hdof_counters_begin")


def hdof_counters_end(ctx: Context) -> dict:
    """Traversal work since hdof_counters_begin: rays, node visits, triangle tests."""
    c = (C.c_int64 * 6)()
    _check(_lib.hdof_counters_end(ctx.handle, c), "hdof_counters_end")
    return dict(gbuffer_rays=c[0], gbuffer_visits=c[1], gbuffer_tests=c[2],
                trace_rays=c[3], trace_visits=c[4], trace_tests=c[5])


# ----------------------------------------------------------------------------
# batched form and tuning
# ----------------------------------------------------------------------------

def _views(views, outs) -> "C.Array":
    if len(views) != len(outs) or not 1 <= len(views) <= MAX_VIEWS:
        raise ValueError(f"need 1..{MAX_VIEWS} views, one output each")
    arr = (View * len(views))()
    for i, (v, o) in enumerate(zip(views, outs)):
        cam, lns, seed, frame, view = v
        arr[i] = View(cam, lns, int(seed), int(frame), int(view),
                      _ptr(o, torch.float32, 3 * int(cam.width) * int(cam.height), f"out[{i}]"))
    return arr


def hdof_frame_batched(ctx: Context, scene: Scene, lit: Light, params: FrameParams, views, outs=None,
                       stream=None):
    """views: list of (Camera, Lens, seed, frame, view); returns the outputs."""
    if outs is None:
        outs = [torch.empty(3, v[0].height, v[0].width, dtype=torch.float32, device="cuda") for v in views]
    arr = _views(views, outs)
    _check(_lib.hdof_frame_batched(ctx.handle, scene.handle, C.byref(lit), C.byref(params), len(views), arr,
                                   _stream(stream)), "hdof_frame_batched")
    return outs


class Batch:
    """A batch of views captured into a HIP graph (hdof_batch_create)."""

    def __init__(self, ctx: Context, scene: Scene, lit: Light, params: FrameParams, views, outs):
        self.outs = outs
        arr = _views(views, outs)
        h = P()
        _check(_lib.hdof_batch_create(ctx.handle, scene.handle, C.byref(lit), C.byref(params), len(views), arr,
                                      C.byref(h)), "hdof_batch_create")
        self.handle = h
        self._keep = (ctx, scene)

    def launch(self, stream=None):
        _check(_lib.hdof_batch_launch(self.handle, _stream(stream)), "hdof_batch_launch")
        return self.outs

    def close(self):
        if self.handle:
            _lib.hdof_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hdof_set_tuning(ctx: Context, blocks_per_cu=10, refill=64, segments=8, wave=0, overlap=1,
                    overlap_ray_quantum=140000) -> None:
    t = Tuning(int(blocks_per_cu), int(refill), int(segments), int(wave), int(overlap), int(overlap_ray_quantum))
    _check(_lib.hdof_set_tuning(ctx.handle, C.byref(t)), "hdof_set_tuning")


def hdof_autotune(ctx: Context, scene: Scene, lit: Light, params: FrameParams, views, outs=None,
                  cache_path: str | None = None, force: bool = False, stream=None,
                  prev: Camera | None = None) -> tuple[dict, dict]:
    """Search (or load from `cache_path`) the fastest launch shape for the
    workload: one view = hdof_frame, several = hdof_frame_batched; `views`
    as for hdof_frame_batched.  prev (one view only): time frames that carry
    the variance history, with this previous camera.  Returns (tuning,
    report); the tuning is set on the context."""
    if outs is None:
        outs = [torch.empty(3, v[0].height, v[0].width, dtype=torch.float32, device="cuda") for v in views]
    arr = _views(views, outs)
    t = Tuning()
    rep = AutotuneReport()
    _check(_lib.hdof_autotune(ctx.handle, scene.handle, C.byref(lit), C.byref(params), len(views), arr,
                              None if prev is None else C.byref(prev),
                              None if cache_path is None else str(cache_path).encode(), int(bool(force)),
                              C.byref(t), C.byref(rep), _stream(stream)), "hdof_autotune")
    tuning = dict(blocks_per_cu=t.blocks_per_cu, refill=t.refill, segments=t.segments, wave=t.wave,
                  overlap=t.overlap, overlap_ray_quantum=t.overlap_ray_quantum)
    report = dict(key=rep.key.decode(), best_ms=rep.best_ms, default_ms=rep.default_ms,
                  candidates=rep.candidates, from_cache=bool(rep.from_cache))
    return tuning, report


def hdof_get_tuning(ctx: Context) -> dict:
    t = Tuning()
    _check(_lib.hdof_get_tuning(ctx.handle, C.byref(t)), "hdof_get_tuning")
    return dict(blocks_per_cu=t.blocks_per_cu, refill=t.refill, segments=t.segments, wave=t.wave,
                overlap=t.overlap, overlap_ray_quantum=t.overlap_ray_quantum)


# ----------------------------------------------------------------------------
# differentiable form
# ----------------------------------------------------------------------------

def hdof_postfilter_composite_backward(ctx: Context, color, depth, spp, rt: RTResult, cam: Camera, lns: Lens,
                                       pp: PPParams, cp: CompositeParams, grad_out, grad_color=None,
                                       grad_lens=None, stream=None):
    """dL/dC_r (3,H,W) and dL/d(S1, A) (2,) on the device for dL/dout = grad_out."""
    n = _npx(cam)
    grad_color = torch.empty(3, cam.height, cam.width, dtype=torch.float32, device=color.device) \
        if grad_color is None else grad_color
    grad_lens = torch.empty(2, dtype=torch.float32, device=color.device) if grad_lens is None else grad_lens
    _check(_lib.hdof_postfilter_composite_backward(
        ctx.handle, _ptr(color, torch.float32, 3 * n, "color"), _ptr(depth, torch.float32, n, "depth"),
        _ptr(spp, torch.uint8, n, "spp"), rt.bufs(n), C.byref(cam), C.byref(lns), C.byref(pp), C.byref(cp),
        _ptr(grad_out, torch.float32, 3 * n, "grad_out"), _ptr(grad_color, torch.float32, 3 * n, "grad_color"),
        _ptr(grad_lens, torch.float32, 2, "grad_lens"), _stream(stream)), "hdof_postfilter_composite_backward")
    return grad_color, grad_lens


class HybridDoFPost(torch.autograd.Function):
    """out = composite(C_r, postfilter(C_r; S1, A); S1, A) with depth, ray
    counts and ray-traced colours fixed.  Differentiable in the sharp colour,
    the focus distance and the aperture; the backward pass is the library's
    hand-written adjoint (gather recomputed, nothing stored but the inputs).

    apply(color, focus, aperture, depth, spp, rt, camera, focal_length, pp, comp, ctx)
    with focus and aperture 0-dim float tensors."""

    @staticmethod
    def forward(fctx, color, focus, aperture, depth, spp, rt, cam, focal_length, pp, comp, hctx):
        lns = lens(focal_length, float(aperture), float(focus))
        cpp = hdof_postfilter(hctx, color, depth, cam, lns, pp)
        out = hdof_composite(hctx, color, cpp, depth, spp, rt, cam, lns, comp)
        fctx.save_for_backward(color, depth, spp)
        fctx.meta = (rt, cam, lns, pp, comp, hctx)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        color, depth, spp = fctx.saved_tensors
        rt, cam, lns, pp, comp, hctx = fctx.meta
        gc, gl = hdof_postfilter_composite_backward(hctx, color, depth, spp, rt, cam, lns, pp, comp,
                                                    grad_out.contiguous())
        return gc, gl[0], gl[1], None, None, None, None, None, None, None, None
