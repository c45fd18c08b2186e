// api.hip -- the C ABI declared in include/hdof.h: argument validation,
// context and scene lifetimes, scratch management, stage sequencing.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "hdof_internal.h"

static thread_local char g_err[512] = "";

hdof_status hdof_set_error(hdof_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

hdof_status hdof_ensure(Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 1;
  if (b.bytes >= bytes) return HDOF_OK;
  if (b.p) {
    // the old buffer may still be read by work in flight
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hdof_set_error(HDOF_ERR_HIP, "hipDeviceSynchronize: %s", hipGetErrorString(e));
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 8;  // some slack so small growth does not reallocate
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return hdof_set_error(HDOF_ERR_OOM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
  }
  b.bytes = want;
  return HDOF_OK;
}

static void buf_free(Buf& b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
#define REQUIRE(cond, ...)                                      \
  do {                                                          \
    if (!(cond)) return hdof_set_error(HDOF_ERR_INVALID_ARG, __VA_ARGS__); \
  } while (0)

static bool finite3(const float* v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

static hdof_status check_camera(const hdof_camera* c, const char* what) {
  REQUIRE(c, "%s camera is NULL", what);
  REQUIRE(c->width > 0 && c->height > 0 && c->width <= 16384 && c->height <= 16384,
          "%s camera size %dx%d outside [1, 16384]", what, c->width, c->height);
  REQUIRE(isfinite(c->tan_half_fov_x) && c->tan_half_fov_x > 0.0f && c->tan_half_fov_x < 1e4f,
          "%s camera tan_half_fov_x must be finite and > 0", what);
  REQUIRE(finite3(c->eye) && finite3(c->right) && finite3(c->up) && finite3(c->fwd),
          "%s camera vectors must be finite", what);
  return HDOF_OK;
}

static hdof_status check_lens(const hdof_lens* l) {
  REQUIRE(l, "lens is NULL");
  REQUIRE(isfinite(l->focal_length) && l->focal_length > 0.0f, "focal_length must be > 0");
  REQUIRE(isfinite(l->aperture) && l->aperture >= 0.0f, "aperture must be >= 0");
  REQUIRE(isfinite(l->focus_distance) && l->focus_distance > l->focal_length,
          "focus_distance (S1) must exceed the focal length");
  REQUIRE(l->blades == 0 || (l->blades >= 3 && l->blades <= HDOF_MAX_BLADES), "blades must be 0 or in [3, %d]",
          HDOF_MAX_BLADES);
  REQUIRE(isfinite(l->rotation) && fabsf(l->rotation) <= 1e3f, "rotation must be finite");
  REQUIRE(isfinite(l->sa) && l->sa >= -4.0f && l->sa <= 4.0f, "sa must be in [-4, 4]");
  return HDOF_OK;
}

static hdof_status check_light(const hdof_light* l) {
  REQUIRE(l, "light is NULL");
  REQUIRE(finite3(l->pos) && finite3(l->intensity) && finite3(l->ambient), "light values must be finite");
  return HDOF_OK;
}

static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

static hdof_status check_mask(const hdof_mask_params* m) {
  REQUIRE(m, "mask params are NULL");
  REQUIRE(isfinite(m->sigma) && m->sigma > 0.0f && m->sigma <= 2.0f, "mask sigma must be in (0, 2]");
  REQUIRE(m->tau_depth > 0.0f && m->tau_normal > 0.0f && m->tau_var > 0.0f && isfinite(m->tau_depth) &&
              isfinite(m->tau_normal) && isfinite(m->tau_var),
          "mask thresholds must be finite and > 0");
  REQUIRE(m->var_alpha >= 0.0f && m->var_alpha <= 1.0f, "var_alpha must be in [0, 1]");
  REQUIRE(m->spp_max >= 1 && m->spp_max <= 255, "spp_max must be in [1, 255]");
  REQUIRE(m->tile == 0 || pow2_in(m->tile, 1, 16), "mask tile must be 0 (scaled by the CoC), 1, 2, 4, 8 or 16");
  REQUIRE(m->dilate >= 0 && m->dilate <= 8, "mask dilate must be in [0, 8]");
  return HDOF_OK;
}

static hdof_status check_pp(const hdof_pp_params* p) {
  REQUIRE(p, "post-filter params are NULL");
  REQUIRE(p->n_taps >= 1 && p->n_taps <= 256, "n_taps must be in [1, 256]");
  REQUIRE(pow2_in(p->tile, 4, 16), "post-filter tile must be 4, 8 or 16");
  REQUIRE(isfinite(p->r_cap) && p->r_cap >= 0.0f && p->r_cap <= 256.0f, "r_cap must be in [0, 256]");
  REQUIRE(isfinite(p->bg_ramp_px) && p->bg_ramp_px > 0.0f, "bg_ramp_px must be > 0");
  return HDOF_OK;
}

static hdof_status check_comp(const hdof_composite_params* c) {
  REQUIRE(c, "composite params are NULL");
  REQUIRE(isfinite(c->h_t) && c->h_t > 0.0f, "h_t must be > 0");
  REQUIRE(isfinite(c->spec_y) && c->spec_y >= 0.0f, "spec_y must be finite and >= 0");
  return HDOF_OK;
}

#define TRY(x)                        \
  do {                                \
    hdof_status s_ = (x);             \
    if (s_ != HDOF_OK) return s_;     \
  } while (0)

static hdof_status check_recon(const hdof_recon_params* r) {
  REQUIRE(r, "recon params are NULL");
  REQUIRE(r->enable == 0 || r->enable == 1, "recon enable must be 0 or 1");
  REQUIRE(isfinite(r->alpha) && r->alpha > 0.0f && r->alpha <= 1.0f, "recon alpha must be in (0, 1]");
  return HDOF_OK;
}

static hdof_status check_spatial(const hdof_spatial_params* sp) {
  REQUIRE(sp, "spatial params are NULL");
  REQUIRE(sp->enable == 0 || sp->enable == 1, "spatial enable must be 0 or 1");
  REQUIRE(sp->n_taps >= 1 && sp->n_taps <= 256, "spatial n_taps must be in [1, 256]");
  REQUIRE(isfinite(sp->r_cap) && sp->r_cap >= 0.0f && sp->r_cap <= 256.0f, "spatial r_cap must be in [0, 256]");
  REQUIRE(isfinite(sp->v_clamp) && sp->v_clamp > 0.0f, "spatial v_clamp must be finite and > 0");
  return HDOF_OK;
}

static hdof_status check_ctx(hdof_ctx* ctx) {
  REQUIRE(ctx, "context is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hdof_set_error(HDOF_ERR_HIP, "hipSetDevice: %s", hipGetErrorString(e));
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" const char* hdof_status_str(hdof_status s) {
  switch (s) {
    case HDOF_OK: return "HDOF_OK";
    case HDOF_ERR_INVALID_ARG: return "HDOF_ERR_INVALID_ARG";
    case HDOF_ERR_UNSUPPORTED: return "HDOF_ERR_UNSUPPORTED";
    case HDOF_ERR_OOM: return "HDOF_ERR_OOM";
    case HDOF_ERR_CAPACITY: return "HDOF_ERR_CAPACITY";
    case HDOF_ERR_HIP: return "HDOF_ERR_HIP";
  }
  return "HDOF_ERR_UNKNOWN";
}

extern "C" const char* hdof_last_error(void) { return g_err; }

extern "C" hdof_status hdof_create(int device, hdof_ctx** out) {
  REQUIRE(out, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return hdof_set_error(HDOF_ERR_UNSUPPORTED, "no HIP device available");
  REQUIRE(device >= 0 && device < n, "device %d out of range [0, %d)", device, n);
  hipDeviceProp_t prop;
  HDOF_HIP(hipGetDeviceProperties(&prop, device));
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "device %d is %s, this library is built for gfx950", device,
                          prop.gcnArchName);
  HDOF_HIP(hipSetDevice(device));
  hdof_ctx* c = new hdof_ctx();
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  e = hipMalloc(&c->d_flags, sizeof(int));
  if (e != hipSuccess) {
    delete c;
    return hdof_set_error(HDOF_ERR_OOM, "hipMalloc(flags): %s", hipGetErrorString(e));
  }
  e = hipMalloc(&c->d_counters, 6 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    hipFree(c->d_flags);
    delete c;
    return hdof_set_error(HDOF_ERR_OOM, "hipMalloc(counters): %s", hipGetErrorString(e));
  }
  e = hipMemset(c->d_counters, 0, 6 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->d_flags, 0, sizeof(int));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  // the fork and join events order work between the context's two streams
  // on one device only: a device-scope release suffices, without the
  // system-scope fence (cache writeback for the host) an event completes
  // with by default
  const unsigned evf = hipEventDisableTiming | hipEventDisableSystemFence;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, evf);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, evf);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork2, evf);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (c->ev_join) hipEventDestroy(c->ev_join);
    if (c->ev_fork2) hipEventDestroy(c->ev_fork2);
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->side) hipStreamDestroy(c->side);
    hipFree(c->d_counters);
    hipFree(c->d_flags);
    delete c;
    return hdof_set_error(HDOF_ERR_HIP, "init: %s", hipGetErrorString(e));
  }
  // the no-alloc post-filter's scratch address on this device (current now)
  const hdof_status ns = postfilter_noalloc_init(device, &c->noalloc_scratch);
  if (ns != HDOF_OK) {
    hdof_destroy(c);
    return ns;
  }
  *out = c;
  return HDOF_OK;
}

extern "C" void hdof_destroy(hdof_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  Buf* all[] = {&ctx->queue, &ctx->ray_col, &ctx->ray_z, &ctx->work_counter, &ctx->mask_tile,
                &ctx->mask_tile_dil, &ctx->mask_xpref, &ctx->mask_rowsum, &ctx->mask_ybase, &ctx->mask_auto,
                &ctx->pp_pack, &ctx->pp_tile, &ctx->pp_rad, &ctx->pp_taps, &ctx->hist_m1,
                &ctx->hist_m2, &ctx->hist_flags, &ctx->hist_z, &ctx->rep_m1, &ctx->rep_m2,
                &ctx->rep_flags, &ctx->rep_z, &ctx->f_depth, &ctx->f_normal, &ctx->f_albedo, &ctx->f_color,
                &ctx->f_triid, &ctx->f_spp, &ctx->f_offsets, &ctx->f_total, &ctx->f_cn, &ctx->f_cf,
                &ctx->f_h, &ctx->f_m1, &ctx->f_m2, &ctx->f_pp, &ctx->f_spec, &ctx->f_pps, &ctx->rec_hist[0], &ctx->rec_hist[1],
                &ctx->rec_valid[0], &ctx->rec_valid[1], &ctx->rec_farpos, &ctx->sp_levels, &ctx->sp_taps,
                &ctx->sp_cn, &ctx->sp_cf, &ctx->sp_coc};
  for (Buf* b : all) buf_free(*b);
  for (hipEvent_t e : ctx->prof_events) hipEventDestroy(e);
  buf_free(ctx->ppb_args);
  buf_free(ctx->ppb_partial);
  buf_free(ctx->b_arena);
  buf_free(ctx->b_views);
  buf_free(ctx->b_totals);
  if (ctx->b_views_host) hipHostFree(ctx->b_views_host);
  if (ctx->b_views_done) hipEventDestroy(ctx->b_views_done);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  if (ctx->ev_fork2) hipEventDestroy(ctx->ev_fork2);
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->side) hipStreamDestroy(ctx->side);
  if (ctx->d_flags) hipFree(ctx->d_flags);
  if (ctx->d_counters) hipFree(ctx->d_counters);
  delete ctx;
}

extern "C" hdof_status hdof_sync(hdof_ctx* ctx, hdof_stream stream) {
  TRY(check_ctx(ctx));
  HDOF_HIP(hipStreamSynchronize((hipStream_t)stream));
  int f = 0;
  HDOF_HIP(hipMemcpy(&f, ctx->d_flags, sizeof(int), hipMemcpyDeviceToHost));
  if (f) {
    HDOF_HIP(hipMemset(ctx->d_flags, 0, sizeof(int)));
    HDOF_HIP(hipDeviceSynchronize());
    if (f & HDOF_FLAG_STACK_OVERFLOW)
      return hdof_set_error(HDOF_ERR_CAPACITY, "traversal stack overflow (tree deeper than %d)",
                            HDOF_LDS_STACK + HDOF_SPILL_STACK);
    return hdof_set_error(HDOF_ERR_CAPACITY, "ray total exceeded the queue capacity (spp above spp_max)");
  }
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// scene
// ---------------------------------------------------------------------------
extern "C" hdof_status hdof_build_bvh(hdof_ctx* ctx, const float* d_verts, const float* d_albedo,
                                      int32_t n_tris, hdof_scene** out, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(out, "out is NULL");
  *out = nullptr;
  REQUIRE(d_verts && d_albedo, "vertex and albedo pointers must be non-NULL");
  REQUIRE(n_tris >= 1 && n_tris <= (1 << 26), "n_tris %d outside [1, 2^26]", n_tris);
  hdof_scene* sc = new hdof_scene();
  sc->ctx = ctx;
  sc->n_tris = n_tris;
  hdof_status s = launch_bvh_build(ctx, d_verts, d_albedo, n_tris, sc, (hipStream_t)stream);
  if (s != HDOF_OK) {
    hdof_scene_destroy(sc);
    return s;
  }
  *out = sc;
  return HDOF_OK;
}

extern "C" void hdof_scene_destroy(hdof_scene* sc) {
  if (!sc) return;
  hipSetDevice(sc->ctx->device);
  hipDeviceSynchronize();
  if (sc->nodes) hipFree(sc->nodes);
  if (sc->tris) hipFree(sc->tris);
  if (sc->albedo) hipFree(sc->albedo);
  if (sc->spec) hipFree(sc->spec);
  if (sc->depth_out) hipFree(sc->depth_out);
  delete sc;
}

extern "C" hdof_status hdof_scene_set_specular(hdof_scene* sc, const float* d_spec, hdof_stream stream) {
  REQUIRE(sc, "scene is NULL");
  TRY(check_ctx(sc->ctx));
  if (!d_spec) {
    if (sc->spec) {
      HDOF_HIP(hipDeviceSynchronize());  // frames in flight may still read the table
      HDOF_HIP(hipFree(sc->spec));
      sc->bytes -= sizeof(float) * 2 * (int64_t)sc->n_tris;
      sc->spec = nullptr;
    }
    return HDOF_OK;
  }
  if (!sc->spec) {
    HDOF_HIP(hipMalloc(&sc->spec, sizeof(float) * 2 * (size_t)sc->n_tris));
    sc->bytes += sizeof(float) * 2 * (int64_t)sc->n_tris;
  }
  HDOF_HIP(hipMemcpyAsync(sc->spec, d_spec, sizeof(float) * 2 * (size_t)sc->n_tris, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
  return HDOF_OK;
}

extern "C" hdof_status hdof_scene_stats(hdof_scene* sc, hdof_scene_info* out) {
  REQUIRE(sc && out, "scene and out must be non-NULL");
  TRY(check_ctx(sc->ctx));
  HDOF_HIP(hipDeviceSynchronize());
  int d = 0;
  HDOF_HIP(hipMemcpy(&d, sc->depth_out, sizeof(int), hipMemcpyDeviceToHost));
  out->n_tris = sc->n_tris;
  out->n_nodes = sc->n_nodes;
  out->max_depth = d;
  out->leaf_size = 0;
  out->device_bytes = sc->bytes;
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// stages
// ---------------------------------------------------------------------------
static hdof_status check_gb(const hdof_gbuffer_bufs* b) {
  REQUIRE(b && b->depth && b->normal && b->albedo && b->color && b->tri_id,
          "all G-buffer planes must be non-NULL");
  return HDOF_OK;
}

static hdof_status check_rt(const hdof_rt_bufs* b) {
  REQUIRE(b->c_near && b->c_far && b->hit_ratio && b->lum_m1 && b->lum_m2,
          "all ray-trace result planes must be non-NULL");
  return HDOF_OK;
}

static hdof_status check_capacity(const hdof_camera* cam, int spp_max) {
  REQUIRE((int64_t)cam->width * cam->height * spp_max < ((int64_t)1 << 31),
          "width * height * spp_max must stay below 2^31");
  return HDOF_OK;
}

extern "C" hdof_status hdof_gbuffer(hdof_ctx* ctx, const hdof_scene* scene, const hdof_camera* cam,
                                    const hdof_lens* lens, const hdof_light* light,
                                    hdof_gbuffer_bufs out, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(scene, "scene is NULL");
  TRY(check_camera(cam, "current"));
  TRY(check_lens(lens));
  TRY(check_light(light));
  TRY(check_gb(&out));
  CamK k = make_camk(cam);
  return launch_gbuffer(ctx, scene, k, make_lensk(lens, k), make_lightk(light), out, (hipStream_t)stream);
}

extern "C" hdof_status hdof_ray_mask(hdof_ctx* ctx, const hdof_gbuffer_bufs* in, const hdof_camera* cam,
                                     const hdof_camera* prev, const hdof_lens* lens,
                                     const hdof_mask_params* params, uint8_t* d_spp, int32_t* d_offsets,
                                     int32_t* d_total, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(in && in->depth && in->normal, "depth and normal planes must be non-NULL");
  TRY(check_camera(cam, "current"));
  if (prev) TRY(check_camera(prev, "previous"));
  TRY(check_lens(lens));
  TRY(check_mask(params));
  TRY(check_capacity(cam, params->spp_max));
  REQUIRE(d_spp && d_offsets && d_total, "spp, offsets and total must be non-NULL");
  CamK k = make_camk(cam);
  CamK pk;
  if (prev) pk = make_camk(prev);
  const LensK l = make_lensk(lens, k);
  return launch_mask(ctx, in->depth, in->normal, k, prev ? &pk : nullptr, *params, d_spp, d_offsets, d_total,
                     (hipStream_t)stream, nullptr, 0, nullptr, &l);
}

extern "C" hdof_status hdof_trace_thin_lens(hdof_ctx* ctx, const hdof_scene* scene, const hdof_camera* cam,
                                            const hdof_lens* lens, const hdof_light* light, int32_t spp_max,
                                            const uint8_t* d_spp, const int32_t* d_offsets,
                                            const int32_t* d_total, uint32_t seed, uint32_t frame,
                                            uint32_t view, hdof_rt_bufs out, int32_t* d_ray_tri_id,
                                            float* d_ray_depth, float* d_far_pos, float* d_coc_nf,
                                            hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(scene, "scene is NULL");
  TRY(check_camera(cam, "current"));
  TRY(check_lens(lens));
  TRY(check_light(light));
  REQUIRE(spp_max >= 1 && spp_max <= 255, "spp_max must be in [1, 255]");
  TRY(check_capacity(cam, spp_max));
  REQUIRE(d_spp && d_offsets && d_total, "spp, offsets and total must be non-NULL");
  TRY(check_rt(&out));
  CamK k = make_camk(cam);
  return launch_trace(ctx, scene, k, make_lensk(lens, k), make_lightk(light), spp_max, d_spp, d_offsets,
                      d_total, seed, frame, view, out, d_ray_tri_id, d_ray_depth, d_far_pos,
                      (hipStream_t)stream, nullptr, false, d_coc_nf);
}

extern "C" hdof_status hdof_variance_update(hdof_ctx* ctx, const hdof_camera* cam,
                                            const hdof_mask_params* params, const uint8_t* d_spp,
                                            const float* d_depth, const float* d_lum_m1,
                                            const float* d_lum_m2, hdof_stream stream) {
  TRY(check_ctx(ctx));
  TRY(check_camera(cam, "current"));
  TRY(check_mask(params));
  REQUIRE(d_spp && d_depth && d_lum_m1 && d_lum_m2, "spp, depth and moment planes must be non-NULL");
  CamK k = make_camk(cam);
  return launch_var_update(ctx, k, params->var_alpha, d_spp, d_depth, d_lum_m1, d_lum_m2, (hipStream_t)stream);
}

extern "C" hdof_status hdof_history_load(hdof_ctx* ctx, int32_t width, int32_t height, const float* d_lum_m1,
                                         const float* d_lum_m2, const uint8_t* d_flags,
                                         const float* d_depth, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(width > 0 && height > 0 && width <= 16384 && height <= 16384, "history size out of range");
  REQUIRE(d_lum_m1 && d_lum_m2 && d_flags && d_depth, "history planes must be non-NULL");
  size_t N = (size_t)width * height;
  TRY(hdof_ensure(ctx->hist_m1, 4 * N));
  TRY(hdof_ensure(ctx->hist_m2, 4 * N));
  TRY(hdof_ensure(ctx->hist_flags, N));
  TRY(hdof_ensure(ctx->hist_z, 4 * N));
  hipStream_t st = (hipStream_t)stream;
  HDOF_HIP(hipMemcpyAsync(ctx->hist_m1.p, d_lum_m1, 4 * N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(ctx->hist_m2.p, d_lum_m2, 4 * N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(ctx->hist_flags.p, d_flags, N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(ctx->hist_z.p, d_depth, 4 * N, hipMemcpyDeviceToDevice, st));
  ctx->hist_w = width;
  ctx->hist_h = height;
  ctx->hist_any = true;
  return HDOF_OK;
}

extern "C" hdof_status hdof_history_save(hdof_ctx* ctx, float* d_lum_m1, float* d_lum_m2, uint8_t* d_flags,
                                         float* d_depth, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(ctx->hist_any, "the context holds no history");
  REQUIRE(d_lum_m1 && d_lum_m2 && d_flags && d_depth, "history planes must be non-NULL");
  size_t N = (size_t)ctx->hist_w * ctx->hist_h;
  hipStream_t st = (hipStream_t)stream;
  HDOF_HIP(hipMemcpyAsync(d_lum_m1, ctx->hist_m1.p, 4 * N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(d_lum_m2, ctx->hist_m2.p, 4 * N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(d_flags, ctx->hist_flags.p, N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(d_depth, ctx->hist_z.p, 4 * N, hipMemcpyDeviceToDevice, st));
  return HDOF_OK;
}

extern "C" hdof_status hdof_history_reset(hdof_ctx* ctx) {
  TRY(check_ctx(ctx));
  HDOF_HIP(hipDeviceSynchronize());
  ctx->hist_any = false;
  ctx->hist_w = ctx->hist_h = 0;
  ctx->rep_valid = false;
  return HDOF_OK;
}

extern "C" hdof_status hdof_rt_reconstruct(hdof_ctx* ctx, const hdof_camera* cam, const hdof_camera* prev,
                                           const float* d_depth, const uint8_t* d_spp, const float* d_far_pos,
                                           hdof_rt_bufs rt, const hdof_recon_params* params, hdof_stream stream) {
  TRY(check_ctx(ctx));
  TRY(check_camera(cam, "current"));
  if (prev) TRY(check_camera(prev, "previous"));
  REQUIRE(d_depth && d_spp && d_far_pos, "depth, spp and far_pos must be non-NULL");
  REQUIRE(rt.c_near && rt.c_far && rt.hit_ratio, "rt c_near, c_far and hit_ratio must be non-NULL");
  TRY(check_recon(params));
  CamK k = make_camk(cam), pk;
  if (prev) pk = make_camk(prev);
  return launch_recon(ctx, k, prev ? &pk : nullptr, d_depth, d_spp, d_far_pos, rt, params->alpha,
                      (hipStream_t)stream);
}

extern "C" hdof_status hdof_recon_history_load(hdof_ctx* ctx, int32_t width, int32_t height, const float* d_planes,
                                               const uint8_t* d_valid, const float* d_depth, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(width > 0 && height > 0 && width <= 16384 && height <= 16384, "history size out of range");
  REQUIRE(d_planes && d_valid && d_depth, "history planes must be non-NULL");
  const size_t N = (size_t)width * height;
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < 2; ++i) {
    TRY(hdof_ensure(ctx->rec_hist[i], sizeof(float) * 9 * N));
    TRY(hdof_ensure(ctx->rec_valid[i], N));
  }
  const int cur = ctx->rec_cur;
  HDOF_HIP(hipMemcpyAsync(ctx->rec_hist[cur].p, d_planes, sizeof(float) * 8 * N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync((float*)ctx->rec_hist[cur].p + 8 * N, d_depth, sizeof(float) * N, hipMemcpyDeviceToDevice,
                          st));
  HDOF_HIP(hipMemcpyAsync(ctx->rec_valid[cur].p, d_valid, N, hipMemcpyDeviceToDevice, st));
  ctx->rec_w = width;
  ctx->rec_h = height;
  ctx->rec_any = true;
  return HDOF_OK;
}

extern "C" hdof_status hdof_recon_history_save(hdof_ctx* ctx, float* d_planes, uint8_t* d_valid, float* d_depth,
                                               hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(ctx->rec_any, "the context holds no reconstruction history");
  REQUIRE(d_planes && d_valid && d_depth, "history planes must be non-NULL");
  const size_t N = (size_t)ctx->rec_w * ctx->rec_h;
  const int cur = ctx->rec_cur;
  hipStream_t st = (hipStream_t)stream;
  HDOF_HIP(hipMemcpyAsync(d_planes, ctx->rec_hist[cur].p, sizeof(float) * 8 * N, hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(d_depth, (const float*)ctx->rec_hist[cur].p + 8 * N, sizeof(float) * N,
                          hipMemcpyDeviceToDevice, st));
  HDOF_HIP(hipMemcpyAsync(d_valid, ctx->rec_valid[cur].p, N, hipMemcpyDeviceToDevice, st));
  return HDOF_OK;
}

extern "C" hdof_status hdof_recon_history_reset(hdof_ctx* ctx) {
  TRY(check_ctx(ctx));
  HDOF_HIP(hipDeviceSynchronize());
  ctx->rec_any = false;
  ctx->rec_w = ctx->rec_h = 0;
  return HDOF_OK;
}

extern "C" hdof_status hdof_rt_spatial(hdof_ctx* ctx, int32_t width, int32_t height, const uint8_t* d_spp,
                                       hdof_rt_bufs rt, const float* d_hit_acc, const float* d_coc_nf,
                                       const float* d_variance, const hdof_spatial_params* params,
                                       float* d_c_near_out, float* d_c_far_out, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(width > 0 && height > 0 && width <= 16384 && height <= 16384, "image size out of range");
  REQUIRE(d_spp && d_coc_nf, "spp and coc_nf must be non-NULL");
  REQUIRE(rt.c_near && rt.c_far && rt.hit_ratio, "rt c_near, c_far and hit_ratio must be non-NULL");
  REQUIRE(d_c_near_out && d_c_far_out, "outputs must be non-NULL");
  REQUIRE(d_c_near_out != rt.c_near && d_c_near_out != rt.c_far && d_c_far_out != rt.c_near &&
              d_c_far_out != rt.c_far && d_c_near_out != d_c_far_out,
          "outputs must not alias the input colours or each other");
  TRY(check_spatial(params));
  return launch_spatial(ctx, width, height, d_spp, rt, d_hit_acc, d_coc_nf, d_variance, false, *params,
                        d_c_near_out, d_c_far_out, (hipStream_t)stream);
}

extern "C" hdof_status hdof_postfilter(hdof_ctx* ctx, const float* d_color, const float* d_depth,
                                       const hdof_camera* cam, const hdof_lens* lens,
                                       const hdof_pp_params* params, float* d_out, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(d_color && d_depth && d_out, "color, depth and out must be non-NULL");
  TRY(check_camera(cam, "current"));
  TRY(check_lens(lens));
  TRY(check_pp(params));
  CamK k = make_camk(cam);
  return launch_postfilter(ctx, d_color, d_depth, k, make_lensk(lens, k), *params, d_out, (hipStream_t)stream);
}

extern "C" hdof_status hdof_postfilter_noalloc(hdof_ctx* ctx, const float* d_color, const float* d_depth,
                                               const hdof_camera* cam, const hdof_lens* lens,
                                               const hdof_pp_params* params, float* d_out, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(d_color && d_depth && d_out, "color, depth and out must be non-NULL");
  TRY(check_camera(cam, "current"));
  TRY(check_lens(lens));
  TRY(check_pp(params));
  CamK k = make_camk(cam);
  return launch_postfilter_noalloc(ctx, d_color, d_depth, k, make_lensk(lens, k), *params, d_out,
                                   (hipStream_t)stream);
}

extern "C" hdof_status hdof_postfilter_specular(hdof_ctx* ctx, const float* d_color, const float* d_depth,
                                                const float* d_spec, const uint8_t* d_spp, const hdof_camera* cam,
                                                const hdof_lens* lens, const hdof_pp_params* params, float* d_out,
                                                float* d_spec_out, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(d_color && d_depth && d_out && d_spec && d_spec_out, "color, depth, out, spec and spec_out must be non-NULL");
  REQUIRE(d_spec_out != d_spec, "spec_out must not alias spec");
  TRY(check_camera(cam, "current"));
  TRY(check_lens(lens));
  TRY(check_pp(params));
  CamK k = make_camk(cam);
  const LensK l = make_lensk(lens, k);
  hipStream_t st = (hipStream_t)stream;
  TRY(launch_postfilter(ctx, d_color, d_depth, k, l, *params, d_out, st));
  return launch_pp_spec(ctx, d_spec, d_spp, k, l, *params, d_spec_out, st);
}

extern "C" hdof_status hdof_composite(hdof_ctx* ctx, const float* d_color, const float* d_pp,
                                      const float* d_depth, const uint8_t* d_spp, hdof_rt_bufs rt,
                                      const hdof_camera* cam, const hdof_lens* lens,
                                      const hdof_composite_params* params, const float* d_pp_spec, float* d_out,
                                      hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(d_color && d_pp && d_depth && d_spp && d_out, "color, pp, depth, spp and out must be non-NULL");
  TRY(check_rt(&rt));
  TRY(check_camera(cam, "current"));
  TRY(check_lens(lens));
  TRY(check_comp(params));
  CamK k = make_camk(cam);
  return launch_composite(ctx, d_color, d_pp, d_depth, d_spp, rt, k, make_lensk(lens, k), *params, d_out,
                          (hipStream_t)stream, d_pp_spec);
}

template <typename T>
static hdof_status pick_buf(T* user, Buf& scratch, size_t bytes, T** out) {
  if (user) {
    *out = user;
    return HDOF_OK;
  }
  TRY(hdof_ensure(scratch, bytes));
  *out = (T*)scratch.p;
  return HDOF_OK;
}

extern "C" hdof_status hdof_frame(hdof_ctx* ctx, const hdof_scene* scene, const hdof_camera* cam,
                                  const hdof_camera* prev, const hdof_lens* lens, const hdof_light* light,
                                  const hdof_frame_params* params, uint32_t seed, uint32_t frame,
                                  uint32_t view, float* d_out, const hdof_frame_bufs* keep,
                                  hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(scene, "scene is NULL");
  TRY(check_camera(cam, "current"));
  if (prev) TRY(check_camera(prev, "previous"));
  TRY(check_lens(lens));
  TRY(check_light(light));
  REQUIRE(params, "frame params are NULL");
  TRY(check_mask(&params->mask));
  TRY(check_pp(&params->pp));
  TRY(check_comp(&params->comp));
  TRY(check_recon(&params->recon));
  TRY(check_spatial(&params->spatial));
  TRY(check_capacity(cam, params->mask.spp_max));
  REQUIRE(d_out, "out is NULL");
  // A captured frame replays with the buffers fixed when it was captured,
  // while the variance history's ping-pong and the temporal
  // reconstruction's history index advance on the host: a captured frame
  // may neither read a history (prev, reconstruction) nor advance one.
  hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
  HDOF_HIP(hipStreamIsCapturing((hipStream_t)stream, &cap_status));
  const bool capturing = cap_status != hipStreamCaptureStatusNone;
  if (capturing && (prev || params->recon.enable || params->spatial.enable))
    return hdof_set_error(HDOF_ERR_UNSUPPORTED,
                          "a frame under stream capture takes no previous camera and no reconstruction "
                          "(their histories advance on the host)");
  hdof_frame_bufs z;
  memset(&z, 0, sizeof z);
  const hdof_frame_bufs& u = keep ? *keep : z;
  const size_t N = (size_t)cam->width * cam->height;
  hdof_gbuffer_bufs gb;
  hdof_rt_bufs rt;
  uint8_t* spp;
  int32_t *offs, *total;
  float* pp;
  TRY(pick_buf(u.gb.depth, ctx->f_depth, 4 * N, &gb.depth));
  TRY(pick_buf(u.gb.normal, ctx->f_normal, 12 * N, &gb.normal));
  TRY(pick_buf(u.gb.albedo, ctx->f_albedo, 12 * N, &gb.albedo));
  TRY(pick_buf(u.gb.color, ctx->f_color, 12 * N, &gb.color));
  TRY(pick_buf(u.gb.tri_id, ctx->f_triid, 4 * N, &gb.tri_id));
  // specular bokeh: the G-buffer's specular luminance and its post-filtered
  // value at the traced pixels (the composite's rule reads no other)
  const bool spec_on = scene->spec && params->comp.spec_y > 0.0f;
  float* pps = nullptr;
  gb.spec = u.gb.spec;
  if (spec_on) {
    TRY(pick_buf(u.gb.spec, ctx->f_spec, 4 * N, &gb.spec));
    TRY(hdof_ensure(ctx->f_pps, 4 * N));
    pps = (float*)ctx->f_pps.p;
  }
  TRY(pick_buf(u.spp, ctx->f_spp, N, &spp));
  TRY(pick_buf(u.offsets, ctx->f_offsets, 4 * N, &offs));
  TRY(pick_buf(u.total, ctx->f_total, 4, &total));
  TRY(pick_buf(u.rt.c_near, ctx->f_cn, 12 * N, &rt.c_near));
  TRY(pick_buf(u.rt.c_far, ctx->f_cf, 12 * N, &rt.c_far));
  TRY(pick_buf(u.rt.hit_ratio, ctx->f_h, 4 * N, &rt.hit_ratio));
  TRY(pick_buf(u.rt.lum_m1, ctx->f_m1, 4 * N, &rt.lum_m1));
  TRY(pick_buf(u.rt.lum_m2, ctx->f_m2, 4 * N, &rt.lum_m2));
  // 16-pixel post-filter tiles: the G-buffer writes the packed texels and
  // tile radii, the gather applies the composite (the filtered colour is
  // stored only when the caller keeps it)
  const bool fused = params->pp.tile == 16;
  // overlapped frame: the gather on the context's second stream beside the
  // mask, trace and reconstruction, the composite after both
  const bool ovl = ctx->tune.overlap != 0;
  if (fused && !ovl) {
    pp = u.pp;
  } else {
    TRY(pick_buf(u.pp, ctx->f_pp, 12 * N, &pp));
  }
  float4* pack = nullptr;
  float* tile_r = nullptr;
  if (fused) {
    const size_t ntile = (size_t)((cam->width + 15) / 16) * ((cam->height + 15) / 16);
    TRY(hdof_ensure(ctx->pp_pack, sizeof(float4) * N));
    TRY(hdof_ensure(ctx->pp_tile, sizeof(float) * ntile));
    pack = (float4*)ctx->pp_pack.p;
    tile_r = (float*)ctx->pp_tile.p;
  }
  hipStream_t st = (hipStream_t)stream;
  CamK k = make_camk(cam);
  LensK l = make_lensk(lens, k);
  LightK li = make_lightk(light);
  CamK pk;
  if (prev) pk = make_camk(prev);
  // reserve every scratch buffer before the first launch so no reallocation
  // (and its device synchronisation) happens between profiled stages
  const size_t cap = N * (size_t)params->mask.spp_max;
  TRY(hdof_ensure(ctx->queue, sizeof(int) * cap));
  TRY(hdof_ensure(ctx->ray_col, sizeof(float) * 3 * cap));
  TRY(hdof_ensure(ctx->ray_z, sizeof(float) * cap));
  // spatial reconstruction: the trace (and the temporal stage) work on
  // scratch colours that the spatial gather reads, writing the frame's
  float* coc_nf = nullptr;
  hdof_rt_bufs rt_tr = rt;
  const bool spatial = params->spatial.enable;
  if (spatial) {
    TRY(hdof_ensure(ctx->sp_cn, sizeof(float) * 3 * N));
    TRY(hdof_ensure(ctx->sp_cf, sizeof(float) * 3 * N));
    TRY(hdof_ensure(ctx->sp_coc, sizeof(float) * 2 * N));
    TRY(spatial_reserve(ctx, cam->width, cam->height));
    rt_tr.c_near = (float*)ctx->sp_cn.p;
    rt_tr.c_far = (float*)ctx->sp_cf.p;
    coc_nf = (float*)ctx->sp_coc.p;
  }
  float* far_pos = nullptr;
  if (params->recon.enable) {
    TRY(hdof_ensure(ctx->rec_farpos, sizeof(float) * 4 * N));
    far_pos = (float*)ctx->rec_farpos.p;
    for (int i = 0; i < 2; ++i) {
      TRY(hdof_ensure(ctx->rec_hist[i], sizeof(float) * 9 * N));
      TRY(hdof_ensure(ctx->rec_valid[i], N));
    }
  }
  TRY(hdof_ensure(ctx->work_counter, sizeof(int) * 8 * HDOF_SEG_STRIDE));
  // the tap table is written on the frame's stream before the fork, so the
  // gathers of both streams read it complete
  if (ovl) TRY(postfilter_reserve(ctx, k, l, params->pp, st));
  ctx->prof_in_frame = true;
  hdof_prof_mark(ctx, 0, st);
  // overlapped frames, uncaptured and unprofiled: the fork event is the
  // G-buffer's own completion and, with 16-pixel tiles, the join event the
  // gather's, so no marker packet follows either kernel on its stream
  // (0.3827 against 0.3885 ms per 1080p frame; events without the
  // system-scope fence: 0.3818)
  const bool ext_ev = ovl && !capturing && !ctx->prof_on;
  hdof_status s = launch_gbuffer(ctx, scene, k, l, li, gb, st, pack, tile_r, ext_ev ? ctx->ev_fork : nullptr);
  hdof_prof_mark(ctx, 1, st);
  bool forked = false;
  if (s == HDOF_OK && ovl) {
    hipError_t e = ext_ev ? hipSuccess : hipEventRecord(ctx->ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0);
    if (e != hipSuccess) {
      s = hdof_set_error(HDOF_ERR_HIP, "overlapped frame fork: %s", hipGetErrorString(e));
    } else {
      forked = true;
      // mark 8 on the side stream (inside), then the gather's end; with
      // 16-pixel tiles its epilogue writes every pixel's output by the
      // untraced pixels' rule, and the composite after the join rewrites
      // only the traced pixels
      hdof_rt_bufs none;
      memset(&none, 0, sizeof none);
      const PostFuse pu{nullptr, none, params->comp, d_out, nullptr, true, ext_ev ? ctx->ev_join : nullptr};
      s = launch_postfilter(ctx, gb.color, gb.depth, k, l, params->pp, pp, ctx->side, fused, fused ? &pu : nullptr);
      hdof_prof_mark(ctx, HDOF_PROF_GATHER_END, ctx->side);
      // a failed gather launch completes no event: the join is then a marker
      e = ext_ev && fused && s == HDOF_OK ? hipSuccess : hipEventRecord(ctx->ev_join, ctx->side);
      if (e != hipSuccess) {
        forked = false;
        if (s == HDOF_OK) s = hdof_set_error(HDOF_ERR_HIP, "overlapped frame join: %s", hipGetErrorString(e));
      }
    }
  }
  // the mask's final pass also fills the ray queue (queue stage empty)
  if (s == HDOF_OK)
    s = launch_mask(ctx, gb.depth, gb.normal, k, prev ? &pk : nullptr, params->mask, spp, offs, total, st,
                    (int*)ctx->queue.p, (long)cap, (int*)ctx->work_counter.p, &l, !capturing);
  // the trace's per-pixel reduction also updates the variance history
  // (variance stage empty); a captured frame writes no history at all: its
  // replays would write planes fixed at capture, which by then may hold the
  // history of a later eager frame
  VarFuse vf{};
  const VarFuse* vfp = nullptr;
  if (s == HDOF_OK && !capturing) {
    s = var_update_prepare(ctx, k, params->mask.var_alpha, gb.depth, &vf, true);
    vfp = &vf;
  }
  // only the composite reads the trace planes, and only at traced pixels,
  // unless the caller keeps them or a reconstruction stage reads them
  vf.sparse_rt = !u.rt.c_near && !u.rt.c_far && !u.rt.hit_ratio && !u.rt.lum_m1 && !u.rt.lum_m2 &&
                 !params->recon.enable && !spatial;
  if (s == HDOF_OK) {
    // beside the gather the trace keeps blocks in proportion to its rays
    ctx->trace_ray_quantum = ovl ? ctx->tune.overlap_ray_quantum : 0;
    s = launch_trace(ctx, scene, k, l, li, params->mask.spp_max, spp, offs, total, seed, frame, view, rt_tr,
                     nullptr, nullptr, far_pos, st, vfp, true, coc_nf);  // marks 3, 4
    ctx->trace_ray_quantum = 0;
    // the reduction updated the history in the reprojected planes
    if (s == HDOF_OK && !capturing) history_swap(ctx);
  }
  if (params->recon.enable || spatial) hdof_prof_mark(ctx, 6, st);  // else the reconstruction stage is empty
  if (s == HDOF_OK && params->recon.enable)
    s = launch_recon(ctx, k, prev ? &pk : nullptr, gb.depth, spp, far_pos, rt_tr, params->recon.alpha, st);
  // the accumulated hit ratio: plane 3 of the temporal history just written
  if (s == HDOF_OK && spatial)
    s = launch_spatial(ctx, cam->width, cam->height, spp, rt_tr,
                       params->recon.enable ? (const float*)ctx->rec_hist[ctx->rec_cur].p + 3 * N : nullptr, coc_nf,
                       nullptr, true, params->spatial, rt.c_near, rt.c_far, st, true);
  hdof_prof_mark(ctx, 7, st);
  if (ovl) {
    // 16-pixel tiles: the specular gather reads the G-buffer's packed texels
    // and runs before the join; other tiles: the side stream's pack
    if (s == HDOF_OK && spec_on && fused) s = launch_pp_spec(ctx, gb.spec, spp, k, l, params->pp, pps, st);
    if (forked) {
      const hipError_t e = hipStreamWaitEvent(st, ctx->ev_join, 0);
      if (e != hipSuccess && s == HDOF_OK)
        s = hdof_set_error(HDOF_ERR_HIP, "overlapped frame join: %s", hipGetErrorString(e));
    }
    if (s == HDOF_OK && spec_on && !fused) s = launch_pp_spec(ctx, gb.spec, spp, k, l, params->pp, pps, st);
    hdof_prof_mark(ctx, 9, st);
    if (s == HDOF_OK)
      s = launch_composite(ctx, gb.color, pp, gb.depth, spp, rt, k, l, params->comp, d_out, st, pps, fused);
  } else if (fused) {
    // the G-buffer wrote the packed texels and tile radii the specular gather reads
    if (s == HDOF_OK && spec_on) s = launch_pp_spec(ctx, gb.spec, spp, k, l, params->pp, pps, st);
    const PostFuse pf{spp, rt, params->comp, d_out, pps, false, nullptr};
    if (s == HDOF_OK) s = launch_postfilter(ctx, gb.color, gb.depth, k, l, params->pp, pp, st, true, &pf);  // mark 8
  } else {
    if (s == HDOF_OK) s = launch_postfilter(ctx, gb.color, gb.depth, k, l, params->pp, pp, st);  // mark 8
    if (s == HDOF_OK && spec_on) s = launch_pp_spec(ctx, gb.spec, spp, k, l, params->pp, pps, st);
    hdof_prof_mark(ctx, 9, st);
    if (s == HDOF_OK)
      s = launch_composite(ctx, gb.color, pp, gb.depth, spp, rt, k, l, params->comp, d_out, st, pps);
  }
  hdof_prof_mark(ctx, 10, st);
  ctx->prof_in_frame = false;
  if (s == HDOF_OK && ctx->prof_on) ctx->prof_frames++;
  return s;
}

// ---------------------------------------------------------------------------
// stage profiling
// ---------------------------------------------------------------------------
void hdof_prof_mark(hdof_ctx* ctx, int i, hipStream_t st) {
  if (!ctx->prof_on || !ctx->prof_in_frame) return;
  const size_t base = (size_t)ctx->prof_frames * HDOF_PROF_SLOTS, idx = base + i;
  while (ctx->prof_events.size() < base + HDOF_PROF_SLOTS) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    ctx->prof_events.push_back(e);
  }
  if (ctx->prof_set.size() < base + HDOF_PROF_SLOTS) ctx->prof_set.resize(base + HDOF_PROF_SLOTS, 0);
  if (i == 0) std::fill(ctx->prof_set.begin() + base, ctx->prof_set.begin() + base + HDOF_PROF_SLOTS, 0);
  if (hipEventRecord(ctx->prof_events[idx], st) == hipSuccess) ctx->prof_set[idx] = 1;
}

extern "C" hdof_status hdof_profile_begin(hdof_ctx* ctx) {
  TRY(check_ctx(ctx));
  ctx->prof_on = true;
  ctx->prof_frames = 0;
  return HDOF_OK;
}

extern "C" hdof_status hdof_profile_end(hdof_ctx* ctx, float* ms_out, int32_t* n_frames) {
  TRY(check_ctx(ctx));
  REQUIRE(ms_out, "ms_out is NULL");
  HDOF_HIP(hipDeviceSynchronize());
  const int S = HDOF_PROFILE_STAGES;
  for (int i = 0; i < S; ++i) ms_out[i] = 0.0f;
  // stage i runs from mark i to the next recorded mark; a stage whose
  // start mark was not recorded (it had no work) counts 0.  An overlapped
  // gather (its end recorded) runs from its mark to its end, and the
  // stage before it on the frame's stream ends at the composite's mark.
  const int G = 8;  // the post-filter gather's stage
  for (int f = 0; f < ctx->prof_frames; ++f) {
    const size_t base = (size_t)f * HDOF_PROF_SLOTS;
    const bool ovl = ctx->prof_set[base + HDOF_PROF_GATHER_END] != 0;
    for (int i = 0; i < S; ++i) {
      if (!ctx->prof_set[base + i]) continue;
      int j = i + 1;
      if (ovl && i == G) {
        j = HDOF_PROF_GATHER_END;
      } else {
        while (j <= S && (!ctx->prof_set[base + j] || (ovl && j == G))) ++j;
        if (j > S) continue;
      }
      float ms = 0.0f;
      HDOF_HIP(hipEventElapsedTime(&ms, ctx->prof_events[base + i], ctx->prof_events[base + j]));
      ms_out[i] += ms;
    }
  }
  if (ctx->prof_frames > 0)
    for (int i = 0; i < S; ++i) ms_out[i] /= (float)ctx->prof_frames;
  if (n_frames) *n_frames = ctx->prof_frames;
  ctx->prof_on = false;
  ctx->prof_frames = 0;
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// traversal work counters
// ---------------------------------------------------------------------------
extern "C" hdof_status hdof_counters_begin(hdof_ctx* ctx) {
  TRY(check_ctx(ctx));
  HDOF_HIP(hipDeviceSynchronize());
  HDOF_HIP(hipMemset(ctx->d_counters, 0, 6 * sizeof(unsigned long long)));
  HDOF_HIP(hipDeviceSynchronize());
  ctx->count_on = true;
  return HDOF_OK;
}

extern "C" hdof_status hdof_counters_end(hdof_ctx* ctx, int64_t* out) {
  TRY(check_ctx(ctx));
  REQUIRE(out, "out is NULL");
  HDOF_HIP(hipDeviceSynchronize());
  unsigned long long c[6];
  HDOF_HIP(hipMemcpy(c, ctx->d_counters, sizeof c, hipMemcpyDeviceToHost));
  for (int i = 0; i < 6; ++i) out[i] = (int64_t)c[i];
  ctx->count_on = false;
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// trace tuning
// ---------------------------------------------------------------------------
extern "C" hdof_status hdof_set_tuning(hdof_ctx* ctx, const hdof_tuning* t) {
  TRY(check_ctx(ctx));
  REQUIRE(t, "tuning is NULL");
  REQUIRE(t->blocks_per_cu >= 1 && t->blocks_per_cu <= 32, "blocks_per_cu must be in [1, 32]");
  REQUIRE(t->refill >= 1 && t->refill <= 64, "refill must be in [1, 64]");
  REQUIRE(t->segments >= 1 && t->segments <= 8, "segments must be in [1, 8]");
  REQUIRE(t->wave >= 0 && t->wave <= 2, "wave must be 0, 1 or 2");
  REQUIRE(t->overlap == 0 || t->overlap == 1, "overlap must be 0 or 1");
  REQUIRE(t->overlap_ray_quantum >= 1, "overlap_ray_quantum must be at least 1");
  ctx->tune = *t;
  return HDOF_OK;
}

extern "C" hdof_status hdof_get_tuning(hdof_ctx* ctx, hdof_tuning* t) {
  TRY(check_ctx(ctx));
  REQUIRE(t, "tuning is NULL");
  *t = ctx->tune;
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------

#ifndef HDOF_BATCH_SPLIT
#define HDOF_BATCH_SPLIT 2  // G-buffer chunks of the overlapped batch (1 or 2)
#endif

struct BatchLayout {
  int n;
  long npx, max_px;
  int max_w, max_h;
  BatchView hv[HDOF_MAX_VIEWS];
  // first 16-pixel post-filter tile of each view in the concatenated tile radii
  long tile_base[HDOF_MAX_VIEWS];
  long ntiles;
  // byte offsets of each concatenated plane set in the arena (o_pack, o_ptile:
  // every view's packed texels and tile radii, for the overlapped batch)
  size_t o_depth, o_normal, o_albedo, o_color, o_tri, o_spp, o_offs, o_cn, o_cf, o_h, o_m1, o_m2, o_pp, o_pack,
      o_ptile, total;
};

static hdof_status batch_check(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                               const hdof_frame_params* params, int32_t n_views, const hdof_view* views,
                               BatchLayout& L) {
  TRY(check_ctx(ctx));
  REQUIRE(scene, "scene is NULL");
  TRY(check_light(light));
  REQUIRE(params, "frame params are NULL");
  TRY(check_mask(&params->mask));
  TRY(check_pp(&params->pp));
  TRY(check_comp(&params->comp));
  TRY(check_recon(&params->recon));
  TRY(check_spatial(&params->spatial));
  if (params->spatial.enable)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "the batched form does not run the spatial reconstruction "
                                                "(call hdof_frame per view)");
  if (scene->spec && params->comp.spec_y > 0.0f)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "the batched form does not apply the specular bokeh rule "
                                                "(call hdof_frame per view)");
  if (params->recon.enable)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "temporal reconstruction needs one history per view: "
                          "not available in the batched form");
  REQUIRE(n_views >= 1 && n_views <= HDOF_MAX_VIEWS, "n_views must be in [1, %d]", HDOF_MAX_VIEWS);
  REQUIRE(views, "views is NULL");
  L.n = n_views;
  L.npx = 0;
  L.max_px = 0;
  L.max_w = L.max_h = 0;
  L.ntiles = 0;
  for (int v = 0; v < n_views; ++v) {
    TRY(check_camera(&views[v].cam, "view"));
    TRY(check_lens(&views[v].lens));
    if (views[v].lens.blades != 0 || views[v].lens.sa != 0.0f)
      return hdof_set_error(HDOF_ERR_UNSUPPORTED, "the batched form takes the disk aperture only (view %d)", v);
    REQUIRE(views[v].d_out, "view %d has no output", v);
    CamK k = make_camk(&views[v].cam);
    L.hv[v] = BatchView{k, make_lensk(&views[v].lens, k), views[v].seed, views[v].frame, views[v].view, (int)L.npx};
    long n = (long)k.W * k.H;
    L.npx += n;
    L.tile_base[v] = L.ntiles;
    L.ntiles += (long)((k.W + 15) / 16) * ((k.H + 15) / 16);
    if (n > L.max_px) L.max_px = n;
    if (k.W > L.max_w) L.max_w = k.W;
    if (k.H > L.max_h) L.max_h = k.H;
  }
  REQUIRE(L.npx * params->mask.spp_max < ((long)1 << 31), "batch pixels * spp_max must stay below 2^31");
  size_t off = 0;
  auto carve = [&](size_t per_px) {
    size_t o = off;
    off += (per_px * (size_t)L.npx + 255) & ~(size_t)255;
    return o;
  };
  L.o_depth = carve(4);
  L.o_normal = carve(12);
  L.o_albedo = carve(12);
  L.o_color = carve(12);
  L.o_tri = carve(4);
  L.o_spp = carve(1);
  L.o_offs = carve(4);
  L.o_cn = carve(12);
  L.o_cf = carve(12);
  L.o_h = carve(4);
  L.o_m1 = carve(4);
  L.o_m2 = carve(4);
  L.o_pp = carve(12);
  L.o_pack = carve(16);
  L.o_ptile = off;
  off += ((size_t)L.ntiles * sizeof(float) + 255) & ~(size_t)255;
  L.total = off;
  return HDOF_OK;
}

// every allocation a batch needs, so that enqueueing it allocates nothing
static hdof_status batch_reserve(hdof_ctx* ctx, const hdof_frame_params* params, const BatchLayout& L) {
  TRY(hdof_ensure(ctx->b_arena, L.total));
  TRY(hdof_ensure(ctx->b_views, batch_view_bytes() * HDOF_MAX_VIEWS));
  TRY(hdof_ensure(ctx->b_totals, sizeof(int) * (3 * HDOF_MAX_VIEWS + 1)));
  TRY(reserve_trace(ctx, (size_t)L.npx * params->mask.spp_max, true));
  // mask scratch for the largest view (tile grids, reprojection planes): the
  // widest and the tallest view bound every grid, the most pixels the planes
  TRY(mask_reserve(ctx, L.max_w, L.max_h, params->mask));
  TRY(mask_reserve_batched(ctx, L.n, L.hv, params->mask));
  TRY(hdof_ensure(ctx->rep_m1, sizeof(float) * L.max_px));
  TRY(hdof_ensure(ctx->rep_m2, sizeof(float) * L.max_px));
  TRY(hdof_ensure(ctx->rep_flags, L.max_px));
  TRY(hdof_ensure(ctx->rep_z, sizeof(float) * L.max_px));
  const int pt = params->pp.tile;
  const size_t ptiles = (size_t)((L.max_w + pt - 1) / pt + 1) * (size_t)((L.max_h + pt - 1) / pt + 1);
  TRY(hdof_ensure(ctx->pp_pack, 16 * (size_t)L.max_px));
  TRY(hdof_ensure(ctx->pp_tile, sizeof(float) * ptiles));
  TRY(hdof_ensure(ctx->pp_rad, sizeof(float) * ptiles));
  TRY(hdof_ensure(ctx->pp_taps, 16 * 256));
  return HDOF_OK;
}

// enqueue one batched frame; `table_host` is pinned memory holding the
// packed view table (copied to the device as the first operation)
static hdof_status batch_enqueue(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                                 const hdof_frame_params* params, const hdof_view* views, const BatchLayout& L,
                                 const void* table_host, hipStream_t st) {
  char* a = (char*)ctx->b_arena.p;
  int32_t* totals = (int32_t*)ctx->b_totals.p;
  int32_t* ebase = totals + HDOF_MAX_VIEWS;
  int32_t* grand = totals + 2 * HDOF_MAX_VIEWS;
  HDOF_HIP(hipMemcpyAsync(ctx->b_views.p, table_host, batch_view_bytes() * L.n, hipMemcpyHostToDevice, st));
  LightK li = make_lightk(light);
  hdof_rt_bufs rt[HDOF_MAX_VIEWS];
  // overlapped batch (16-pixel post-filter tiles, overlap on): one G-buffer
  // launch over all views (packing texels and tile radii), then the views'
  // gathers on the context's second stream beside the masks and the one
  // trace, each writing its untraced pixels' composite; after the join a
  // sparse composite rewrites each view's traced pixels -- the overlapped
  // frame's order over the whole batch
  const bool ovl = ctx->tune.overlap != 0 && params->pp.tile == 16;
  float4* packs = (float4*)(a + L.o_pack);
  float* ptiles = (float*)(a + L.o_ptile);
  for (int v = 0; v < L.n; ++v) {
    const size_t pb = (size_t)L.hv[v].px_base;
    rt[v].c_near = (float*)(a + L.o_cn) + 3 * pb;
    rt[v].c_far = (float*)(a + L.o_cf) + 3 * pb;
    rt[v].hit_ratio = (float*)(a + L.o_h) + pb;
    rt[v].lum_m1 = (float*)(a + L.o_m1) + pb;
    rt[v].lum_m2 = (float*)(a + L.o_m2) + pb;
  }
  hdof_gbuffer_bufs gball;
  gball.depth = (float*)(a + L.o_depth);
  gball.normal = (float*)(a + L.o_normal);
  gball.albedo = (float*)(a + L.o_albedo);
  gball.color = (float*)(a + L.o_color);
  gball.tri_id = (int32_t*)(a + L.o_tri);
  gball.spec = nullptr;
  float* outs[HDOF_MAX_VIEWS];
  for (int v = 0; v < L.n; ++v) outs[v] = views[v].d_out;
  if (ovl) {
    TRY(postfilter_reserve(ctx, L.hv[0].k, L.hv[0].l, params->pp, st));  // tap table, before the fork
    // the views in HDOF_BATCH_SPLIT chunks of about equal pixels, each a
    // G-buffer launch and a fork of its gather, so the next chunk's G-buffer
    // runs beside the gather (a replayed graph pays tens of microseconds per
    // cross-stream dependency: forking per view was slower replayed)
    int cut[3] = {0, L.n, L.n};
    int nch = 1;
    if (HDOF_BATCH_SPLIT > 1 && L.n > 1) {
      int vs = 1;
      while (vs < L.n - 1 && 2 * (long)L.hv[vs].px_base < L.npx) ++vs;
      cut[1] = vs;
      nch = 2;
    }
    const hipEvent_t evs[2] = {ctx->ev_fork, ctx->ev_fork2};
    for (int c = 0; c < nch; ++c) {
      const int v0 = cut[c], n = cut[c + 1] - cut[c];
      const void* vt = (const char*)ctx->b_views.p + batch_view_bytes() * v0;
      TRY(launch_gbuffer_batched(ctx, scene, li, n, L.hv + v0, vt, gball, packs, ptiles + L.tile_base[v0], st));
      HDOF_HIP(hipEventRecord(evs[c], st));
      HDOF_HIP(hipStreamWaitEvent(ctx->side, evs[c], 0));
      TRY(launch_postfilter_batched(ctx, packs, ptiles + L.tile_base[v0], n, L.hv + v0, vt, outs + v0, params->pp,
                                    (float*)(a + L.o_pp), ctx->side));
    }
    HDOF_HIP(hipEventRecord(ctx->ev_join, ctx->side));
  }
  // the masks: one launch per pass over every view with fixed mask tiles,
  // per view with the tile scaled by the view's CoC
  const bool mask1 = params->mask.tile > 0;
  for (int v = 0; v < L.n; ++v) {
    const BatchView& bv = L.hv[v];
    const size_t pb = (size_t)bv.px_base;
    hdof_gbuffer_bufs gb;
    gb.depth = gball.depth + pb;
    gb.normal = gball.normal + 3 * pb;
    gb.albedo = gball.albedo + 3 * pb;
    gb.color = gball.color + 3 * pb;
    gb.tri_id = gball.tri_id + pb;
    gb.spec = nullptr;
    if (!ovl) TRY(launch_gbuffer(ctx, scene, bv.k, bv.l, li, gb, st));
    if (!mask1)
      TRY(launch_mask(ctx, gb.depth, gb.normal, bv.k, nullptr, params->mask, (uint8_t*)(a + L.o_spp) + pb,
                      (int32_t*)(a + L.o_offs) + pb, totals + v, st, nullptr, 0, nullptr, &bv.l, false));
  }
  if (mask1)
    TRY(launch_mask_batched(ctx, gball.depth, gball.normal, L.n, L.hv, ctx->b_views.p, params->mask,
                            (uint8_t*)(a + L.o_spp), (int32_t*)(a + L.o_offs), totals, st));
  TRY(launch_trace_batched(ctx, scene, li, params->mask.spp_max, L.n, L.hv, ctx->b_views.p,
                           (const uint8_t*)(a + L.o_spp), (const int32_t*)(a + L.o_offs), totals, ebase, grand, rt,
                           st));
  if (ovl) {
    HDOF_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
    TRY(launch_composite_traced_batched(ctx, (const float*)(a + L.o_color), (const float*)(a + L.o_pp),
                                        (const float*)(a + L.o_depth), (const uint8_t*)(a + L.o_spp), rt[0], L.n,
                                        L.hv, ctx->b_views.p, outs, params->comp, st));
  }
  for (int v = 0; v < L.n && !ovl; ++v) {
    const BatchView& bv = L.hv[v];
    const size_t pb = (size_t)bv.px_base;
    float* color = (float*)(a + L.o_color) + 3 * pb;
    float* depth = (float*)(a + L.o_depth) + pb;
    float* pp = (float*)(a + L.o_pp) + 3 * pb;
    const uint8_t* spp = (const uint8_t*)(a + L.o_spp) + pb;
    if (params->pp.tile == 16) {  // composite in the gather's epilogue, as in hdof_frame
      const PostFuse pf{spp, rt[v], params->comp, views[v].d_out, nullptr, false, nullptr};
      TRY(launch_postfilter(ctx, color, depth, bv.k, bv.l, params->pp, nullptr, st, false, &pf));
    } else {
      TRY(launch_postfilter(ctx, color, depth, bv.k, bv.l, params->pp, pp, st));
      TRY(launch_composite(ctx, color, pp, depth, spp, rt[v], bv.k, bv.l, params->comp, views[v].d_out, st));
    }
  }
  ctx->rep_valid = false;  // the views' reprojection planes are no frame history
  return HDOF_OK;
}

extern "C" hdof_status hdof_frame_batched(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                                          const hdof_frame_params* params, int32_t n_views,
                                          const hdof_view* views, hdof_stream stream) {
  static thread_local BatchLayout L;
  TRY(batch_check(ctx, scene, light, params, n_views, views, L));
  TRY(batch_reserve(ctx, params, L));
  hipStream_t st = (hipStream_t)stream;
  // pinned staging for the view table: wait until the previous batch's copy
  // has consumed it before overwriting
  const size_t tb = batch_view_bytes() * HDOF_MAX_VIEWS;
  if (!ctx->b_views_host) {
    HDOF_HIP(hipHostMalloc(&ctx->b_views_host, tb, hipHostMallocDefault));
    ctx->b_views_host_bytes = tb;
    HDOF_HIP(hipEventCreateWithFlags(&ctx->b_views_done, hipEventDisableTiming));
  } else {
    HDOF_HIP(hipEventSynchronize(ctx->b_views_done));
  }
  batch_view_pack(L.hv, L.n, ctx->b_views_host);
  ctx->prof_in_frame = false;
  TRY(batch_enqueue(ctx, scene, light, params, views, L, ctx->b_views_host, st));
  HDOF_HIP(hipEventRecord(ctx->b_views_done, st));
  return HDOF_OK;
}

// A batch owns a private context (scratch, flags) so that later frames on
// the caller's context cannot reallocate buffers the graph refers to.
struct hdof_batch {
  hdof_ctx* ctx;
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
  void* table_host;
};

extern "C" void hdof_batch_destroy(hdof_batch* b) {
  if (!b) return;
  hipSetDevice(b->ctx->device);
  hipDeviceSynchronize();
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->stream) hipStreamDestroy(b->stream);
  if (b->table_host) hipHostFree(b->table_host);
  hdof_destroy(b->ctx);
  delete b;
}

extern "C" hdof_status hdof_batch_create(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                                         const hdof_frame_params* params, int32_t n_views,
                                         const hdof_view* views, hdof_batch** out) {
  REQUIRE(out, "out is NULL");
  *out = nullptr;
  static thread_local BatchLayout L;
  TRY(batch_check(ctx, scene, light, params, n_views, views, L));
  hdof_ctx* ictx = nullptr;
  TRY(hdof_create(ctx->device, &ictx));
  ictx->tune = ctx->tune;
  hdof_batch* b = new hdof_batch();
  b->ctx = ictx;
  hdof_status s = batch_reserve(ictx, params, L);
  if (s != HDOF_OK) {
    hdof_batch_destroy(b);
    return s;
  }
  ctx = ictx;
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc(&b->table_host, batch_view_bytes() * HDOF_MAX_VIEWS, hipHostMallocDefault);
  if (e != hipSuccess) {
    hdof_batch_destroy(b);
    return hdof_set_error(HDOF_ERR_HIP, "batch setup: %s", hipGetErrorString(e));
  }
  batch_view_pack(L.hv, L.n, b->table_host);
  // one eager pass builds anything computed on first use (the tap table)
  s = batch_enqueue(ctx, scene, light, params, views, L, b->table_host, b->stream);
  if (s == HDOF_OK && (e = hipStreamSynchronize(b->stream)) != hipSuccess)
    s = hdof_set_error(HDOF_ERR_HIP, "batch warm-up: %s", hipGetErrorString(e));
  ctx->pp_taps_n = 0;  // the graph recomputes its own tap table
  if (s == HDOF_OK) {
    e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) s = hdof_set_error(HDOF_ERR_HIP, "begin capture: %s", hipGetErrorString(e));
  }
  if (s == HDOF_OK) {
    hdof_status se = batch_enqueue(ctx, scene, light, params, views, L, b->table_host, b->stream);
    e = hipStreamEndCapture(b->stream, &b->graph);
    if (se != HDOF_OK) s = se;
    else if (e != hipSuccess) s = hdof_set_error(HDOF_ERR_HIP, "end capture: %s", hipGetErrorString(e));
  }
  if (s == HDOF_OK && (e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
    s = hdof_set_error(HDOF_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
  if (s != HDOF_OK) {
    hdof_batch_destroy(b);
    return s;
  }
  *out = b;
  return HDOF_OK;
}

extern "C" hdof_status hdof_batch_launch(hdof_batch* b, hdof_stream stream) {
  REQUIRE(b, "batch is NULL");
  TRY(check_ctx(b->ctx));
  HDOF_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// differentiable form
// ---------------------------------------------------------------------------
extern "C" hdof_status hdof_postfilter_composite_backward(
    hdof_ctx* ctx, const float* d_color, const float* d_depth, const uint8_t* d_spp, hdof_rt_bufs rt,
    const hdof_camera* cam, const hdof_lens* lens, const hdof_pp_params* pp, const hdof_composite_params* comp,
    const float* d_grad_out, float* d_grad_color, float* d_grad_lens, hdof_stream stream) {
  TRY(check_ctx(ctx));
  REQUIRE(d_color && d_depth && d_spp && d_grad_out && d_grad_color && d_grad_lens,
          "color, depth, spp and gradient buffers must be non-NULL");
  REQUIRE(rt.c_near && rt.c_far && rt.hit_ratio, "c_near, c_far and hit_ratio must be non-NULL");
  TRY(check_camera(cam, "current"));
  TRY(check_lens(lens));
  TRY(check_pp(pp));
  TRY(check_comp(comp));
  if (comp->spec_y > 0.0f)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "the adjoint does not differentiate the specular bokeh rule");
  if (lens->blades != 0 || lens->sa != 0.0f)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "the adjoint takes the disk aperture only");
  CamK k = make_camk(cam);
  return launch_ppc_backward(ctx, d_color, d_depth, d_spp, rt, k, make_lensk(lens, k), *pp, *comp, d_grad_out,
                             d_grad_color, d_grad_lens, (hipStream_t)stream);
}
