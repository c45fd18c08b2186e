// hdof_internal.h -- device helpers and library-internal types of the
// gfx950 hybrid depth-of-field path.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/hdof.h"

#define HDOF_ZMAX 1.0e4f
#define HDOF_SQRT2 1.41421356237309505f
#define HDOF_PI 3.14159265358979324f

// traversal stack: this many entries per lane live in LDS, the rest spill to
// a small private array; beyond both the ray sets the overflow flag.
#define HDOF_LDS_STACK 20
#define HDOF_SPILL_STACK 44
#define HDOF_TRACE_BLOCK 128
#ifndef HDOF_DEFAULT_BPC
#define HDOF_DEFAULT_BPC 10  // persistent trace blocks per CU (its register-limited residency)
#endif
#ifndef HDOF_TRACE_WAVES_PER_EU
#define HDOF_TRACE_WAVES_PER_EU 1  // occupancy the trace kernel's register budget is sized for
#endif
// ints between the persistent trace's per-segment work counters: one
// 128-byte line each (counters sharing a line serialise across XCDs)
#define HDOF_SEG_STRIDE 32

// device flag bits (ctx->d_flags)
#define HDOF_FLAG_STACK_OVERFLOW 1
#define HDOF_FLAG_CAPACITY 2

// history flag bits
#define HDOF_HIST_VALID 1
#define HDOF_HIST_NEW 2

// leaf child encoding: bit 31 set, bits 27..30 = count - 1, bits 0..26 = first
#define HDOF_LEAF_BIT 0x80000000u
#define HDOF_LEAF_FIRST_MASK 0x07FFFFFFu

struct hdof_scene {
  hdof_ctx* ctx;
  int32_t n_tris;
  int32_t n_nodes;
  float4* nodes;   // 4 float4 per node: child boxes x/y (2), z (1), children (1)
  float4* tris;    // 3 float4 per triangle in leaf order; .w of the first = input index
  float* albedo;   // 3 floats per triangle, input order
  float* spec;     // 2 floats per triangle (k_s, shininess), input order; NULL: Lambertian
  int32_t* depth_out;  // [1] tree depth (computed at build)
  int64_t bytes;
};

// host-side description of one view of a batch
struct BatchView;

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct hdof_ctx {
  int device = 0;
  int n_cu = 0;
  int* d_flags = nullptr;  // device-side fault flags
  // trace scratch
  Buf queue, ray_col, ray_z, work_counter;
  // mask scratch
  Buf mask_tile, mask_tile_dil, mask_xpref, mask_rowsum, mask_ybase;
  Buf mask_auto;  // tile 0: per-score-block CoC radius maxima + the chosen tile edge
  // post-filter scratch
  Buf pp_pack, pp_tile, pp_rad, pp_taps;
  // the no-alloc post-filter's scratch on this context's device (the
  // address hipGetSymbolAddress gave for the library's file-scope array)
  void* noalloc_scratch = nullptr;
  int pp_taps_n = 0;  // tap count the table currently holds
  int pp_taps_blades = 0;
  float pp_taps_rot = 0.0f, pp_taps_sa = 0.0f;  // and the aperture it was built for
  // adjoint scratch: CoC per unit aperture, tile / radius arg pixels, block partials
  Buf ppb_args, ppb_partial;
  // variance history (previous frame) and its reprojection into this frame
  int hist_w = 0, hist_h = 0;
  bool hist_any = false;
  Buf hist_m1, hist_m2, hist_flags, hist_z;
  int rep_w = 0, rep_h = 0;
  bool rep_valid = false;
  Buf rep_m1, rep_m2, rep_flags, rep_z;
  // temporal reconstruction of the traced colours: ping-pong history of
  // 9 planes (premultiplied near rgb, near hit ratio, premultiplied far rgb,
  // far-path hit ratio, depth) + valid bytes, and the frame's far positions
  int rec_w = 0, rec_h = 0, rec_cur = 0;
  bool rec_any = false;
  Buf rec_hist[2], rec_valid[2], rec_farpos;
  // spatial reconstruction: box pyramid of the traced pixels (levels 1..5),
  // its tap table, and the frame's pre-gather colours and CoC averages
  Buf sp_levels, sp_taps, sp_cn, sp_cf, sp_coc;
  int sp_taps_n = 0;
  // frame intermediates when the caller keeps none
  Buf f_depth, f_normal, f_albedo, f_color, f_triid, f_spp, f_offsets, f_total;
  Buf f_cn, f_cf, f_h, f_m1, f_m2, f_pp, f_spec, f_pps;
  // persistent-trace launch shape (performance only)
  hdof_tuning tune = {HDOF_DEFAULT_BPC, 64, 8, 0, 1, 140000};
  // the trace's ray quantum while a frame overlaps it with the gather (0: all blocks)
  int trace_ray_quantum = 0;
  // batched form: per-view intermediates, view table (device + pinned host)
  Buf b_arena, b_views, b_totals;
  void* b_views_host = nullptr;
  size_t b_views_host_bytes = 0;
  hipEvent_t b_views_done = nullptr;
  // traversal work counters (rays, node visits, triangle tests) x (G-buffer, trace)
  bool count_on = false;
  unsigned long long* d_counters = nullptr;
  // overlapped frame: the post-filter gather's stream, forked from the
  // frame's stream after the G-buffer and joined before the composite
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_fork2 = nullptr;  // the overlapped batch's second chunk
  // stage profiling: HDOF_PROF_SLOTS events per profiled frame (the stage
  // marks, then the end of an overlapped gather)
  bool prof_on = false, prof_in_frame = false;
  int prof_frames = 0;
  std::vector<hipEvent_t> prof_events;
  std::vector<uint8_t> prof_set;  // which marks of each frame were recorded
};

// record stage boundary `i` of the current profiled frame (no-op when off)
// per profiled frame: marks 0..HDOF_PROFILE_STAGES, then the end of an
// overlapped post-filter gather (recorded on its own stream)
#define HDOF_PROF_SLOTS (HDOF_PROFILE_STAGES + 2)
#define HDOF_PROF_GATHER_END (HDOF_PROFILE_STAGES + 1)
void hdof_prof_mark(hdof_ctx* ctx, int i, hipStream_t st);

// ---------------------------------------------------------------------------
// host-side helpers (api.hip)
// ---------------------------------------------------------------------------
hdof_status hdof_set_error(hdof_status s, const char* fmt, ...);
hdof_status hdof_ensure(Buf& b, size_t bytes);
#define HDOF_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return hdof_set_error(HDOF_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// small vector math (float3 with explicit fma order)
// ---------------------------------------------------------------------------
struct V3 {
  float x, y, z;
};
__host__ __device__ inline V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__host__ __device__ inline V3 v3(const float* p) { return V3{p[0], p[1], p[2]}; }
__device__ inline V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ inline float dot3(V3 a, V3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ inline V3 cross3(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline float comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
__device__ inline float clamp01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }

// pixels per block of the batched per-pixel passes (queue fill, reduction,
// traced pixels' composite): 16 per thread, so a block's view lookup is
// paid once per 4096 pixels
#define HDOF_BATCH_PX_BLOCK 4096
// the view of unit g (a block or a tile) of a launch over a batch's views:
// the last view whose first unit base[v] is <= g (base ascending, base[0] 0)
__device__ inline int batch_view_of(const int* base, int n, int g) {
  int v = 0;
  for (int step = 32; step >= 1; step >>= 1)
    if (v + step < n && base[v + step] <= g) v += step;
  return v;
}

// logical block index so that XCD x (blocks dispatched round-robin over 8
// XCDs) processes one contiguous range of logical blocks
__device__ inline int xcd_block(int b, int nb) {
  int per = nb >> 3, rem = nb & 7;
  int x = b & 7, i = b >> 3;
  return x * per + min(x, rem) + i;
}

// camera constants gathered once per launch
struct CamK {
  V3 e, r, u, w;
  float tx, ty, spx;
  int W, H;
};
inline CamK make_camk(const hdof_camera* c) {
  CamK k;
  k.e = v3(c->eye);
  k.r = v3(c->right);
  k.u = v3(c->up);
  k.w = v3(c->fwd);
  k.tx = c->tan_half_fov_x;
  k.ty = (float)((double)c->tan_half_fov_x * c->height / c->width);
  k.spx = (float)((double)c->width / (2.0 * c->tan_half_fov_x));
  k.W = c->width;
  k.H = c->height;
  return k;
}

// pinhole direction through the centre of pixel (x, y), unit forward part
__device__ inline V3 pixel_dir(const CamK& k, int x, int y) {
  float sx = ((float)(2 * x + 1) / (float)k.W - 1.0f) * k.tx;
  float sy = (1.0f - (float)(2 * y + 1) / (float)k.H) * k.ty;
  return V3{fmaf(sy, k.u.x, fmaf(sx, k.r.x, k.w.x)), fmaf(sy, k.u.y, fmaf(sx, k.r.y, k.w.y)),
            fmaf(sy, k.u.z, fmaf(sx, k.r.z, k.w.z))};
}

#define HDOF_MAX_BLADES 16

// signed CoC diameter in pixels: A (1/S1 - 1/z) s_px; the aperture's
// silhouette (blades 0: disk, else a regular polygon whose first vertex is
// at rot_ht half turns) and spherical aberration sa
struct LensK {
  float f, A, S1, invS1, coc_scale;  // coc_scale = A * s_px
  int blades;
  float rot_ht, sa;
};
inline LensK make_lensk(const hdof_lens* l, const CamK& k) {
  LensK q;
  q.f = l->focal_length;
  q.A = l->aperture;
  q.S1 = l->focus_distance;
  q.invS1 = 1.0f / l->focus_distance;
  q.coc_scale = l->aperture * k.spx;
  q.blades = l->blades;
  q.rot_ht = (float)((double)l->rotation / 3.14159265358979323846);
  q.sa = l->sa;
  return q;
}
__device__ inline float coc_px(const LensK& l, float z) { return l.coc_scale * (l.invS1 - 1.0f / z); }

struct LightK {
  V3 p, I, ka;
};
inline LightK make_lightk(const hdof_light* l) {
  LightK q;
  q.p = v3(l->pos);
  q.I = v3(l->intensity);
  q.ka = v3(l->ambient);
  return q;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): 10 rounds of two 64x64 -> 128-bit
// multiplies, key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                     uint64_t k1, uint64_t& o0, uint64_t& o1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  o0 = c0;
  o1 = c1;
}

// thin-lens ray for sample j of pixel (x, y); pinhole when A == 0.  Disk:
// radius A/2, polar sqrt(u0), 2 pi u1.  Regular B-gon inscribed in it: the
// fan triangle k = floor(B u0) (integer arithmetic on u0's 24 bits, so the
// choice is exact) and in it sqrt(f) (V_k + u1 (V_k+1 - V_k)), f = B u0 - k.
// w (nullable): the sample's spherical-aberration weight
// max(0, 1 + sa (2 rho^2 - 1)), rho = |lens point| / (A/2).
__device__ inline void lens_ray(const CamK& k, const LensK& l, int x, int y, uint32_t j, uint32_t view,
                                uint32_t seed, uint32_t frame, V3& O, V3& D, float* w = nullptr) {
  V3 v = pixel_dir(k, x, y);
  uint64_t w0, w1;
  philox4x64_10((uint64_t)y * (uint64_t)k.W + (uint64_t)x, j, view, 0, seed, frame, w0, w1);
  const uint32_t m0 = (uint32_t)(w0 >> 40);
  float u1 = (float)(uint32_t)(w1 >> 40) * (1.0f / 16777216.0f);
  float lx, ly;
  const float a = 0.5f * l.A;
  if (l.blades >= 3) {
    const uint32_t mb = m0 * (uint32_t)l.blades;
    const int kk = (int)(mb >> 24);
    const float sq = a * sqrtf((float)(mb & 0xFFFFFFu) * (1.0f / 16777216.0f));
    const float step = 2.0f / (float)l.blades;
    float s0, c0, s1, c1;
    sincospif(fmaf((float)kk, step, l.rot_ht), &s0, &c0);
    sincospif(fmaf((float)(kk + 1), step, l.rot_ht), &s1, &c1);
    lx = sq * fmaf(u1, c1 - c0, c0);
    ly = sq * fmaf(u1, s1 - s0, s0);
  } else {
    float u0 = (float)m0 * (1.0f / 16777216.0f);
    float rho = a * sqrtf(u0);
    float s, c;
    sincospif(2.0f * u1, &s, &c);
    lx = rho * c;
    ly = rho * s;
  }
  if (w) {
    const float r2 = a > 0.0f ? fmaf(lx, lx, ly * ly) / (a * a) : 0.0f;
    *w = fmaxf(0.0f, fmaf(l.sa, fmaf(2.0f, r2, -1.0f), 1.0f));
  }
  V3 lv = V3{fmaf(ly, k.u.x, lx * k.r.x), fmaf(ly, k.u.y, lx * k.r.y), fmaf(ly, k.u.z, lx * k.r.z)};
  O = k.e + lv;
  D = V3{fmaf(l.S1, v.x, -lv.x), fmaf(l.S1, v.y, -lv.y), fmaf(l.S1, v.z, -lv.z)};
}

// ---------------------------------------------------------------------------
// launchers (one per translation unit)
// ---------------------------------------------------------------------------
hdof_status launch_bvh_build(hdof_ctx* ctx, const float* verts, const float* albedo, int n,
                             hdof_scene* sc, hipStream_t st);
hdof_status launch_gbuffer(hdof_ctx* ctx, const hdof_scene* sc, const CamK& k, const LensK& l,
                           const LightK& li, hdof_gbuffer_bufs out, hipStream_t st, float4* pack = nullptr,
                           float* tile_r = nullptr, hipEvent_t done = nullptr);
struct BatchView {
  CamK k;
  LensK l;
  uint32_t seed, frame, view;
  int px_base;  // first pixel of the view in the batch's concatenated planes
};
// every view's G-buffer in one launch (packed texels and 16-pixel tile
// radii too): planes concatenated per view from its px_base, tile radii from
// the view's first 16x16 block; views_dev is the device copy of hviews
hdof_status launch_gbuffer_batched(hdof_ctx* ctx, const hdof_scene* sc, const LightK& li, int n_views,
                                   const BatchView* hviews, const void* views_dev, hdof_gbuffer_bufs out,
                                   float4* pack, float* tile_r, hipStream_t st);
hdof_status reserve_trace(hdof_ctx* ctx, size_t cap, bool own_depth);
hdof_status launch_trace_batched(hdof_ctx* ctx, const hdof_scene* sc, const LightK& li, int spp_max,
                                 int n_views, const BatchView* hviews, const void* views_dev,
                                 const uint8_t* spp, const int32_t* offsets, const int32_t* totals,
                                 int32_t* ebase, int32_t* grand, hdof_rt_bufs* rt, hipStream_t st);
size_t batch_view_bytes();
void batch_view_pack(const BatchView* hv, int n, void* out);
// Variance history update fused into the trace's per-pixel reduction
// (whole frames): the reprojected history in, the new history out.
struct VarFuse {
  float alpha;
  const float* depth;
  const float *rm1, *rm2;
  const uint8_t* rfl;
  float *m1, *m2;
  uint8_t* fl;
  float* hz;
  // untraced pixels leave the trace planes (near, far, hit ratio, luminance
  // moments) unwritten: a frame whose caller keeps none of them and whose
  // later stages read them only where the pixel was traced
  int sparse_rt;
  // the history is updated in the reprojected planes themselves (m1, m2, fl
  // are rm1, rm2, rfl): traced pixels only, the depth already there; the
  // frame then swaps the reprojected and the history planes
  int in_place;
};
// checks the frame's reprojection, reserves the history and marks it
// written (as launch_var_update does before its launch)
hdof_status var_update_prepare(hdof_ctx* ctx, const CamK& k, float alpha, const float* depth, VarFuse* vf,
                               bool in_place = false);
// the frame's in-place history update: the reprojected planes become the
// history (after the reduction that updated them is enqueued)
void history_swap(hdof_ctx* ctx);
hdof_status launch_trace(hdof_ctx* ctx, const hdof_scene* sc, const CamK& k, const LensK& l,
                         const LightK& li, int spp_max, const uint8_t* spp, const int32_t* offsets,
                         const int32_t* total, uint32_t seed, uint32_t frame, uint32_t view,
                         hdof_rt_bufs out, int32_t* ray_id, float* ray_depth, float* far_pos, hipStream_t st,
                         const VarFuse* vf = nullptr, bool queue_ready = false, float* coc_nf = nullptr);
hdof_status launch_recon(hdof_ctx* ctx, const CamK& k, const CamK* prev, const float* depth, const uint8_t* spp,
                         const float* far_pos, hdof_rt_bufs rt, float alpha, hipStream_t st);
// spatial reconstruction: in -> (cn_out, cf_out); hacc nullable (latest hit
// ratio); variance plane nullable; var_from_history: the variance estimate
// of the context's current variance history instead; zero_untraced: the
// untraced inputs are known to be 0 (written without reading them)
hdof_status spatial_reserve(hdof_ctx* ctx, int W, int H);
hdof_status launch_spatial(hdof_ctx* ctx, int W, int H, const uint8_t* spp, hdof_rt_bufs in, const float* hacc,
                           const float* coc_nf, const float* variance, bool var_from_history,
                           const hdof_spatial_params& sp, float* cn_out, float* cf_out, hipStream_t st,
                           bool zero_untraced = false);
// the mask's scratch for a W x H frame (tile 0: every candidate grid)
hdof_status mask_reserve(hdof_ctx* ctx, int W, int H, const hdof_mask_params& mp);
// the batched form's masks (fixed mask tiles; no history), one launch per
// pass over every view: counts and view-local offsets into each view's
// spp/offsets planes (concatenated from px_base), each view's ray total
// into totals[v]; views_dev is the device copy of hviews
hdof_status mask_reserve_batched(hdof_ctx* ctx, int n_views, const BatchView* hviews, const hdof_mask_params& mp);
hdof_status launch_mask_batched(hdof_ctx* ctx, const float* depth, const float* normal, int n_views,
                                const BatchView* hviews, const void* views_dev, const hdof_mask_params& mp,
                                uint8_t* spp, int32_t* offsets, int32_t* totals, hipStream_t st);
// lens: needed for tile 0 (the mask tile scaled by the frame's maximum CoC);
// write_rep false: the reprojected history is not written (no later
// variance update of this frame reads it: batched views, captured frames)
hdof_status launch_mask(hdof_ctx* ctx, const float* depth, const float* normal, const CamK& k,
                        const CamK* prev, const hdof_mask_params& mp, uint8_t* spp, int32_t* offsets,
                        int32_t* total, hipStream_t st,
                        int* queue = nullptr, long cap = 0, int* counter = nullptr, const LensK* lens = nullptr,
                        bool write_rep = true);
hdof_status launch_var_update(hdof_ctx* ctx, const CamK& k, float alpha, const uint8_t* spp,
                              const float* depth, const float* m1, const float* m2, hipStream_t st);
// Composite fused into the post-filter of a whole frame (the gather writes
// the final colour; its filtered colour goes to `out` only when non-NULL).
struct PostFuse {
  const uint8_t* spp;
  hdof_rt_bufs rt;
  hdof_composite_params cp;
  float* out;
  const float* pps;  // nullable: post-filtered specular luminance (the specular bokeh rule)
  // 16-pixel tiles: the epilogue applies the untraced pixels' rule to every
  // pixel and reads none of spp, rt, pps (the trace may still be writing
  // them); a sparse composite then rewrites the traced pixels
  bool untraced_only;
  // nullable (untraced_only): an event the gather's own dispatch completes,
  // so no separate marker follows it on its stream
  hipEvent_t done;
};
// the post-filter's scratch and tap table for this image and lens, on st
// (a frame that runs the gather on another stream calls it before forking)
hdof_status postfilter_reserve(hdof_ctx* ctx, const CamK& k, const LensK& l, const hdof_pp_params& pp,
                               hipStream_t st);
// the no-alloc post-filter: the scratch address on the current device
// (looked up once per device), and the launch into it
hdof_status postfilter_noalloc_init(int device, void** out);
hdof_status launch_postfilter_noalloc(hdof_ctx* ctx, const float* color, const float* depth, const CamK& k,
                                      const LensK& l, const hdof_pp_params& pp, float* out, hipStream_t st);
// the batched form's gathers over every view in one launch (16-pixel
// tiles; each view's pixels by the composite's untraced rule into outs[v],
// its filtered colour into pp_out from its px_base), and its traced pixels'
// composite in one launch; planes concatenated per view from px_base, tile
// radii from the view's first tile; views_dev is the device copy of hviews
hdof_status launch_postfilter_batched(hdof_ctx* ctx, const float4* pack, const float* tile_r, int n_views,
                                      const BatchView* hviews, const void* views_dev, float* const* outs,
                                      const hdof_pp_params& pp, float* pp_out, hipStream_t st);
hdof_status launch_composite_traced_batched(hdof_ctx* ctx, const float* color, const float* pp, const float* depth,
                                            const uint8_t* spp, hdof_rt_bufs rt, int n_views,
                                            const BatchView* hviews, const void* views_dev, float* const* outs,
                                            const hdof_composite_params& cp, hipStream_t st);
// packed: pack and per-tile radius already written (by the G-buffer)
hdof_status launch_postfilter(hdof_ctx* ctx, const float* color, const float* depth, const CamK& k,
                              const LensK& l, const hdof_pp_params& pp, float* out, hipStream_t st,
                              bool packed = false, const PostFuse* fuse = nullptr);
hdof_status launch_ppc_backward(hdof_ctx* ctx, const float* color, const float* depth, const uint8_t* spp,
                                hdof_rt_bufs rt, const CamK& k, const LensK& l, const hdof_pp_params& pp,
                                const hdof_composite_params& cp, const float* grad_out, float* grad_color,
                                float* grad_lens, hipStream_t st);
// sparse: only the traced pixels (spp > 0) are written; the others already
// hold the untraced rule's result (the overlapped frame's gather epilogue)
hdof_status launch_composite(hdof_ctx* ctx, const float* color, const float* pp, const float* depth,
                             const uint8_t* spp, hdof_rt_bufs rt, const CamK& k, const LensK& l,
                             const hdof_composite_params& cp, float* out, hipStream_t st,
                             const float* pps = nullptr, bool sparse = false);
// the post-filtered specular luminance of the traced pixels (all pixels when
// spp is NULL); reads the frame's post-filter preparation (packed CoC, tile
// radii, taps), so it follows the G-buffer's packing or launch_postfilter
hdof_status launch_pp_spec(hdof_ctx* ctx, const float* ys, const uint8_t* spp, const CamK& k, const LensK& l,
                           const hdof_pp_params& pp, float* out, hipStream_t st);
