/*
 * hdof.h -- C ABI of the MI355X (gfx950) hybrid depth-of-field hot path.
 *
 * Method: Tan, Chua, Biette, Bhojan, "Hybrid DoF: Ray-Traced and
 * Post-Processed Hybrid Depth of Field Effect for Real-Time Rendering"
 * (SIGGRAPH 2020 posters).  One frame runs, in the paper's order:
 *   G-buffer with a sharp image (Design)                     -> hdof_gbuffer
 *   adaptive ray mask: Gaussian, Sobel on normal and depth,
 *   temporally accumulated luminance variance (Ray Trace)    -> hdof_ray_mask
 *   thin-lens distributed ray tracing of the masked pixels,
 *   near/far split and hit ratio (Ray Trace)                 -> hdof_trace_thin_lens
 *   temporal reconstruction of the near and far traced
 *   colours (Reconstruction)                                 -> hdof_rt_reconstruct
 *   spatial reconstruction of the traced colours
 *   (Reconstruction)                                         -> hdof_rt_spatial
 *   variance history update (Ray Trace)                      -> hdof_variance_update
 *   post-process gather filter (Design; rejection rule from
 *   Reconstruction)                                          -> hdof_postfilter
 *   near/far composite (Composite)                           -> hdof_composite
 * and hdof_frame chains all of them.  Scene acceleration (the paper relies on
 * hardware BVHs) is hdof_build_bvh.
 *
 * Conventions shared by every entry point
 *  - Pointers named d_* are DEVICE pointers on the context's GPU, owned by
 *    the caller, contiguous.  Images are planar float32 [C][H][W] in
 *    row-major pixel order (pixel (x, y) at y*W + x, y pointing down).
 *  - Every call only enqueues work on `stream` (a hipStream_t; NULL = the
 *    null stream) and returns; results are ready when the stream is.
 *    No call synchronises the host except hdof_create, hdof_destroy,
 *    hdof_scene_destroy, hdof_scene_stats, hdof_history_reset and hdof_sync.
 *  - Arguments are validated before anything is enqueued; a failing call
 *    enqueues nothing and returns a status; hdof_last_error() then holds a
 *    message for the calling thread.  Nothing throws across this ABI.
 *  - Faults found on the device (traversal stack overflow) set a flag that
 *    hdof_sync reports as HDOF_ERR_CAPACITY.
 *  - A context is not thread-safe; use one per host thread.
 *  - Camera and lens scalars are float32, so a reference implementation in
 *    double precision can widen exactly the same values.
 */
#ifndef HDOF_H
#define HDOF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HDOF_OK = 0,
  HDOF_ERR_INVALID_ARG = 1, /* a pointer, size or parameter out of range      */
  HDOF_ERR_UNSUPPORTED = 2, /* device is not gfx950                            */
  HDOF_ERR_OOM = 3,         /* device allocation of library scratch failed     */
  HDOF_ERR_CAPACITY = 4,    /* a device-side limit was hit (see hdof_sync)     */
  HDOF_ERR_HIP = 5          /* a HIP runtime call failed                       */
} hdof_status;

typedef struct hdof_ctx hdof_ctx;     /* device, scratch, variance history   */
typedef struct hdof_scene hdof_scene; /* BVH + triangles + albedo on device  */
typedef void* hdof_stream;            /* hipStream_t                          */

/* Pinhole frame of the thin-lens camera (paper, Design: thin lens model).
 * right/up/fwd orthonormal; the ray through the centre of pixel (x, y) has
 * direction v = fwd + sx right + sy up with
 *   sx = (2 (x + 0.5) / width - 1) tan_half_fov_x,
 *   sy = (1 - 2 (y + 0.5) / height) tan_half_fov_x height / width. */
typedef struct {
  float eye[3], right[3], up[3], fwd[3];
  float tan_half_fov_x;
  int32_t width, height;
} hdof_camera;

/* Thin lens: focal length f (m), aperture DIAMETER A = f / N (m; 0 = pinhole),
 * focus distance S1 (m, axial, > f).  Signed circle of confusion of axial
 * depth z, in pixels: c(z) = A (1/S1 - 1/z) width / (2 tan_half_fov_x);
 * negative = near field (in front of the focus plane), positive = far. */
typedef struct {
  float focal_length, aperture, focus_distance;
  /* aperture silhouette and spherical aberration (paper, Discussion: bokeh
   * shapes other than the disk, relative weights of the samples): blades 0
   * = the disk, 3..16 = the regular polygon inscribed in the aperture
   * circle with its first vertex at `rotation` (rad); sa in [-4, 4]: a lens
   * sample (or post-filter tap) at normalised radius rho weighs
   * max(0, 1 + sa (2 rho^2 - 1)).  0, 0, 0 = the thin lens of the paper. */
  int32_t blades;
  float rotation, sa;
} hdof_lens;

/* One point light (position, rgb intensity) and an rgb ambient term for the
 * two-sided Lambertian shading of both the G-buffer and the traced rays. */
typedef struct {
  float pos[3], intensity[3], ambient[3];
} hdof_light;

/* Adaptive ray mask (paper, Ray Trace).  sigma in (0, 2]: Gaussian on depth
 * and normal before the 3x3 Sobel; tau_*: score normalisers (> 0);
 * var_alpha in [0, 1]: EMA weight of the luminance moments; spp_max in
 * [1, 255]; tile in {1, 2, 4, 8, 16}: mask tile edge in pixels (tile max),
 * or 0: the edge scaled by the frame's largest CoC radius R over its pixels
 * (paper, Discussion: mask resolution from the maximum CoC), 4 for R < 16 px,
 * 8 for R < 32 px, else 16, chosen on the device each frame;
 * dilate in [0, 8]: tile dilation radius. */
typedef struct {
  float sigma, tau_depth, tau_normal, tau_var, var_alpha;
  int32_t spp_max, tile, dilate;
} hdof_mask_params;

/* Post-process gather filter.  n_taps in [1, 256]; tile in {4, 8, 16}:
 * CoC tile edge in pixels; r_cap in [0, 256]: largest gather radius (px);
 * bg_ramp_px > 0: width of the background clamp ramp in CoC pixels. */
typedef struct {
  int32_t n_taps, tile;
  float r_cap, bg_ramp_px;
} hdof_pp_params;

/* Composite.  h_t > 0: hit ratio below which far pixels blend towards the
 * ray-traced colour; rt_override != 0: output the ray-traced colour wherever
 * a pixel was traced (full ray-traced reference mode); spec_y >= 0: the
 * specular bokeh rule (paper, Composite): near traced pixels move from the
 * ray-traced towards the post-process colour by clamp(Y_s,pp / spec_y, 0, 1),
 * Y_s,pp the post-filtered specular luminance (0 = off). */
typedef struct {
  float h_t;
  int32_t rt_override;
  float spec_y;
} hdof_composite_params;

/* Temporal reconstruction of the traced colours (paper, Reconstruction).
 * enable in {0, 1}; alpha in (0, 1]: weight of the current frame in the
 * exponential moving average. */
typedef struct {
  int32_t enable;
  float alpha;
} hdof_recon_params;

/* Spatial reconstruction of the traced colours (paper, Reconstruction, last
 * paragraph).  enable in {0, 1} (read by hdof_frame only); n_taps in
 * [1, 256]: golden-angle taps of the gather; r_cap in [0, 256]: largest
 * gather radius (px); v_clamp > 0: variance estimate at and above which the
 * gathered colour fully replaces the pixel's own. */
typedef struct {
  int32_t enable, n_taps;
  float r_cap, v_clamp;
} hdof_spatial_params;

typedef struct {
  hdof_mask_params mask;
  hdof_pp_params pp;
  hdof_composite_params comp;
  hdof_recon_params recon;
  hdof_spatial_params spatial;
} hdof_frame_params;

/* G-buffer planes: depth [H][W] (axial, 1e4 on a miss), normal [3][H][W]
 * (face normal facing the viewer; 0 on a miss), albedo [3][H][W], color
 * [3][H][W] (shaded sharp image C_r), tri_id [H][W] (input triangle index,
 * -1 on a miss), spec [H][W] (optional, may be NULL: luminance of the
 * specular part of color; 0 for a Lambertian scene). */
typedef struct {
  float *depth, *normal, *albedo, *color;
  int32_t* tri_id;
  float* spec;
} hdof_gbuffer_bufs;

/* Per-pixel ray-trace results: c_near, c_far [3][H][W] (near- and far-field
 * weighted mean colours), hit_ratio [H][W] (near weight / rays), lum_m1,
 * lum_m2 [H][W] (mean luminance and mean squared luminance of the rays).
 * All zero where no ray was traced. */
typedef struct {
  float *c_near, *c_far, *hit_ratio, *lum_m1, *lum_m2;
} hdof_rt_bufs;

/* Optional caller-owned intermediates of hdof_frame.  A NULL member makes the
 * frame use library scratch for that buffer. */
typedef struct {
  hdof_gbuffer_bufs gb;
  uint8_t* spp;      /* [H][W] */
  int32_t* offsets;  /* [H][W] */
  int32_t* total;    /* [1] */
  hdof_rt_bufs rt;
  float* pp;         /* [3][H][W] */
} hdof_frame_bufs;

typedef struct {
  int32_t n_tris, n_nodes, max_depth, leaf_size;
  int64_t device_bytes;
} hdof_scene_info;

/* ---------------------------------------------------------------------- */
/* Context                                                                 */
/* ---------------------------------------------------------------------- */

/* Create a context on HIP device `device` (must be gfx950, else
 * HDOF_ERR_UNSUPPORTED).  Makes `device` current on the calling thread. */
hdof_status hdof_create(int device, hdof_ctx** out);
/* Synchronises the device, then frees all library scratch. NULL is a no-op. */
void hdof_destroy(hdof_ctx* ctx);
const char* hdof_status_str(hdof_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* hdof_last_error(void);
/* Waits for `stream`, then reports and clears device-side flags
 * (HDOF_ERR_CAPACITY after a traversal stack overflow). */
hdof_status hdof_sync(hdof_ctx* ctx, hdof_stream stream);

/* ---------------------------------------------------------------------- */
/* Scene (acceleration structure; the paper uses the driver's hardware BVH) */
/* ---------------------------------------------------------------------- */

/* Specular materials (paper, Composite: specular bokeh): d_spec holds
 * n_tris x 2 floats (k_s >= 0, shininess >= 1) in input triangle order,
 * copied on `stream`; every shading (G-buffer, traced rays) then adds the
 * Blinn-Phong lobe k_s I max(0, n.h)^shininess / max(d^2, 1e-4) while the
 * light is on the viewer's side (h: unit half vector of the light direction
 * and the direction back along the ray).  d_spec == NULL synchronises the
 * device and makes the scene Lambertian again. */
hdof_status hdof_scene_set_specular(hdof_scene* scene, const float* d_spec, hdof_stream stream);

/* Build a binary BVH over n_tris triangles: Morton-ordered leaves clustered
 * bottom-up by PLOC (nearest neighbour by merged-box surface area within a
 * window of the Morton order), nodes placed depth-first, leaves of at most 4
 * triangles.  d_verts: n_tris x 9 floats (v0.xyz v1.xyz v2.xyz);
 * d_albedo: n_tris x 3 floats.  The inputs are read on `stream` and may be
 * freed once the stream has passed this call.  n_tris in [1, 2^26].
 * *out is owned by the caller and freed with hdof_scene_destroy. */
hdof_status hdof_build_bvh(hdof_ctx* ctx, const float* d_verts, const float* d_albedo,
                           int32_t n_tris, hdof_scene** out, hdof_stream stream);
/* Synchronises the device, then frees the scene.  NULL is a no-op. */
void hdof_scene_destroy(hdof_scene* scene);
/* Synchronises the device and reports node count, tree depth and bytes. */
hdof_status hdof_scene_stats(hdof_scene* scene, hdof_scene_info* out);

/* ---------------------------------------------------------------------- */
/* Hot-path stages                                                          */
/* ---------------------------------------------------------------------- */

/* G-buffer (paper, Design): one pinhole ray per pixel centre (lens offset 0),
 * closest hit (smallest t > 0, ties to the lowest triangle index), face
 * normal, albedo and two-sided Lambertian colour (no shadow rays).  All five
 * planes of `out` must be non-NULL. */
hdof_status hdof_gbuffer(hdof_ctx* ctx, const hdof_scene* scene, const hdof_camera* cam,
                         const hdof_lens* lens, const hdof_light* light,
                         hdof_gbuffer_bufs out, hdof_stream stream);

/* Adaptive ray mask (paper, Ray Trace).  Reads in->depth and in->normal.
 * Score m = max(g_z / tau_depth, g_n / tau_normal, V / tau_var), where g_z and
 * g_n are Sobel magnitudes of the Gaussian-blurred depth (relative to depth)
 * and normal, and V the variance of the reprojected luminance history
 * (+inf where the history is new, 0 without history).  Per-pixel count
 * min(spp_max, ceil(m)) for m >= 1, else 0; tile max; dilation over tiles.
 * Writes d_spp [H][W], d_offsets [H][W] (exclusive prefix sum of d_spp in
 * pixel order) and d_total [1].  prev == NULL: no history (first frame or a
 * camera cut); otherwise the context's history (written by the previous
 * hdof_variance_update at prev's resolution) is reprojected into the current
 * frame and kept for the next hdof_variance_update. */
hdof_status hdof_ray_mask(hdof_ctx* ctx, const hdof_gbuffer_bufs* in, const hdof_camera* cam,
                          const hdof_camera* prev, const hdof_lens* lens,
                          const hdof_mask_params* params, uint8_t* d_spp, int32_t* d_offsets,
                          int32_t* d_total, hdof_stream stream);

/* Thin-lens distributed ray trace of the masked pixels (paper, Ray Trace).
 * Sample j of pixel p draws Philox4x64-10 with counter (p, j, view, 0) and
 * key (seed, frame); the top 24 bits of words 0 and 1 give u0, u1; lens point
 * (A/2) sqrt(u0) (cos 2 pi u1, sin 2 pi u1) in the right/up plane; the ray
 * aims through the pixel's focus-plane point.  Per pixel over its d_spp[p]
 * rays: near weight w = clamp(0.5 - c(z)/(2 sqrt 2), 0, 1) of each hit depth z,
 * c_near / c_far = w- and (1-w)-weighted mean colours, hit_ratio = sum w / s,
 * luminance moments.  d_offsets must be the exclusive prefix sum of d_spp and
 * *d_total its sum (as hdof_ray_mask writes them); d_total stays on the
 * device.  Optional debug outputs per queue entry (index d_offsets[p] + j):
 * d_ray_tri_id (hit triangle, -1 on miss) and d_ray_depth (axial depth);
 * each needs W*H*spp_max entries.  Optional d_far_pos [4][H][W]: over the
 * pixel's rays that hit, the (1 - w)-weighted mean hit point (planes 0-2,
 * world coordinates) and the weight sum (plane 3; 0: no far hit), the input
 * of hdof_rt_reconstruct.  Optional d_coc_nf [2][H][W]: the average CoC
 * size (diameter, px) of the pixel's near rays, sum w |c| / sum w, and of
 * its far rays, sum (1 - w) |c| / sum (1 - w) (0 where the weight sum is 0;
 * a miss counts at depth 1e4), the input of hdof_rt_spatial. */
hdof_status hdof_trace_thin_lens(hdof_ctx* ctx, const hdof_scene* scene, const hdof_camera* cam,
                                 const hdof_lens* lens, const hdof_light* light, int32_t spp_max,
                                 const uint8_t* d_spp, const int32_t* d_offsets,
                                 const int32_t* d_total, uint32_t seed, uint32_t frame,
                                 uint32_t view, hdof_rt_bufs out, int32_t* d_ray_tri_id,
                                 float* d_ray_depth, float* d_far_pos, float* d_coc_nf,
                                 hdof_stream stream);

/* Temporal reconstruction of the near and far traced colours (paper,
 * Reconstruction: exponential moving average as in TAA; near pixels
 * reprojected by their screen-space motion, far pixels through the average
 * world position of their far hits or of their neighbours'; colours
 * normalised by the accumulated hit ratio, composed with the latest one by
 * hdof_composite).  Per traced pixel (d_spp > 0) with hit ratio h:
 *   near: the G-buffer point e + z v reprojected into `prev` (nearest pixel
 *     q_n), usable when the history is valid there and its depth agrees
 *     within 1 %; far: d_far_pos of the pixel when its weight is > 0, else
 *     the mean of its 8 neighbours' that are, reprojected (nearest pixel
 *     q_f), usable when the history is valid there.
 *   N = (1-alpha) N(q_n) + alpha h C_tn,     Hn = (1-alpha) Hn(q_n) + alpha h
 *   F = (1-alpha) F(q_f) + alpha (1-h) C_tf, Hf = (1-alpha) Hf(q_f) + alpha h
 *   (restarted as h C_tn, h, (1-h) C_tf, h without usable history);
 *   rt.c_near <- N / Hn, rt.c_far <- F / (1 - Hf) (unchanged when the
 *   denominator is 0).  Untraced pixels keep their colours.
 * The context's history (written by the previous call at the same size) is
 * read when prev != NULL and replaced by this frame's.  rt.c_near and
 * rt.c_far are updated in place; rt.hit_ratio is read.  params->enable is
 * not consulted (the call always reconstructs). */
hdof_status hdof_rt_reconstruct(hdof_ctx* ctx, const hdof_camera* cam, const hdof_camera* prev,
                                const float* d_depth, const uint8_t* d_spp, const float* d_far_pos,
                                hdof_rt_bufs rt, const hdof_recon_params* params, hdof_stream stream);

/* Replace / read / clear the context's reconstruction history (width x
 * height): d_planes [8][H][W] = premultiplied near rgb, near hit ratio,
 * premultiplied far rgb, far-path hit ratio; d_valid [H][W] (1 = valid);
 * d_depth [H][W] = the depth of the frame that wrote it.  Load/save enqueue
 * copies on `stream`. */
hdof_status hdof_recon_history_load(hdof_ctx* ctx, int32_t width, int32_t height, const float* d_planes,
                                    const uint8_t* d_valid, const float* d_depth, hdof_stream stream);
hdof_status hdof_recon_history_save(hdof_ctx* ctx, float* d_planes, uint8_t* d_valid, float* d_depth,
                                    hdof_stream stream);
hdof_status hdof_recon_history_reset(hdof_ctx* ctx);

/* Spatial reconstruction of the near and far traced colours (paper,
 * Reconstruction: the near and far CoC sizes blended by the accumulated hit
 * ratio scale a circular gather and set its level of detail; samples whose
 * CoC radius is smaller than their distance are rejected; a clamped variance
 * estimate weights the gathered colour).  Per traced pixel q (d_spp > 0),
 * with H the accumulated hit ratio (d_hit_acc, or rt.hit_ratio when NULL)
 * and d_coc_nf as hdof_trace_thin_lens writes it:
 *   r_q = min(r_cap, (H c_near_avg + (1 - H) c_far_avg) / 2).
 * A level-L texel (L = 1..5, 2^L x 2^L pixels) sums over its traced pixels
 * s h C_near, s h, s (1-h) C_far, s (1-h), r and their count (s = rays,
 * h = hit ratio); level 0 is the pixels themselves.  A traced pixel p uses
 * L = floor(log2(r_p sqrt(pi / n_taps))) clamped to [0, 5] and the taps
 * u_k of hdof_postfilter scaled by r_p: each tap takes the level-L texel of
 * the pixel it falls in (clamped to the image) with weight
 * clamp(rbar - r_p |u_k| + 0.5, 0, 1), rbar the texel's mean radius.
 * G_near = (s h C_near(p) + sum of weighted near sums) / (s h + sum of
 * weighted near weights) (C_near(p) when the denominator is 0), G_far
 * alike; lambda = clamp(V / v_clamp, 0, 1) with V = d_variance[p] (+inf or
 * d_variance == NULL: lambda = 1); out = C + lambda (G - C).  Untraced
 * pixels are copied.  Outputs [3][H][W] must not alias the inputs.  Uses
 * library scratch (the pyramid, 48 B per 4 pixels). */
hdof_status hdof_rt_spatial(hdof_ctx* ctx, int32_t width, int32_t height, const uint8_t* d_spp,
                            hdof_rt_bufs rt, const float* d_hit_acc, const float* d_coc_nf,
                            const float* d_variance, const hdof_spatial_params* params,
                            float* d_c_near_out, float* d_c_far_out, hdof_stream stream);

/* Variance history update (paper, Ray Trace: temporally accumulated variance).
 * Where traced: EMA with weight params->var_alpha over the reprojected
 * history, or a restart flagged "new" where no history was valid; where not
 * traced: the reprojected history is carried.  Stores d_depth as the history
 * depth for the next frame's reprojection depth test.  Must follow the
 * hdof_ray_mask call of the same frame. */
hdof_status hdof_variance_update(hdof_ctx* ctx, const hdof_camera* cam,
                                 const hdof_mask_params* params, const uint8_t* d_spp,
                                 const float* d_depth, const float* d_lum_m1,
                                 const float* d_lum_m2, hdof_stream stream);

/* Replace / read / clear the context's variance history (width x height;
 * flags bit0 = valid, bit1 = new).  Load/save enqueue copies on `stream`. */
hdof_status hdof_history_load(hdof_ctx* ctx, int32_t width, int32_t height, const float* d_lum_m1,
                              const float* d_lum_m2, const uint8_t* d_flags,
                              const float* d_depth, hdof_stream stream);
hdof_status hdof_history_save(hdof_ctx* ctx, float* d_lum_m1, float* d_lum_m2, uint8_t* d_flags,
                              float* d_depth, hdof_stream stream);
hdof_status hdof_history_reset(hdof_ctx* ctx);

/* Post-process gather DoF filter (paper, Design: adapted post-process; the
 * CoC-radius rejection of Reconstruction).  Gather radius = min(r_cap, max
 * CoC radius over the tiles within ceil(r_cap / tile) tiles); n_taps
 * golden-angle taps u_k = sqrt((k - 0.5)/n) (cos k g, sin k g),
 * g = pi (3 - sqrt 5); bilinear colour + signed CoC; a tap at distance d
 * counts with clamp(r_eff - d + 0.5, 0, 1), r_eff its CoC radius clamped to
 * the centre's when it lies behind; weights (R^2/n) / max(r, 0.5)^2, centre
 * 1 / max(r_p, 0.5)^2.  d_color [3][H][W], d_depth [H][W] -> d_out [3][H][W]
 * (must not alias d_color). */
hdof_status hdof_postfilter(hdof_ctx* ctx, const float* d_color, const float* d_depth,
                            const hdof_camera* cam, const hdof_lens* lens,
                            const hdof_pp_params* params, float* d_out, hdof_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * post-filter as hdof_postfilter, same kernels and same results bit for bit,
 * with its scratch (tap table, tile radii, dilated radii, packed texels) in
 * one file-scope device array of HDOF_POSTFILTER_NOALLOC_BYTES that every
 * device the library runs on holds from the library's first context on that
 * device until the process ends.  It calls no hipMalloc, hipFree or
 * allocating routine; the caller still owns d_color, d_depth and d_out.
 * Images above HDOF_POSTFILTER_NOALLOC_MAX_PX pixels (2560 x 1440) are
 * refused with HDOF_ERR_CAPACITY before any launch; other arguments are
 * checked as for hdof_postfilter.  Every call on one device shares that
 * device's array: calls whose work overlaps on one device (two streams, two
 * contexts, two threads) race; a call rewrites everything it reads, so
 * nothing needs clearing between calls. */
#define HDOF_POSTFILTER_NOALLOC_MAX_PX 3686400
#define HDOF_POSTFILTER_NOALLOC_BYTES (4096u + 2u * 954624u + 16u * HDOF_POSTFILTER_NOALLOC_MAX_PX) /* 58.1 MiB */
hdof_status hdof_postfilter_noalloc(hdof_ctx* ctx, const float* d_color, const float* d_depth,
                                    const hdof_camera* cam, const hdof_lens* lens,
                                    const hdof_pp_params* params, float* d_out, hdof_stream stream);

/* The post-filter plus the post-filtered specular luminance (paper,
 * Composite: the specular component's intensity in the post-process colour):
 * hdof_postfilter on d_color into d_out, and the same gather (radius, taps,
 * weights) applied to d_spec [H][W] (the G-buffer's specular luminance) into
 * d_spec_out [H][W].  d_spp (nullable): where given, only pixels with
 * d_spp > 0 gather the specular plane (the composite reads no other), the
 * rest are 0. */
hdof_status hdof_postfilter_specular(hdof_ctx* ctx, const float* d_color, const float* d_depth,
                                     const float* d_spec, const uint8_t* d_spp, const hdof_camera* cam,
                                     const hdof_lens* lens, const hdof_pp_params* params, float* d_out,
                                     float* d_spec_out, hdof_stream stream);

/* Composite (paper, Composite).  phi = clamp(|c| - sqrt 2, 0, 1) blends the
 * sharp colour (focus zone |c| < sqrt 2) with the out-of-focus colour; near
 * field: ray-traced colour where traced, else post-process; far field:
 * beta = clamp(1 - h / h_t, 0, 1) of ray-traced over post-process where
 * traced.  C_rt = h c_near + (1 - h) c_far.  With d_pp_spec (the post-
 * filtered specular luminance, as hdof_postfilter_specular writes it) and
 * params->spec_y > 0, the near traced colour is C_rt + sigma (C_pp - C_rt),
 * sigma = clamp(d_pp_spec / spec_y, 0, 1); d_pp_spec may be NULL (rule
 * off).  d_out may alias d_pp. */
hdof_status hdof_composite(hdof_ctx* ctx, const float* d_color, const float* d_pp,
                           const float* d_depth, const uint8_t* d_spp, hdof_rt_bufs rt,
                           const hdof_camera* cam, const hdof_lens* lens,
                           const hdof_composite_params* params, const float* d_pp_spec, float* d_out,
                           hdof_stream stream);

/* Whole frame: G-buffer -> mask (reprojecting the history when prev != NULL)
 * -> trace -> variance update -> temporal reconstruction of the traced
 * colours (when params->recon.enable; its history is read when prev !=
 * NULL) -> spatial reconstruction (when params->spatial.enable; accumulated
 * hit ratio from the temporal history when that runs, variance estimate from
 * the variance history just updated) -> post-process -> composite.
 * d_out [3][H][W].  `keep` (nullable) supplies caller buffers for
 * intermediates (keep->rt receives the reconstructed colours when
 * reconstruction is on).  The batched form refuses both reconstructions.
 * Under stream capture (a HIP graph), once an eager frame of the same size
 * has reserved the scratch, a frame records kernels and events only; it
 * then refuses prev != NULL and both reconstructions (HDOF_ERR_UNSUPPORTED:
 * their histories advance on the host, which a replay would not see), and
 * it neither reads nor writes the variance history (a replay leaves the
 * history of the last eager frame as it was). */
hdof_status hdof_frame(hdof_ctx* ctx, const hdof_scene* scene, const hdof_camera* cam,
                       const hdof_camera* prev, const hdof_lens* lens, const hdof_light* light,
                       const hdof_frame_params* params, uint32_t seed, uint32_t frame,
                       uint32_t view, float* d_out, const hdof_frame_bufs* keep,
                       hdof_stream stream);

/* ---------------------------------------------------------------------- */
/* Batched form: many views (uneven sizes and lenses) in one frame          */
/* ---------------------------------------------------------------------- */

#define HDOF_MAX_VIEWS 64

/* One view of a batch: its camera and lens, the random-number key and the
 * view index that enters the lens-sample counter (so view v of a batch
 * equals a plain hdof_frame with the same seed, frame and view), and its
 * caller-owned output [3][H][W]. */
typedef struct {
  hdof_camera cam;
  hdof_lens lens;
  uint32_t seed, frame, view;
  float* d_out;
} hdof_view;

/* The batched form rejects params->recon.enable = 1 and
 * params->spatial.enable = 1 (HDOF_ERR_UNSUPPORTED): a reconstruction
 * history belongs to one view's camera path, and the spatial stage is not
 * batched; it takes the disk aperture only (blades = 0, sa = 0) and no
 * specular rule.
 * With 16-pixel post-filter tiles and the tuning's overlap on (the
 * defaults): the views' G-buffers in two launches (two chunks of about
 * equal pixels), each followed by ONE gather launch over its views' tiles
 * on the context's second stream (with the untraced pixels' composite);
 * meanwhile ONE launch per mask pass over every view (fixed mask tiles; the
 * CoC-scaled tile runs per view), one device-side scan of the per-view ray
 * totals, ONE queue fill, ONE persistent thin-lens trace launch and ONE
 * reduction for the whole batch; after both, ONE composite launch over
 * every view's traced pixels.  Otherwise a G-buffer, mask and post-filter
 * with composite per view around the same single trace.  No variance
 * history (each view is a first frame).  1 <= n_views <= HDOF_MAX_VIEWS;
 * all views share the scene, light and parameters. */
hdof_status hdof_frame_batched(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                               const hdof_frame_params* params, int32_t n_views,
                               const hdof_view* views, hdof_stream stream);

/* The same batch captured once into a HIP graph (all scratch reserved at
 * creation) and replayed by hdof_batch_launch.  The graph keeps the views,
 * output pointers and tuning of creation time; the scene and context must
 * outlive the batch, and one context's batches and frames must not run
 * concurrently (they share its scratch). */
typedef struct hdof_batch hdof_batch;
hdof_status hdof_batch_create(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                              const hdof_frame_params* params, int32_t n_views,
                              const hdof_view* views, hdof_batch** out);
hdof_status hdof_batch_launch(hdof_batch* batch, hdof_stream stream);
/* Synchronises the device, then frees the graph.  NULL is a no-op. */
void hdof_batch_destroy(hdof_batch* batch);

/* Launch shape of the persistent thin-lens trace (performance only: results
 * do not depend on it).  blocks_per_cu in [1, 32]; refill in [1, 64]: idle
 * lanes of a wave that trigger a refill from the queue (64 = batches of 64
 * rays); segments in [1, 8]: queue segments, one per XCD group; wave 0, 1
 * or 2: 1 walks the 64 rays of a batch of consecutive queue entries as one
 * wave (one node sequence, the union of their paths, with wave-uniform node
 * loads; refill is then unused), 0 traverses each lane's ray on its own and
 * refills idle lanes, 2 takes 1 for scenes of at least HDOF_WAVE_AUTO_TRIS
 * triangles and 0 below (the per-lane form is the faster one on the 200k-
 * and the 1M-triangle scenes measured; the wave form remains for callers
 * and the autotuner to try); overlap 0
 * or 1: 1 runs hdof_frame's post-filter gather on a second stream of the
 * context beside the mask, trace and reconstruction (it needs only the
 * G-buffer) and applies the composite once both are done, the results
 * being the same as with 0; overlap_ray_quantum >= 1: while overlapped, the
 * trace keeps, on average, one block per CU for every overlap_ray_quantum
 * rays of the frame (at least one per CU, at most blocks_per_cu; the count
 * is read on the device, the other blocks return at once), so a light
 * trace leaves CUs to the gather and a heavy one keeps them.  Defaults {10, 64, 8, 0, 1,
 * 140000}: ten two-wave blocks per CU (more are slower: the trace is bound
 * by its per-CU cache working set and latency, not by resident waves). */
#define HDOF_WAVE_AUTO_TRIS (1 << 19)
typedef struct {
  int32_t blocks_per_cu, refill, segments, wave, overlap, overlap_ray_quantum;
} hdof_tuning;
hdof_status hdof_set_tuning(hdof_ctx* ctx, const hdof_tuning* tuning);
hdof_status hdof_get_tuning(hdof_ctx* ctx, hdof_tuning* tuning);

/* The library's autotuner of the launch shape (not in the paper: its tile
 * and queue sizes are scheduling choices of this implementation).  It times
 * the caller's workload -- hdof_frame on views[0] when n_views = 1,
 * hdof_frame_batched on all views otherwise -- on `stream` under candidate
 * tunings (coordinate descent from the defaults over blocks_per_cu,
 * refill, segments, wave, and for single frames overlap and
 * overlap_ray_quantum; a change is kept when it is at least 0.5 % faster;
 * each candidate is the median of several timed runs), sets the fastest on
 * the context and returns it in *out.  The workload's outputs
 * (views[v].d_out) are written.  prev (nullable, single frames only): every
 * timed frame is hdof_frame(views[0].cam, prev), so it carries the
 * variance history of the frame before it, as frames along a camera path
 * do (the mask then also traces the pixels whose luminance varies); NULL:
 * every timed frame is a first frame.  Either way the context's variance
 * history is replaced.  cache_path (nullable): a JSON-lines file, one
 * object per workload class keyed by the device's architecture, its CU
 * count and the class (image sizes, spp_max, tiles, the scene's triangle
 * count as a power of two, view count, optional stages, history); an entry
 * for the class is applied without timing unless force != 0, and a search
 * writes (or replaces) its entry.  A search that fails (a candidate's
 * frame returns an error) leaves the context's tuning as it was on entry
 * and writes no cache entry.  Not under stream capture
 * (HDOF_ERR_UNSUPPORTED); not thread-safe per context or per cache file. */
typedef struct {
  char key[256];        /* the workload class */
  float best_ms;        /* per run of the workload under the chosen tuning */
  float default_ms;     /* per run under the defaults (as cached, for cache hits) */
  int32_t candidates;   /* tunings timed (0: taken from the cache) */
  int32_t from_cache;
} hdof_autotune_report;
hdof_status hdof_autotune(hdof_ctx* ctx, const hdof_scene* scene, const hdof_light* light,
                          const hdof_frame_params* params, int32_t n_views, const hdof_view* views,
                          const hdof_camera* prev, const char* cache_path, int32_t force, hdof_tuning* out,
                          hdof_autotune_report* report, hdof_stream stream);

/* ---------------------------------------------------------------------- */
/* Differentiable form                                                      */
/* ---------------------------------------------------------------------- */

/* Adjoint of hdof_postfilter followed by hdof_composite, as a function of the
 * sharp colour C_r, the focus distance S1 and the aperture A, with depth,
 * ray counts and ray-traced colours held fixed.  Given dL/dout
 * (d_grad_out [3][H][W]) it writes dL/dC_r (d_grad_color [3][H][W]; the
 * post-filter's transpose is scattered with float atomics, so its low bits
 * depend on their order) and {dL/dS1, dL/dA} (d_grad_lens, 2 device floats,
 * summed in a fixed order).  The gather is recomputed, no weights are
 * stored.  Derivatives: dc/dS1 = -A s_px / S1^2, dc/dA = (1/S1 - 1/z) s_px;
 * the gather radius follows the CoC of the pixel that sets its tile maximum
 * (lowest index on ties) unless capped at r_cap; clamp ramps have slope 0 at
 * and beyond their ends.  d_grad_color must not alias the inputs. */
hdof_status hdof_postfilter_composite_backward(hdof_ctx* ctx, const float* d_color, const float* d_depth,
                                               const uint8_t* d_spp, hdof_rt_bufs rt,
                                               const hdof_camera* cam, const hdof_lens* lens,
                                               const hdof_pp_params* pp, const hdof_composite_params* comp,
                                               const float* d_grad_out, float* d_grad_color,
                                               float* d_grad_lens, hdof_stream stream);

/* ---------------------------------------------------------------------- */
/* Stage timing                                                             */
/* ---------------------------------------------------------------------- */

/* Stages hdof_frame brackets with HIP events while profiling is on, in
 * order: G-buffer, ray mask, queue build, thin-lens trace kernel, per-pixel
 * reduction, variance update, temporal and spatial reconstruction (0 when
 * both are disabled),
 * post-filter preparation (pack, tile radius, taps), post-filter gather,
 * composite.  With the overlapped frame (tuning overlap = 1) the
 * gather is timed on its own stream from its start to its end, while the
 * preparation stage runs from the end of the reconstruction to the start
 * of the composite (the specular gather, then the wait for the post-filter
 * gather), so the stages then add up to more than the frame. */
#define HDOF_PROFILE_STAGES 10

/* Start recording stage events in every following hdof_frame call (events
 * are recorded on the frame's stream; the host is not synchronised). */
hdof_status hdof_profile_begin(hdof_ctx* ctx);
/* Synchronise, stop recording and return the mean duration in milliseconds
 * of each stage over the recorded frames (ms_out[HDOF_PROFILE_STAGES]) and
 * the number of frames (*n_frames, may be NULL). */
hdof_status hdof_profile_end(hdof_ctx* ctx, float* ms_out, int32_t* n_frames);

/* Traversal work counters.  Between begin and end, hdof_gbuffer,
 * hdof_trace_thin_lens and hdof_frame run variants of their traversal
 * kernels that count, per ray, the BVH nodes entered and the triangles
 * tested (slower; for measurement only).  end synchronises and writes
 * out[6] = {G-buffer rays, node visits, triangle tests, thin-lens rays,
 * node visits, triangle tests}. */
hdof_status hdof_counters_begin(hdof_ctx* ctx);
hdof_status hdof_counters_end(hdof_ctx* ctx, int64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* HDOF_H */
