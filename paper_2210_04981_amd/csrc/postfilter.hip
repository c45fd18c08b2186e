// postfilter.hip -- post-process gather DoF filter and the composite.
//
// k_pp_pack: colour + signed CoC packed into one float4 per pixel (one
//   16-byte load per bilinear texel in the gather) and the per-tile maximum
//   CoC radius.
// k_pp_dilate: gather radius per tile = min(r_cap, max radius over the tiles
//   within ceil(r_cap / tile) tiles).
// k_pp_gather16q / k_pp_gather16 / k_pp_gather_any: golden-angle taps,
//   bilinear float4 texels, weights recomputed per tap, nothing stored but
//   the result.  16-pixel tiles stage each tap's footprint in LDS: one wave
//   per tile gathering 2x2 pixel quads (k_pp_gather16q), or, beside the
//   trace in the overlapped frame, four waves per tile (k_pp_gather16).
// k_composite: focus zone / near / far rules, one pass over the pixels.
#include "hdof_internal.h"

#include <hip/hip_ext.h>

#include <mutex>

namespace {

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__global__ __launch_bounds__(256) void k_pp_pack(const float* __restrict__ color,
                                                 const float* __restrict__ depth, CamK k, LensK l,
                                                 int tile, float4* __restrict__ pack,
                                                 float* __restrict__ tile_r) {
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const int BX = (k.W + 15) >> 4, lb = xcd_block(blockIdx.x, BX * ((k.H + 15) >> 4));
  const int x = (lb % BX) * 16 + (tid & 15), y = (lb / BX) * 16 + (tid >> 4);
  const size_t N = (size_t)k.W * k.H;
  float r = 0.0f;
  if (x < k.W && y < k.H) {
    size_t p = (size_t)y * k.W + x;
    float c = coc_px(l, depth[p]);
    pack[p] = make_float4(color[p], color[N + p], color[2 * N + p], c);
    r = 0.5f * fabsf(c);
  }
  red[tid] = r;
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;
  if ((tx % tile) == 0 && (ty % tile) == 0 && x < k.W && y < k.H) {
    float m = 0.0f;
    for (int dy = 0; dy < tile; ++dy)
      for (int dx = 0; dx < tile; ++dx) m = fmaxf(m, red[(ty + dy) * 16 + tx + dx]);
    const int TW = (k.W + tile - 1) / tile;
    tile_r[(y / tile) * TW + x / tile] = m;
  }
}

// golden-angle taps u_k = sqrt((k - 0.5)/n) (cos k g, sin k g), g = pi (3 - sqrt 5),
// evaluated in double and stored as (ux, uy, |u|, omega).  A polygonal
// aperture (blades >= 3, first vertex at rot radians) moves each tap
// radially onto the polygon, u' = u P(angle), P its boundary radius at
// circumradius 1, keeping |u| (the tap's gauge distance in the polygonal
// CoC); omega = max(0, 1 + sa (2 |u'|^2 - 1)) is the tap's aberration weight.
__global__ void k_pp_taps(int n, int blades, double rot, float sa, float4* __restrict__ taps) {
  int k = threadIdx.x + 1;
  if (k > n) {  // the table's unused entries are zero (gathers read whole groups of taps)
    taps[k - 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const double pi = 3.14159265358979323846;
  const double g = pi * (3.0 - sqrt(5.0));
  double rr = sqrt((k - 0.5) / n);
  double sc = 1.0;
  if (blades >= 3) {
    const double sector = 2.0 * pi / blades;
    double a = fmod(k * g - rot, sector);
    if (a < 0.0) a += sector;
    sc = cos(pi / blades) / cos(a - pi / blades);
  }
  const double r2 = rr * sc;
  const double om = fmax(0.0, 1.0 + (double)sa * (2.0 * r2 * r2 - 1.0));
  taps[k - 1] = make_float4((float)(r2 * cos(k * g)), (float)(r2 * sin(k * g)), (float)rr, (float)om);
}

// (re)build the context's tap table when the tap count or the aperture changed
void pp_taps_ensure(hdof_ctx* ctx, int n, const LensK& l, hipStream_t st) {
  const int blades = l.blades >= 3 ? l.blades : 0;
  if (ctx->pp_taps_n == n && ctx->pp_taps_blades == blades && ctx->pp_taps_rot == l.rot_ht &&
      ctx->pp_taps_sa == l.sa)
    return;
  hipLaunchKernelGGL(k_pp_taps, dim3(1), dim3(256), 0, st, n, blades, (double)l.rot_ht * 3.14159265358979323846,
                     l.sa, (float4*)ctx->pp_taps.p);
  ctx->pp_taps_n = n;
  ctx->pp_taps_blades = blades;
  ctx->pp_taps_rot = l.rot_ht;
  ctx->pp_taps_sa = l.sa;
}

__global__ void k_pp_dilate(const float* __restrict__ tile_r, int TW, int TH, int K, float r_cap,
                            float* __restrict__ rad) {
  int tx = blockIdx.x * blockDim.x + threadIdx.x, ty = blockIdx.y;
  if (tx >= TW) return;
  float m = 0.0f;
  for (int dy = -K; dy <= K; ++dy) {
    int yy = ty + dy;
    if (yy < 0 || yy >= TH) continue;
    for (int dx = -K; dx <= K; ++dx) {
      int xx = tx + dx;
      if (xx < 0 || xx >= TW) continue;
      m = fmaxf(m, tile_r[yy * TW + xx]);
    }
  }
  rad[ty * TW + tx] = fminf(r_cap, m);
}


// ---------------------------------------------------------------- gather
// Tap weights are carried in CoC-diameter units: for a tap with bilinear CoC
// c_q, the paper's weight (R^2/N) a / max(r_q, 0.5)^2 equals
// 4 (R^2/N) a / max(c_q^2, 1), so every tap uses a / max(c_q^2, 1) and the
// centre weight 1 / max(r_p, 0.5)^2 becomes 1 / ((R^2/N) max(c_p^2, 1)); the
// normalised sum is unchanged.  The effective radius in the same units is
// |c_q| - t max(0, |c_q| - |c_p|) (twice the radius form).
struct GatherAcc {
  float ap, ncpr, inv_ramp;  // |c_p|, -c_p / ramp, 1 / ramp
  float ar, ag, ab, ws;
  // (no implicit contraction of a product into a sum here or in tap(): the
  // gather's forms inline these into different code and must round alike)
  __device__ __forceinline__ void init(const float4& cp4, float R, int n_taps, float inv_ramp_) {
#pragma clang fp contract(off)
    inv_ramp = inv_ramp_;
    ap = fabsf(cp4.w);
    ncpr = -cp4.w * inv_ramp;
    const float q = fmaxf(cp4.w * cp4.w, 1.0f);
    const float w0 = R > 0.0f ? __builtin_amdgcn_rcpf(R * R / (float)n_taps * q) : 1.0f;
    ar = w0 * cp4.x;
    ag = w0 * cp4.y;
    ab = w0 * cp4.z;
    ws = w0;
  }
  // one tap: bilinear (rgb, c) from the four texels with weights
  // (w00, w10, w01, w11), d = 0.5 - R |u|
  // om: the tap's aberration weight (1: the disk's uniform weights)
  __device__ __forceinline__ void tap(float w00, float w10, float w01, float w11, float d, const float4& v00,
                                      const float4& v10, const float4& v01, const float4& v11, float om = 1.0f) {
#pragma clang fp contract(off)
    const float sr = fmaf(w11, v11.x, fmaf(w01, v01.x, fmaf(w10, v10.x, w00 * v00.x)));
    const float sg = fmaf(w11, v11.y, fmaf(w01, v01.y, fmaf(w10, v10.y, w00 * v00.y)));
    const float sb = fmaf(w11, v11.z, fmaf(w01, v01.z, fmaf(w10, v10.z, w00 * v00.z)));
    const float cq = fmaf(w11, v11.w, fmaf(w01, v01.w, fmaf(w10, v10.w, w00 * v00.w)));
    const float aq = fabsf(cq);
    const float tk = clamp01(fmaf(cq, inv_ramp, ncpr));
    const float reff2 = fmaf(-tk, fmaxf(0.0f, aq - ap), aq);
    const float a = clamp01(fmaf(reff2, 0.5f, d)) * om;
    const float wt = a * __builtin_amdgcn_rcpf(fmaxf(cq * cq, 1.0f));
    ar = fmaf(wt, sr, ar);
    ag = fmaf(wt, sg, ag);
    ab = fmaf(wt, sb, ab);
    ws += wt;
  }
  __device__ __forceinline__ void store(float* __restrict__ out, size_t N, size_t p) const {
    const float iw = 1.0f / ws;
    out[p] = ar * iw;
    out[N + p] = ag * iw;
    out[2 * N + p] = ab * iw;
  }
};

// Four clamp-to-edge texels of the bilinear footprint whose corner is (xa, ya).
__device__ __forceinline__ void texels_clamped(const float4* __restrict__ pack, int W, int H, int xa, int ya,
                                               float4& v00, float4& v10, float4& v01, float4& v11) {
  const int xa_ = clampi(xa, 0, W - 1), xb_ = clampi(xa + 1, 0, W - 1);
  const int ya_ = clampi(ya, 0, H - 1), yb_ = clampi(ya + 1, 0, H - 1);
  v00 = pack[(size_t)ya_ * W + xa_];
  v10 = pack[(size_t)ya_ * W + xb_];
  v01 = pack[(size_t)yb_ * W + xa_];
  v11 = pack[(size_t)yb_ * W + xb_];
}

// Tap record of the 16-pixel-tile gather: bilinear weights.
struct TapRec {
  float w00, w10, w01, w11;
};

#define PPG_G 4                 // taps per staged group (one per wave)
#define PPG_SIDE 17             // footprint side: 16 pixels + 1 bilinear neighbour
#define PPG_TEX (PPG_SIDE * PPG_SIDE)
#define PPG_SLOTS 5             // ceil(PPG_TEX / 64) texels staged per lane
#ifndef PPG_STRIDE
#define PPG_STRIDE 17           // LDS row stride of a staged footprint, in texels
#endif
#define PPG_TAPSZ (PPG_SIDE * PPG_STRIDE)
#ifndef PPG_BUFS
#define PPG_BUFS 2              // LDS ring: 2 = double-buffered groups, 1 = one group and a second barrier
#endif

// 16-pixel tiles: one 16x16 block per tile, blocks in XCD-contiguous order;
// the gather radius R and with it every tap's footprint offset and bilinear
// weights are uniform over the block.  For one tap the block's 256 pixels
// read the 17x17 texels at the tap's offset, each four times.  Taps are
// processed in groups of four: wave w stages tap w of the next group (its
// 17x17 clamp-to-edge texels, five 16-byte loads per lane, and the tap
// record) into one half of a double-buffered LDS ring while the block
// gathers the current group from the other half, so the vector-memory
// address unit (16 clocks per 64-lane load) handles 5 loads per wave and
// group instead of 16.
struct Stage {
  float4 v0, v1, v2, v3, v4;  // texels s * 64 + lane of the footprint, s = 0..4
  TapRec tr;
};

// Lane constants of the staging: footprint texel idx = s * 64 + lane lies at
// row idx / 17, column idx % 17 (lanes past the 289th texel repeat texel
// 256 + lane - 64 and do not store it); interior blocks address texels by a
// 32-bit byte offset from the footprint corner.
struct StageLane {
  int sr[PPG_SLOTS], sc[PPG_SLOTS];
  unsigned so[PPG_SLOTS];
  int lo[PPG_SLOTS];  // LDS texel index within the tap's footprint
  bool last;          // slot 4 holds a footprint texel of its own
};

// word 3 of a raw buffer resource on gfx9 (32-bit data format, no swizzle)
#define HDOF_BUFFER_WORD3 0x00020000

__device__ __forceinline__ float4 buffer_texel(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, soff, 0);
  float4 f;
  __builtin_memcpy(&f, &v, sizeof f);
  return f;
}

// Texels and record of the tap with table entry u (wave-uniform) for the
// block at (x0, y0).
template <bool INTERIOR>
__device__ __forceinline__ Stage stage_load(const float4* __restrict__ pack, const float4 u, float R, int x0,
                                            int y0, int W, int H, const StageLane& sl) {
#pragma clang fp contract(off)
  Stage st;
  const float ox = R * u.x, oy = R * u.y;
  const float fx = floorf(ox), fy = floorf(oy);
  const float ax = ox - fx, ay = oy - fy, bx = 1.0f - ax, by = 1.0f - ay;
  st.tr.w00 = bx * by;
  st.tr.w10 = ax * by;
  st.tr.w01 = bx * ay;
  st.tr.w11 = ax * ay;
  const int gx0 = x0 + __builtin_amdgcn_readfirstlane((int)fx);
  const int gy0 = y0 + __builtin_amdgcn_readfirstlane((int)fy);
  if (INTERIOR) {
    // buffer loads: the footprint corner's byte offset as the scalar
    // offset, each lane's texel offset as the vector one (no per-lane 64-bit
    // address arithmetic; the resource spans the image, which interior
    // blocks require to be under 2 GiB)
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float4*>(pack), (short)0, W * H * 16, HDOF_BUFFER_WORD3);
    const int corner = __builtin_amdgcn_readfirstlane((gy0 * W + gx0) * 16);
    st.v0 = buffer_texel(rs, sl.so[0], corner);
    st.v1 = buffer_texel(rs, sl.so[1], corner);
    st.v2 = buffer_texel(rs, sl.so[2], corner);
    st.v3 = buffer_texel(rs, sl.so[3], corner);
    st.v4 = buffer_texel(rs, sl.so[4], corner);
  } else {
#define PPG_CLAMPED(s) pack[(size_t)clampi(gy0 + sl.sr[s], 0, H - 1) * W + clampi(gx0 + sl.sc[s], 0, W - 1)]
    st.v0 = PPG_CLAMPED(0);
    st.v1 = PPG_CLAMPED(1);
    st.v2 = PPG_CLAMPED(2);
    st.v3 = PPG_CLAMPED(3);
    st.v4 = PPG_CLAMPED(4);
#undef PPG_CLAMPED
  }
  return st;
}

__device__ __forceinline__ void stage_store_texels(float4* __restrict__ dst, const Stage& st, const StageLane& sl) {
  dst[sl.lo[0]] = st.v0;
  dst[sl.lo[1]] = st.v1;
  dst[sl.lo[2]] = st.v2;
  dst[sl.lo[3]] = st.v3;
  if (sl.last) dst[sl.lo[4]] = st.v4;
}

__device__ __forceinline__ void stage_store(float4* __restrict__ dst, TapRec* __restrict__ rdst, const Stage& st,
                                            const StageLane& sl, int lane) {
  stage_store_texels(dst, st, sl);
  if (lane == 0) *rdst = st.tr;
}

// The tap loop of one block.  Groups are always full: a wave whose tap of
// the group lies past n_taps stages the table's zero entry (the footprint
// at the block's corner), and that slot's distance term is -1e30 so its
// coverage, and with it its weight, is 0.
template <bool INTERIOR, bool SA>
__device__ __forceinline__ void gather_taps(float4 (*stg)[PPG_G * PPG_TAPSZ], TapRec (*rec)[PPG_G],
                                            const float4* __restrict__ pack, const float4* __restrict__ taps,
                                            int n_taps, float R, int x0, int y0, int W, int H, int wave, int lane,
                                            int lofs, bool inside, GatherAcc& g) {
  StageLane sl;
#pragma unroll
  for (int s = 0; s < PPG_SLOTS; ++s) {
    const int idx = s * 64 + lane < PPG_TEX ? s * 64 + lane : s * 64 + lane - 64;
    sl.sr[s] = idx / PPG_SIDE;
    sl.sc[s] = idx - sl.sr[s] * PPG_SIDE;
    sl.so[s] = (unsigned)(sl.sr[s] * W + sl.sc[s]) * 16u;
    sl.lo[s] = sl.sr[s] * PPG_STRIDE + sl.sc[s];
  }
  sl.last = lane < PPG_TEX - 4 * 64;
  const int ng = (n_taps + PPG_G - 1) / PPG_G;
  // The table entries of a group (four taps, 64 contiguous bytes of the
  // 256-entry table whose unused entries are zero) are read together right
  // after the group's barrier: the staging wave takes its own tap's offset
  // from them, the gather the taps' radii |u| and weights.  A scalar load's
  // wait also drains the LDS reads in flight, so no table read is left
  // inside the tap loop.
  // (four named values, and the wave's own entry read by its own scalar
  // load: an indexed array of them would live in scratch memory, and value
  // selects among them cost 14 vector instructions per group)
  float4 c0 = taps[0], c1 = taps[1], c2 = taps[2], c3 = taps[3];
  {
    const Stage st = stage_load<INTERIOR>(pack, taps[wave], R, x0, y0, W, H, sl);
    stage_store(stg[0] + wave * PPG_TAPSZ, &rec[0][wave], st, sl, lane);
  }
  for (int gi = 0; gi < ng; ++gi) {
    __syncthreads();
    const int b = PPG_BUFS == 2 ? gi & 1 : 0;
    const bool more = gi + 1 < ng;
    Stage st;
    float4 n0, n1, n2, n3;
    if (more) {
      const float4* tg = taps + (gi + 1) * PPG_G;
      n0 = tg[0];
      n1 = tg[1];
      n2 = tg[2];
      n3 = tg[3];
      st = stage_load<INTERIOR>(pack, tg[wave], R, x0, y0, W, H, sl);
    }
    if (inside) {
      const float4* src = stg[b] + lofs;
      const float uz[PPG_G] = {c0.z, c1.z, c2.z, c3.z}, uw[PPG_G] = {c0.w, c1.w, c2.w, c3.w};
#pragma unroll
      for (int jj = 0; jj < PPG_G; ++jj) {
        const bool valid = gi * PPG_G + jj < n_taps;
        const float d = valid ? fmaf(-R, uz[jj], 0.5f) : -1e30f;
        const float om = SA && valid ? uw[jj] : 1.0f;
        const float4* a = src + jj * PPG_TAPSZ;
        const TapRec t = rec[b][jj];
        g.tap(t.w00, t.w10, t.w01, t.w11, d, a[0], a[1], a[PPG_STRIDE], a[PPG_STRIDE + 1], om);
      }
    }
    if (more) {
      if (PPG_BUFS == 1) __syncthreads();  // every wave has read the group the next one overwrites
      stage_store(stg[PPG_BUFS == 2 ? b ^ 1 : 0] + wave * PPG_TAPSZ, &rec[PPG_BUFS == 2 ? b ^ 1 : 0][wave], st, sl,
                  lane);
      c0 = n0;
      c1 = n1;
      c2 = n2;
      c3 = n3;
    }
  }
}

// Composite applied in the gather's epilogue (whole frames): the same rules
// as k_composite, with the raster colour and CoC from the packed texel.
struct FuseK {
  const uint8_t* spp;
  const float *cn, *cf, *hr;
  float inv_ht;
  int rt_override;
  float* out;
  const float* pps;  // nullable: post-filtered specular luminance
  float inv_sy;      // 1 / spec_y, 0: no specular bokeh rule
};

// The composite's blend of one channel (paper, Composite): the traced
// colour crt = h C_tn + (1 - h) C_tf, the near rule nu, the focus-zone
// weight phi, the far blend beta and the specular weight sig.  Every
// product that meets a sum is an explicit fmaf, so the fused gather
// epilogue and the separate composite kernel round alike.
__device__ __forceinline__ float traced_mix(float h, float cn, float cf) { return fmaf(h, cn, (1.0f - h) * cf); }

__device__ __forceinline__ float composite_mix(float col, float cpp, float crt, float phi, float nu, float rho,
                                               float beta, float sig) {
  const float cnear = fmaf(sig, cpp - crt, crt);
  const float v_near = fmaf(rho, cnear, (1.0f - rho) * cpp);
  const float v_far = fmaf(beta, crt, (1.0f - beta) * cpp);
  const float oof = fmaf(nu, v_near, (1.0f - nu) * v_far);
  return fmaf(phi, oof, (1.0f - phi) * col);
}

// UNTRACED: every pixel takes the untraced pixels' rule (spp, the traced
// colours and pps are not read).
template <bool UNTRACED>
__device__ __forceinline__ void composite_px(const FuseK& fz, size_t N, size_t p, const float4& cp4, float pr,
                                             float pg, float pb) {
  const float c = cp4.w;
  const float phi = clamp01(fabsf(c) - HDOF_SQRT2);
  const float nu = clamp01(fmaf(-c, 0.35355339059327376f, 0.5f));
  const bool traced = !UNTRACED && fz.spp[p] > 0;
  const float h = traced ? fz.hr[p] : 0.0f;
  const float rho = traced ? 1.0f : 0.0f;
  const float beta = traced ? clamp01(1.0f - h * fz.inv_ht) : 0.0f;
  const float sig = (fz.pps && traced && fz.inv_sy > 0.0f) ? clamp01(fz.pps[p] * fz.inv_sy) : 0.0f;
  const float col[3] = {cp4.x, cp4.y, cp4.z}, cpp[3] = {pr, pg, pb};
  for (int q = 0; q < 3; ++q) {
    const size_t i = (size_t)q * N + p;
    const float crt = traced ? traced_mix(h, fz.cn[i], fz.cf[i]) : 0.0f;
    float o = composite_mix(col[q], cpp[q], crt, phi, nu, rho, beta, sig);
    if (fz.rt_override && traced) o = crt;
    fz.out[i] = o;
  }
}

// the filtered colour of pixel p: to `out` (may be NULL when fused) and,
// FUSE 1, through the composite, or FUSE 2, through the untraced pixels'
// rule of the composite
template <int FUSE>
__device__ __forceinline__ void pp_emit(float* __restrict__ out, const FuseK& fz, size_t N, size_t p,
                                        const float4& cp4, float pr, float pg, float pb) {
  if (out) {
    out[p] = pr;
    out[N + p] = pg;
    out[2 * N + p] = pb;
  }
  if (FUSE == 1) composite_px<false>(fz, N, p, cp4, pr, pg, pb);
  if (FUSE == 2) composite_px<true>(fz, N, p, cp4, pr, pg, pb);
}

// The gather radius of tile (tx, ty): min(r_cap, max tile radius within K
// tiles), reduced by the block (uniform result).
__device__ __forceinline__ float block_dilated_radius(const float* __restrict__ tile_r, int TW, int TH, int tx,
                                                      int ty, int K, float r_cap, float* wred) {
  const int D = 2 * K + 1, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float m = 0.0f;
  for (int i = tid; i < D * D; i += 256) {
    const int yy = ty - K + i / D, xx = tx - K + i % D;
    if (yy >= 0 && yy < TH && xx >= 0 && xx < TW) m = fmaxf(m, tile_r[yy * TW + xx]);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) wred[wave] = m;
  __syncthreads();
  return fminf(r_cap, fmaxf(fmaxf(wred[0], wred[1]), fmaxf(wred[2], wred[3])));
}

// 16-pixel tiles.  The block first reduces its tile's dilated radius from
// the per-tile maxima; FUSE 1 applies the composite to the result, FUSE 2
// the composite's rule for untraced pixels (the traced ones are rewritten
// later); SA weights the taps by the lens's spherical aberration (the
// table's fourth entry).
template <int FUSE, bool SA>
__device__ __forceinline__ void gather16_tile(float4 (*stg)[PPG_G * PPG_TAPSZ], TapRec (*rec)[PPG_G], float* wred,
                                              const float4* __restrict__ pack, const float* __restrict__ tile_r,
                                              int K, float r_cap, const float4* __restrict__ taps, int n_taps, int W,
                                              int H, float inv_ramp, float* __restrict__ out, const FuseK& fz,
                                              int tile) {
  const int TW = (W + 15) >> 4, TH = (H + 15) >> 4;
  const int x0 = (tile % TW) * 16, y0 = (tile / TW) * 16;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lx = lane & 15, ly = wave * 4 + (lane >> 4);
  const int x = x0 + lx, y = y0 + ly;
  const bool inside = x < W && y < H;
  const size_t N = (size_t)W * H, p = (size_t)y * W + x;
  const float R = block_dilated_radius(tile_r, TW, TH, tile % TW, tile / TW, K, r_cap, wred);
  if (!(R > 0.0f)) {
    if (inside) {
      const float4 c = pack[p];
      pp_emit<FUSE>(out, fz, N, p, c, c.x, c.y, c.z);
    }
    return;
  }
  const int E = (int)ceilf(R);
  const bool interior = x0 - E - 1 >= 0 && x0 + 16 + E < W && y0 - E - 1 >= 0 && y0 + 16 + E < H &&
                        (long long)W * H * 16 < (1ll << 31);
  const float4 cp4 = inside ? pack[p] : make_float4(0.f, 0.f, 0.f, 0.f);
  GatherAcc g;
  g.init(cp4, R, n_taps, inv_ramp);
  const int lofs = ly * PPG_STRIDE + lx;
  if (interior)
    gather_taps<true, SA>(stg, rec, pack, taps, n_taps, R, x0, y0, W, H, wave, lane, lofs, inside, g);
  else
    gather_taps<false, SA>(stg, rec, pack, taps, n_taps, R, x0, y0, W, H, wave, lane, lofs, inside, g);
  if (inside) {
    const float iw = 1.0f / g.ws;
    pp_emit<FUSE>(out, fz, N, p, cp4, g.ar * iw, g.ag * iw, g.ab * iw);
  }
}

// The tile at position L of an order that walks the tile grid in eight
// rectangles (4 across, 2 down), each row by row.  An XCD's contiguous
// share of positions (xcd_block) then covers about one rectangle, whose
// footprints (up to R_cap + 1 pixels around it) stay in that XCD's L2,
// instead of a full-width band of tile rows whose footprint rows exceed it
// (the quad form: 77.3 -> 49.2 MB fetched per 1080p launch, 151 -> 147 us).
__device__ __forceinline__ int rect_tile(int L, int TW, int TH) {
  int base = 0;
  for (int ry = 0; ry < 2; ++ry) {
    const int y0 = TH * ry / 2, y1 = TH * (ry + 1) / 2;
    for (int rx = 0; rx < 4; ++rx) {
      const int x0 = TW * rx / 4, x1 = TW * (rx + 1) / 4;
      const int n = (x1 - x0) * (y1 - y0);
      if (L < base + n) {
        const int o = L - base, w = x1 - x0;
        return (y0 + o / w) * TW + x0 + o % w;
      }
      base += n;
    }
  }
  return L;  // not reached for L < TW * TH
}

template <int FUSE, bool SA>
__global__ __launch_bounds__(256) void k_pp_gather16(const float4* __restrict__ pack, const float* __restrict__ tile_r,
                                                     int K, float r_cap, const float4* __restrict__ taps, int n_taps,
                                                     int W, int H, float inv_ramp, float* __restrict__ out, FuseK fz) {
  __shared__ float4 stg[PPG_BUFS][PPG_G * PPG_TAPSZ];
  __shared__ TapRec rec[PPG_BUFS][PPG_G];
  __shared__ float wred[4];
  // band order (an XCD's share is a band of tile rows): the rectangle
  // order cut this form's fetches from 57.9 to 41.4 MB but made the
  // overlapped frame slower (0.3923 against 0.3896 ms)
  const int tile = xcd_block(blockIdx.x, ((W + 15) >> 4) * ((H + 15) >> 4));
  gather16_tile<FUSE, SA>(stg, rec, wred, pack, tile_r, K, r_cap, taps, n_taps, W, H, inv_ramp, out, fz, tile);
}

// The batched form's gathers (the quad form) and traced pixels'
// composites, one launch each over every view: a wave (gather) or block
// (composite) finds its view by a binary search over the views' first
// tiles or first pixel blocks; a view's planes start at its px_base and its
// tile radii at its first tile.  The quad form is the batch's: there the
// gather sets the pace (32 views replayed 10.05 ms against 10.68 with the
// four-wave form).
struct PPBatch {
  int n;
  int tile_base[HDOF_MAX_VIEWS + 1];  // [n]: all tiles
  int blk_base[HDOF_MAX_VIEWS + 1];   // [n]: all blocks of HDOF_BATCH_PX_BLOCK pixels
  float* out[HDOF_MAX_VIEWS];
};

// The gather radius of tile (tx, ty) reduced by one wave (uniform result).
__device__ __forceinline__ float wave_dilated_radius(const float* __restrict__ tile_r, int TW, int TH, int tx,
                                                     int ty, int K, float r_cap) {
  const int D = 2 * K + 1, lane = threadIdx.x & 63;
  float m = 0.0f;
  for (int i = lane; i < D * D; i += 64) {
    const int yy = ty - K + i / D, xx = tx - K + i % D;
    if (yy >= 0 && yy < TH && xx >= 0 && xx < TW) m = fmaxf(m, tile_r[yy * TW + xx]);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  return fminf(r_cap, m);
}

// Orders a wave's LDS stores before its later LDS loads (and its earlier
// loads before its later stores) across lanes: every LDS access in flight
// completes and the compiler moves none across.  No other wave takes part.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The tap loop of one wave whose lanes gather 2x2 pixel quads of one tile;
// per tap a lane reads the 3x3 staged texels its four bilinear footprints
// cover.  Software-pipelined over a two-buffer LDS ring: iteration t stores
// tap t + 1's texels (loaded during iteration t - 1, so a whole gather has
// covered their latency), issues tap t + 2's loads, and gathers tap t.
// Table entries are read two taps ahead; past the last tap the last one is
// staged again (unused), so nothing is carried on a conditional path.
template <bool INTERIOR, bool SA>
__device__ __forceinline__ void gather_taps_quad(float4 (*stg)[PPG_TAPSZ], const float4* __restrict__ pack,
                                                 const float4* __restrict__ taps, int n_taps, float R, int x0,
                                                 int y0, int W, int H, int lane, int lofs, GatherAcc (&g)[4]) {
  StageLane sl;
#pragma unroll
  for (int s = 0; s < PPG_SLOTS; ++s) {
    const int idx = s * 64 + lane < PPG_TEX ? s * 64 + lane : s * 64 + lane - 64;
    sl.sr[s] = idx / PPG_SIDE;
    sl.sc[s] = idx - sl.sr[s] * PPG_SIDE;
    sl.so[s] = (unsigned)(sl.sr[s] * W + sl.sc[s]) * 16u;
    sl.lo[s] = sl.sr[s] * PPG_STRIDE + sl.sc[s];
  }
  sl.last = lane < PPG_TEX - 4 * 64;
  const int last = n_taps - 1;
  const float4 e0 = taps[0];
  float4 e1 = taps[last < 1 ? last : 1], e2 = taps[last < 2 ? last : 2];
  TapRec tr;
  {
    const Stage s0 = stage_load<INTERIOR>(pack, e0, R, x0, y0, W, H, sl);
    stage_store_texels(stg[0], s0, sl);
    tr = s0.tr;
  }
  float uz = e0.z, uw = e0.w;
  Stage sn = stage_load<INTERIOR>(pack, e1, R, x0, y0, W, H, sl);  // tap 1 (in flight)
  for (int t = 0; t < n_taps; ++t) {
    wave_lds_sync();  // tap t's texels stored; tap t - 1's reads done
    const int b = t & 1;
    stage_store_texels(stg[b ^ 1], sn, sl);  // tap t + 1
    const TapRec trn = sn.tr;
    const float unz = e1.z, unw = e1.w;
    sn = stage_load<INTERIOR>(pack, e2, R, x0, y0, W, H, sl);  // tap t + 2
    e1 = e2;
    e2 = taps[t + 3 < last ? t + 3 : last];
    {
      const float4* a = stg[b] + lofs;
      const float4 v00 = a[0], v10 = a[1], v20 = a[2];
      const float4 v01 = a[PPG_STRIDE], v11 = a[PPG_STRIDE + 1], v21 = a[PPG_STRIDE + 2];
      const float4 v02 = a[2 * PPG_STRIDE], v12 = a[2 * PPG_STRIDE + 1], v22 = a[2 * PPG_STRIDE + 2];
      const float d = fmaf(-R, uz, 0.5f);
      const float om = SA ? uw : 1.0f;
      g[0].tap(tr.w00, tr.w10, tr.w01, tr.w11, d, v00, v10, v01, v11, om);
      g[1].tap(tr.w00, tr.w10, tr.w01, tr.w11, d, v10, v20, v11, v21, om);
      g[2].tap(tr.w00, tr.w10, tr.w01, tr.w11, d, v01, v11, v02, v12, om);
      g[3].tap(tr.w00, tr.w10, tr.w01, tr.w11, d, v11, v21, v12, v22, om);
    }
    tr = trn;
    uz = unz;
    uw = unw;
  }
}

// 16-pixel tiles, one wave per tile (the quad form): lane l gathers the
// 2x2 quad at (2 (l mod 8), 2 (l div 8)) of its tile, so per tap a tile
// reads 2.25 staged texels per pixel from LDS instead of 4, and each wave
// stages its own taps into its own ring (no barrier between waves).  A
// block holds four neighbouring tiles, so it frees as much LDS at a time
// as the four-wave form does (a kernel running beside it, such as the ray
// mask, needs whole blocks' worth).  Same arithmetic, in the same tap
// order, as k_pp_gather16, so the same results bit for bit.
template <int FUSE, bool SA>
__device__ __forceinline__ void gather16q_tile(float4 (*stg)[PPG_TAPSZ], const float4* __restrict__ pack,
                                               const float* __restrict__ tile_r, int K, float r_cap,
                                               const float4* __restrict__ taps, int n_taps, int W, int H,
                                               float inv_ramp, float* __restrict__ out, const FuseK& fz, int tile) {
  const int TW = (W + 15) >> 4, TH = (H + 15) >> 4;
  const int x0 = (tile % TW) * 16, y0 = (tile / TW) * 16;
  const int lane = threadIdx.x & 63;
  const int qx = (lane & 7) * 2, qy = (lane >> 3) * 2;
  const size_t N = (size_t)W * H;
  const float R = wave_dilated_radius(tile_r, TW, TH, tile % TW, tile / TW, K, r_cap);
  if (!(R > 0.0f)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int x = x0 + qx + (q & 1), y = y0 + qy + (q >> 1);
      if (x < W && y < H) {
        const size_t p = (size_t)y * W + x;
        const float4 c = pack[p];
        pp_emit<FUSE>(out, fz, N, p, c, c.x, c.y, c.z);
      }
    }
    return;
  }
  const int E = (int)ceilf(R);
  const bool interior = x0 - E - 1 >= 0 && x0 + 16 + E < W && y0 - E - 1 >= 0 && y0 + 16 + E < H &&
                        (long long)W * H * 16 < (1ll << 31);
  GatherAcc g[4];
  float4 cp[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int x = x0 + qx + (q & 1), y = y0 + qy + (q >> 1);
    cp[q] = x < W && y < H ? pack[(size_t)y * W + x] : make_float4(0.f, 0.f, 0.f, 0.f);
    g[q].init(cp[q], R, n_taps, inv_ramp);
  }
  const int lofs = qy * PPG_STRIDE + qx;
  if (interior)
    gather_taps_quad<true, SA>(stg, pack, taps, n_taps, R, x0, y0, W, H, lane, lofs, g);
  else
    gather_taps_quad<false, SA>(stg, pack, taps, n_taps, R, x0, y0, W, H, lane, lofs, g);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int x = x0 + qx + (q & 1), y = y0 + qy + (q >> 1);
    if (x < W && y < H) {
      const size_t p = (size_t)y * W + x;
      const float iw = 1.0f / g[q].ws;
      pp_emit<FUSE>(out, fz, N, p, cp[q], g[q].ar * iw, g[q].ag * iw, g[q].ab * iw);
    }
  }
}

template <int FUSE, bool SA>
__global__ __launch_bounds__(256) void k_pp_gather16q(const float4* __restrict__ pack,
                                                      const float* __restrict__ tile_r, int K, float r_cap,
                                                      const float4* __restrict__ taps, int n_taps, int W, int H,
                                                      float inv_ramp, float* __restrict__ out, FuseK fz) {
  __shared__ float4 stg[4][2][PPG_TAPSZ];
  const int TW = (W + 15) >> 4, TH = (H + 15) >> 4;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int pos = xcd_block(blockIdx.x, (TW * TH + 3) >> 2) * 4 + wave;
  if (pos >= TW * TH) return;
  const int tile = rect_tile(pos, TW, TH);
  gather16q_tile<FUSE, SA>(stg[wave], pack, tile_r, K, r_cap, taps, n_taps, W, H, inv_ramp, out, fz, tile);
}

// The batched form's gathers in the quad form: each wave finds the view of
// its own tile (a block's four tiles may straddle two views).
template <bool SA>
__global__ __launch_bounds__(256) void k_pp_gather16q_batch(const float4* __restrict__ pack,
                                                            const float* __restrict__ tile_r, int K, float r_cap,
                                                            const float4* __restrict__ taps, int n_taps,
                                                            float inv_ramp, float* __restrict__ pp_out,
                                                            const BatchView* __restrict__ views, PPBatch b) {
  __shared__ float4 stg[4][2][PPG_TAPSZ];
  const int total = b.tile_base[b.n];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int g = xcd_block(blockIdx.x, (total + 3) >> 2) * 4 + wave;
  if (g >= total) return;
  const int v = __builtin_amdgcn_readfirstlane(batch_view_of(b.tile_base, b.n, g));
  const int W = views[v].k.W, H = views[v].k.H;
  const size_t pb = (size_t)views[v].px_base;
  FuseK fz{};
  fz.out = b.out[v];
  gather16q_tile<2, SA>(stg[wave], pack + pb, tile_r + b.tile_base[v], K, r_cap, taps, n_taps, W, H, inv_ramp,
                        pp_out + 3 * pb, fz, g - b.tile_base[v]);
}

// Tiles of 4 or 8 pixels: per-lane radius and per-lane tap geometry, every
// texel clamped to the edge.
__global__ __launch_bounds__(256) void k_pp_gather_any(const float4* __restrict__ pack, const float* __restrict__ rad,
                                                       const float4* __restrict__ taps, int n_taps, int W, int H,
                                                       int tile, float inv_ramp, float* __restrict__ out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x = blockIdx.x * 16 + (lane & 15), y = blockIdx.y * 16 + wave * 4 + (lane >> 4);
  if (x >= W || y >= H) return;
  const int TW = (W + tile - 1) / tile;
  const size_t N = (size_t)W * H, p = (size_t)y * W + x;
  const float R = rad[(y / tile) * TW + x / tile];
  const float4 cp4 = pack[p];
  GatherAcc g;
  g.init(cp4, R, n_taps, inv_ramp);
  if (R > 0.0f) {
    for (int k = 0; k < n_taps; ++k) {
      const float4 u = taps[k];
      const float ox = R * u.x, oy = R * u.y;
      const float fx = floorf(ox), fy = floorf(oy);
      const float ax = ox - fx, ay = oy - fy, bx = 1.0f - ax, by = 1.0f - ay;
      float4 v00, v10, v01, v11;
      texels_clamped(pack, W, H, x + (int)fx, y + (int)fy, v00, v10, v01, v11);
      g.tap(bx * by, ax * by, bx * ay, ax * ay, 0.5f - R * u.z, v00, v10, v01, v11, u.w);
    }
  }
  g.store(out, N, p);
}

// The post-filtered specular luminance (the specular bokeh rule of the
// composite): the post-filter's gather, radius, taps and weights, applied to
// the G-buffer's specular luminance plane.  With spp given only traced
// pixels gather (the rule reads no other), the rest are 0.  Texels are
// fetched directly: a frame traces a few percent of its pixels.  One 8x8
// block (a ray-mask tile) per 256 threads, four lanes per pixel splitting
// its taps (tap j on lane j mod 4, sums joined by lane exchanges), so the
// few traced tiles get four times the memory parallelism of a lane per
// pixel; a block without a traced pixel writes 0 and leaves.  Blocks run in
// launch order, round-robin over the XCDs (the traced pixels cluster along
// a few silhouettes, which XCD-contiguous ranges would give to one XCD).
// Radius: tile 16, the dilated radius of the block's 16-pixel tile from
// tile_r; otherwise the pixel's tile entry of the dilated radii.
__global__ __launch_bounds__(256) void k_pp_spec(const float4* __restrict__ pack, const float* __restrict__ ys,
                                                 const uint8_t* __restrict__ spp, const float* __restrict__ tile_r,
                                                 const float* __restrict__ rad, int tile, int K, float r_cap,
                                                 const float4* __restrict__ taps, int n_taps, int W, int H,
                                                 float inv_ramp, float* __restrict__ out) {
  __shared__ float wred[4];
  const int BW = (W + 7) >> 3;
  const int bx = blockIdx.x % BW, by = blockIdx.x / BW;
  const int pi = threadIdx.x >> 2, sub = threadIdx.x & 3;
  const int x = bx * 8 + (pi & 7), y = by * 8 + (pi >> 3);
  const bool in = x < W && y < H;
  const size_t p = in ? (size_t)y * W + x : 0;
  const bool act = in && (!spp || spp[p] > 0);
  if (!__syncthreads_or(act)) {
    if (in && sub == 0) out[p] = 0.0f;
    return;
  }
  float R;
  if (tile == 16) {
    R = block_dilated_radius(tile_r, (W + 15) >> 4, (H + 15) >> 4, bx >> 1, by >> 1, K, r_cap, wred);
  } else {
    const int TW = (W + tile - 1) / tile;
    R = in ? rad[(y / tile) * TW + x / tile] : 0.0f;
  }
  if (!act) {  // the pixel's four lanes leave together
    if (in && sub == 0) out[p] = 0.0f;
    return;
  }
  GatherAcc g;
  g.init(make_float4(ys[p], 0.0f, 0.0f, pack[p].w), R, n_taps, inv_ramp);
  if (sub != 0) g.ar = g.ws = 0.0f;  // the centre counts once
  // this lane's taps sub, sub + 4, ... in groups of four: a group's loads
  // are all issued before its sums (a tap past the end accepts nothing)
  for (int j0 = sub; j0 < n_taps; j0 += 16) {
    float4 v[4][4];
    float wb[4][4], d[4], om[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = min(j0 + 4 * q, n_taps - 1);
      const float4 u = taps[j];
      om[q] = u.w;
      const float ox = R * u.x, oy = R * u.y;
      const float fx = floorf(ox), fy = floorf(oy);
      const float ax = ox - fx, ay = oy - fy, bxw = 1.0f - ax, byw = 1.0f - ay;
      wb[q][0] = bxw * byw;
      wb[q][1] = ax * byw;
      wb[q][2] = bxw * ay;
      wb[q][3] = ax * ay;
      d[q] = j0 + 4 * q < n_taps ? 0.5f - R * u.z : -1e30f;
      const int xa = x + (int)fx, ya = y + (int)fy;
      const int xa_ = clampi(xa, 0, W - 1), xb_ = clampi(xa + 1, 0, W - 1);
      const int ya_ = clampi(ya, 0, H - 1), yb_ = clampi(ya + 1, 0, H - 1);
      const size_t i00 = (size_t)ya_ * W + xa_, i10 = (size_t)ya_ * W + xb_;
      const size_t i01 = (size_t)yb_ * W + xa_, i11 = (size_t)yb_ * W + xb_;
      v[q][0] = make_float4(ys[i00], 0.0f, 0.0f, pack[i00].w);
      v[q][1] = make_float4(ys[i10], 0.0f, 0.0f, pack[i10].w);
      v[q][2] = make_float4(ys[i01], 0.0f, 0.0f, pack[i01].w);
      v[q][3] = make_float4(ys[i11], 0.0f, 0.0f, pack[i11].w);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      g.tap(wb[q][0], wb[q][1], wb[q][2], wb[q][3], d[q], v[q][0], v[q][1], v[q][2], v[q][3], om[q]);
  }
  float ar = g.ar, ws = g.ws;
  ar += __shfl_xor(ar, 1);
  ws += __shfl_xor(ws, 1);
  ar += __shfl_xor(ar, 2);
  ws += __shfl_xor(ws, 2);
  if (sub == 0) out[p] = ar / ws;
}

// pps (nullable): the post-filtered specular luminance; inv_sy = 1 / spec_y
// (0: the specular bokeh rule is off)
struct CompK {
  const float *color, *pp, *depth;
  const uint8_t* spp;
  const float *cn, *cf, *hr;
  LensK l;
  int N;
  float inv_ht;
  int rt_override;
  const float* pps;
  float inv_sy;
  float* out;
};

__device__ __forceinline__ void composite_at(const CompK& a, int p) {
  const int N = a.N;
  const float c = coc_px(a.l, a.depth[p]);
  const float phi = clamp01(fabsf(c) - HDOF_SQRT2);
  const float nu = clamp01(fmaf(-c, 0.35355339059327376f, 0.5f));
  // the traced colours enter only where the pixel was traced, the filtered
  // colour only outside the focus zone: other loads are skipped (the mask
  // leaves most 64-pixel rows untraced, so their lines are never fetched)
  const bool traced = a.spp[p] > 0;
  const float h = traced ? a.hr[p] : 0.0f;
  const float rho = traced ? 1.0f : 0.0f;
  const float beta = traced ? clamp01(1.0f - h * a.inv_ht) : 0.0f;
  const float sig = (a.pps && traced && a.inv_sy > 0.0f) ? clamp01(a.pps[p] * a.inv_sy) : 0.0f;
  for (int q = 0; q < 3; ++q) {
    size_t i = (size_t)q * N + p;
    const float crt = traced ? traced_mix(h, a.cn[i], a.cf[i]) : 0.0f;
    const float cpp = phi > 0.0f ? a.pp[i] : 0.0f;
    float o = composite_mix(a.color[i], cpp, crt, phi, nu, rho, beta, sig);
    if (a.rt_override && traced) o = crt;
    a.out[i] = o;
  }
}

__global__ void k_composite(CompK a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < a.N) composite_at(a, p);
}

// Traced pixels only (the others hold the untraced rule's result).  One
// thread per pixel: with four pixels per thread the traced pixels' loads
// serialise and the pass is slower (12.5 against 9.8 µs at 1080p).
__global__ void k_composite_traced(CompK a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < a.N && a.spp[p] > 0) composite_at(a, p);
}

// every view's traced pixels in one launch, HDOF_BATCH_PX_BLOCK pixels per
// block; `a` holds the first view's planes (all views' planes are
// concatenated from their px_base)
__global__ void k_composite_traced_batch(CompK a, const BatchView* __restrict__ views, PPBatch b) {
  const int v = batch_view_of(b.blk_base, b.n, blockIdx.x);
  const int N = views[v].k.W * views[v].k.H;
  const size_t pb = (size_t)views[v].px_base;
  CompK c = a;
  c.color += 3 * pb;
  c.pp += 3 * pb;
  c.depth += pb;
  c.spp += pb;
  c.cn += 3 * pb;
  c.cf += 3 * pb;
  c.hr += pb;
  c.l = views[v].l;
  c.N = N;
  c.out = b.out[v];
  const int p0 = (blockIdx.x - b.blk_base[v]) * HDOF_BATCH_PX_BLOCK;
  for (int i = threadIdx.x; i < HDOF_BATCH_PX_BLOCK; i += blockDim.x) {
    const int p = p0 + i;
    if (p >= N) break;
    if (c.spp[p] > 0) composite_at(c, p);
  }
}

// ---------------------------------------------------------------------------
// Adjoint of post-filter + composite (differentiable form).
// Reverse mode for the colour (the gather's transpose: every tap's share goes
// back to its four bilinear texels), forward mode for
// the focus distance S1 and aperture A (each value carries its two
// derivatives through the recomputed gather: no weights are stored).
// ---------------------------------------------------------------------------
struct D3 {
  float v, s, a;  // value, d/dS1, d/dA
};
__device__ inline D3 dk(float v, float s, float a) { return D3{v, s, a}; }
__device__ inline D3 dc(float v) { return D3{v, 0.f, 0.f}; }
__device__ inline D3 operator+(D3 x, D3 y) { return D3{x.v + y.v, x.s + y.s, x.a + y.a}; }
__device__ inline D3 operator-(D3 x, D3 y) { return D3{x.v - y.v, x.s - y.s, x.a - y.a}; }
__device__ inline D3 operator*(D3 x, D3 y) { return D3{x.v * y.v, fmaf(x.s, y.v, x.v * y.s), fmaf(x.a, y.v, x.v * y.a)}; }
__device__ inline D3 operator*(float k, D3 x) { return D3{k * x.v, k * x.s, k * x.a}; }
__device__ inline D3 dquot(D3 x, D3 y) {
  const float iy = __builtin_amdgcn_rcpf(y.v), q = x.v * iy;
  return D3{q, (x.s - q * y.s) * iy, (x.a - q * y.a) * iy};
}
// clamp with zero slope outside the open interval (lo, hi)
__device__ inline D3 dclamp(D3 x, float lo, float hi) { return x.v <= lo ? dc(lo) : (x.v >= hi ? dc(hi) : x); }
__device__ inline D3 dmaxc(D3 x, float c) { return x.v > c ? x : dc(c); }
__device__ inline D3 dabs(D3 x) { return x.v >= 0.f ? x : D3{-x.v, -x.s, -x.a}; }

// pack (rgb, c), tile max with its pixel
__global__ __launch_bounds__(256) void k_ppb_pack(const float* __restrict__ color, const float* __restrict__ depth,
                                                  CamK k, LensK l, int tile, float4* __restrict__ pack,
                                                  float* __restrict__ tile_r, int* __restrict__ tile_arg) {
  __shared__ float red[256];
  __shared__ int redi[256];
  const int tid = threadIdx.x;
  const int BX = (k.W + 15) >> 4, lb = xcd_block(blockIdx.x, BX * ((k.H + 15) >> 4));
  const int x = (lb % BX) * 16 + (tid & 15), y = (lb / BX) * 16 + (tid >> 4);
  const size_t N = (size_t)k.W * k.H;
  float r = -1.0f;
  int idx = 0x7fffffff;
  if (x < k.W && y < k.H) {
    size_t p = (size_t)y * k.W + x;
    float c = coc_px(l, depth[p]);
    pack[p] = make_float4(color[p], color[N + p], color[2 * N + p], c);
    r = 0.5f * fabsf(c);
    idx = (int)p;
  }
  red[tid] = r;
  redi[tid] = idx;
  __syncthreads();
  // the largest radius of each tile and its lowest pixel index: first along
  // each tile row (the row's first thread), then over the tile's rows
  const int tx = tid & 15, ty = tid >> 4;
  __shared__ float rowm[256];
  __shared__ int rowi[256];
  if ((tx % tile) == 0) {
    float m = -1.0f;
    int mi = 0x7fffffff;
    for (int dx = 0; dx < tile; ++dx) {
      const float v = red[ty * 16 + tx + dx];
      const int vi = redi[ty * 16 + tx + dx];
      if (v > m || (v == m && vi < mi)) {
        m = v;
        mi = vi;
      }
    }
    rowm[tid] = m;
    rowi[tid] = mi;
  }
  __syncthreads();
  if ((tx % tile) == 0 && (ty % tile) == 0 && x < k.W && y < k.H) {
    float m = -1.0f;
    int mi = 0x7fffffff;
    for (int dy = 0; dy < tile; ++dy) {
      const float v = rowm[(ty + dy) * 16 + tx];
      const int vi = rowi[(ty + dy) * 16 + tx];
      if (v > m || (v == m && vi < mi)) {
        m = v;
        mi = vi;
      }
    }
    const int TW = (k.W + tile - 1) / tile;
    tile_r[(y / tile) * TW + x / tile] = m;
    tile_arg[(y / tile) * TW + x / tile] = mi;
  }
}

// dilated radius and the pixel that sets it (-1 when capped or zero)
__global__ void k_ppb_dilate(const float* __restrict__ tile_r, const int* __restrict__ tile_arg, int TW, int TH,
                             int K, float r_cap, float* __restrict__ rad, int* __restrict__ rad_arg) {
  int tx = blockIdx.x * blockDim.x + threadIdx.x, ty = blockIdx.y;
  if (tx >= TW) return;
  float m = -1.0f;
  int mi = 0x7fffffff;
  for (int dy = -K; dy <= K; ++dy) {
    int yy = ty + dy;
    if (yy < 0 || yy >= TH) continue;
    for (int dx = -K; dx <= K; ++dx) {
      int xx = tx + dx;
      if (xx < 0 || xx >= TW) continue;
      float v = tile_r[yy * TW + xx];
      int vi = tile_arg[yy * TW + xx];
      if (v > m || (v == m && vi < mi)) {
        m = v;
        mi = vi;
      }
    }
  }
  rad[ty * TW + tx] = fminf(r_cap, m);
  rad_arg[ty * TW + tx] = (m < r_cap && m > 0.0f) ? mi : -1;
}

__global__ void k_fill_f(float* __restrict__ p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

#ifndef PPB_WIN_E
#define PPB_WIN_E 21                     // largest ceil(R) accumulated in one LDS window per block
#endif
#define PPB_WIN (17 + 2 * PPB_WIN_E)     // window side at that radius
#define PPB_FOOT (PPG_SIDE * PPG_SIDE)   // one tap's 17x17 footprint
#define PPB_PAD 18                       // the posts' 16x16 grid with a zero border

// Sample geometry of tap u at radius R relative to a pixel's texel grid: the
// footprint corner offset (floor R u) and the bilinear fractions.
struct TapGeo {
  int ix, iy;
  float ax, ay;
};
__device__ __forceinline__ TapGeo tap_geo(float R, float4 u) {
  const float ox = R * u.x, oy = R * u.y;
  const float fx = floorf(ox), fy = floorf(oy);
  return TapGeo{(int)fx, (int)fy, ox - fx, oy - fy};
}

// texels_clamped with 32-bit byte offsets (images below 2^28 pixels)
__device__ __forceinline__ void texels_clamped32(const float4* __restrict__ pack, int W, int H, int xa, int ya,
                                                 float4& v00, float4& v10, float4& v01, float4& v11) {
  const unsigned xa_ = (unsigned)clampi(xa, 0, W - 1), xb_ = (unsigned)clampi(xa + 1, 0, W - 1);
  const unsigned ya_ = (unsigned)clampi(ya, 0, H - 1) * (unsigned)W, yb_ = (unsigned)clampi(ya + 1, 0, H - 1) * (unsigned)W;
  const char* pb = (const char*)pack;
  v00 = *(const float4*)(pb + ((ya_ + xa_) << 4));
  v10 = *(const float4*)(pb + ((ya_ + xb_) << 4));
  v01 = *(const float4*)(pb + ((yb_ + xa_) << 4));
  v11 = *(const float4*)(pb + ((yb_ + xb_) << 4));
}

// The forward-mode gather's taps of one pixel (value, d/dS1, d/dA).  SLOPE:
// the tile radius R moves with S1 and A, so every sample moves with it and
// its spatial slopes enter the derivatives.
template <bool SLOPE>
__device__ __forceinline__ void fwd_taps(const float4* __restrict__ pack, const float4* __restrict__ taps, int ntap,
                                         int n_taps, int W, int H, int x, int y, const D3& R, const D3& cpv,
                                         const D3& rp, float dcs, float inv_A, float inv_ramp, D3& nr, D3& ng,
                                         D3& nb, D3& den) {
  if (ntap <= 0) return;
  // each tap's texels are requested one tap ahead, so their latency overlaps
  // the previous tap's arithmetic (the last tap's are requested twice)
  float4 v00, v10, v01, v11;
  {
    const TapGeo t0 = tap_geo(R.v, taps[0]);
    texels_clamped32(pack, W, H, x + t0.ix, y + t0.iy, v00, v10, v01, v11);
  }
  for (int kk = 0; kk < ntap; ++kk) {
    const float4 u = taps[kk];
    const TapGeo tg = tap_geo(R.v, u);
    const float ax = tg.ax, ay = tg.ay, bx = 1.f - ax, by = 1.f - ay;
    float4 n00, n10, n01, n11;
    {
      const TapGeo tn = tap_geo(R.v, taps[kk + 1 < ntap ? kk + 1 : kk]);
      texels_clamped32(pack, W, H, x + tn.ix, y + tn.iy, n00, n10, n01, n11);
    }
    const float w00 = bx * by, w10 = ax * by, w01 = bx * ay, w11 = ax * ay;
    // samples, their spatial slopes, and their motion with R
    const float dxs = u.x * R.s, dxa = u.x * R.a, dys = u.y * R.s, dya = u.y * R.a;
#define SAMPLE(c)                                                                                   \
  const float s_##c = w00 * v00.c + w10 * v10.c + w01 * v01.c + w11 * v11.c;                        \
  const float sx_##c = SLOPE ? by * (v10.c - v00.c) + ay * (v11.c - v01.c) : 0.f;                    \
  const float sy_##c = SLOPE ? bx * (v01.c - v00.c) + ax * (v11.c - v10.c) : 0.f;
    SAMPLE(x) SAMPLE(y) SAMPLE(z) SAMPLE(w)
#undef SAMPLE
    const D3 cq = SLOPE ? dk(s_w, dcs + sx_w * dxs + sy_w * dys, s_w * inv_A + sx_w * dxa + sy_w * dya)
                        : dk(s_w, dcs, s_w * inv_A);
    const D3 rq = 0.5f * dabs(cq);
    const D3 tk = dclamp(inv_ramp * (cq - cpv), 0.f, 1.f);
    const D3 dpos = dmaxc(rq - rp, 0.f);
    const D3 reff = rq - tk * dpos;
    const D3 a = dclamp(reff - u.z * R + dc(0.5f), 0.f, 1.f);
    const D3 rq5 = dmaxc(rq, 0.5f);
    const D3 w = dquot(a * ((1.0f / (float)n_taps) * (R * R)), rq5 * rq5);
    if (SLOPE) {
      nr = nr + w * dk(s_x, sx_x * dxs + sy_x * dys, sx_x * dxa + sy_x * dya);
      ng = ng + w * dk(s_y, sx_y * dxs + sy_y * dys, sx_y * dxa + sy_y * dya);
      nb = nb + w * dk(s_z, sx_z * dxs + sy_z * dys, sx_z * dxa + sy_z * dya);
    } else {
      nr = nr + s_x * w;
      ng = ng + s_y * w;
      nb = nb + s_z * w;
    }
    den = den + w;
    v00 = n00;
    v10 = n10;
    v01 = n01;
    v11 = n11;
  }
}

// The CoCs (w) of the four clamp-to-edge texels of the bilinear footprint
// whose corner is (xa, ya), in the order 00, 10, 01, 11 (images below 2^28
// pixels: 32-bit byte offsets).
__device__ __forceinline__ float4 cocs_clamped(const float4* __restrict__ pack, int W, int H, int xa, int ya) {
  const unsigned xa_ = (unsigned)clampi(xa, 0, W - 1), xb_ = (unsigned)clampi(xa + 1, 0, W - 1);
  const unsigned ya_ = (unsigned)clampi(ya, 0, H - 1) * (unsigned)W, yb_ = (unsigned)clampi(ya + 1, 0, H - 1) * (unsigned)W;
  const char* pw = (const char*)pack + 12;
  return make_float4(*(const float*)(pw + ((ya_ + xa_) << 4)), *(const float*)(pw + ((ya_ + xb_) << 4)),
                     *(const float*)(pw + ((yb_ + xa_) << 4)), *(const float*)(pw + ((yb_ + xb_) << 4)));
}

// Footprint texel t = (r, q) of one tap collects the posts of pixels
// (r - dy, q - dx) with the block-uniform bilinear weight of corner (dx, dy);
// kb is the padded post grid (zero border), so no bounds checks.  MODE 1:
// added to the block's LDS window; MODE 2: added to the image (clamped to
// the edge) with global atomics.
template <int MODE>
__device__ __forceinline__ void foot_texel(const float4* kb, int t, float w00, float w10, float w01, float w11,
                                           const TapGeo& tg, int E, int wd, float* acc, float* __restrict__ gcol,
                                           int x0, int y0, int W, int H, size_t N) {
  const int r = t / PPG_SIDE, q = t - r * PPG_SIDE;
  const float4* b = kb + r * PPB_PAD + q;  // padded (r - dy + 1, q - dx + 1) = b[(1 - dy) PPB_PAD + 1 - dx]
  const float4 k00 = b[PPB_PAD + 1], k01 = b[PPB_PAD], k10 = b[1], k11 = b[0];
  float3 v;
  v.x = fmaf(w11, k11.x, fmaf(w01, k10.x, fmaf(w10, k01.x, w00 * k00.x)));
  v.y = fmaf(w11, k11.y, fmaf(w01, k10.y, fmaf(w10, k01.y, w00 * k00.y)));
  v.z = fmaf(w11, k11.z, fmaf(w01, k10.z, fmaf(w10, k01.z, w00 * k00.z)));
  if (MODE == 1) {
    float* wp = acc + (tg.iy + E + r) * wd + tg.ix + E + q;
    wp[0] += v.x;
    wp[wd * wd] += v.y;
    wp[2 * wd * wd] += v.z;
  } else if (v.x != 0.f || v.y != 0.f || v.z != 0.f) {
    // footprint texel (r, q) is image texel (y0 + iy + r, x0 + ix + q), clamped to the edge
    const size_t gi = (size_t)clampi(y0 + tg.iy + r, 0, H - 1) * W + clampi(x0 + tg.ix + q, 0, W - 1);
    atomicAdd(&gcol[gi], v.x);
    atomicAdd(&gcol[N + gi], v.y);
    atomicAdd(&gcol[2 * N + gi], v.z);
  }
}

// Adjoint of post-filter + composite.  Pass 1 per pixel: the gather again in
// forward mode (value, d/dS1, d/dA through the CoC, the tile radius and the
// sample positions), then the composite backward, which gives the focus and
// aperture gradients (block partials) and the colour gradient of the pixel
// itself.  Pass 2: the colour gradient flowing through the gather weights,
// scattered to the four texels of every tap.  16-pixel tiles (UNI) share
// one tap geometry per block: per tap the block's contributions land on one
// 17x17 footprint, which is formed in LDS as a transposed bilinear gather of
// the pixels' posts (no LDS atomics) and then added to one
// (17 + 2 ceil R)^2 LDS window for ceil R <= PPB_WIN_E (flushed once with
// global atomics) or straight to global memory (larger R); window and
// footprint texels are image texels clamped to the edge, as in the gather.
// Other tile sizes add straight to global memory per pixel and tap.
template <bool UNI>
__global__ __launch_bounds__(256) void k_ppc_backward(
    const float4* __restrict__ pack, const float* __restrict__ rad, const int* __restrict__ rad_arg,
    const float4* __restrict__ taps, int n_taps, int W, int H, int tile, float inv_ramp, LensK l, float spx,
    const uint8_t* __restrict__ spp, const float* __restrict__ cn, const float* __restrict__ cf,
    const float* __restrict__ hr, float inv_ht, int rt_override, const float* __restrict__ g,
    float* __restrict__ gcol, float2* __restrict__ partial) {
  __shared__ float acc[UNI ? 3 * PPB_WIN * PPB_WIN : 1];
  // two buffers of the 16x16 pixels' posts, each with a zero border (18x18)
  __shared__ float4 posts[UNI ? 2 : 1][UNI ? PPB_PAD * PPB_PAD : 128];
  float2* red = (float2*)&posts[0][0];  // the partials' reduction, after pass 2
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int TWb = (W + 15) >> 4, THb = (H + 15) >> 4;
  const int blk = UNI ? xcd_block(blockIdx.x, TWb * THb) : blockIdx.x;
  const int x0 = (blk % TWb) * 16, y0 = (blk / TWb) * 16;
  const int lx = lane & 15, ly = wave * 4 + (lane >> 4);
  const int x = x0 + lx, y = y0 + ly;
  float gs = 0.0f, ga = 0.0f;
  const size_t N = (size_t)W * H;
  const float dcs = -l.A * spx * l.invS1 * l.invS1;  // dc/dS1 (every pixel)
  const float inv_A = l.A > 0.0f ? 1.0f / l.A : 0.0f;  // unit CoC = c / A
  const bool inside = x < W && y < H;
  const size_t p = inside ? (size_t)y * W + x : 0;
  const bool traced = inside && spp[p] > 0;
  const bool active = inside && !(rt_override && traced);
  const int TW = (W + tile - 1) / tile;
  const int ti = UNI ? blk : (inside ? (y / tile) * TW + x / tile : 0);
  const float Rv = rad[ti];
  const int E = (int)ceilf(Rv);
  // scatter mode of the block (UNI): 0 global, 1 window, 2 per-tap footprint
  int mode = 0;
  if (UNI && Rv > 0.0f) mode = E <= PPB_WIN_E ? 1 : 2;
  const int wd = 17 + 2 * E;
  if (UNI && mode == 1)
    for (int i = tid; i < 3 * wd * wd; i += 256) acc[i] = 0.0f;
  if (UNI && mode != 0) {
    for (int i = tid; i < 2 * PPB_PAD * PPB_PAD; i += 256) (&posts[0][0])[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
  }
  const int ntap = Rv > 0.0f ? n_taps : 0;
  float4 cp4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float gpp[3] = {0.f, 0.f, 0.f};
  float area = 0.0f;
  if (active) {
    cp4 = pack[p];
    const D3 cpv = dk(cp4.w, dcs, cp4.w * inv_A);
    // composite weights
    const D3 phi = dclamp(dabs(cpv) - dc(HDOF_SQRT2), 0.f, 1.f);
    const D3 nu = dclamp(dc(0.5f) - 0.35355339059327376f * cpv, 0.f, 1.f);
    const float h = hr[p];
    const float rho = traced ? 1.0f : 0.0f;
    const float beta = traced ? clamp01(1.0f - h * inv_ht) : 0.0f;
    const D3 acoef = rho * nu + beta * (dc(1.f) - nu);
    const D3 bcoef = (1.f - rho) * nu + (1.f - beta) * (dc(1.f) - nu);
    // forward-mode gather
    const D3 rp = 0.5f * dabs(cpv);
    const D3 rp5 = dmaxc(rp, 0.5f);
    const D3 w0 = dquot(dc(1.f), rp5 * rp5);
    D3 R = dc(Rv);
    const int m = rad_arg[ti];
    if (m >= 0) {
      const float cm = pack[m].w;
      const float sg = cm >= 0.f ? 0.5f : -0.5f;
      R = dk(R.v, sg * dcs, sg * cm * inv_A);
    }
    D3 nr = w0 * dc(cp4.x), ng = w0 * dc(cp4.y), nb = w0 * dc(cp4.z), den = w0;
    // a tile radius at the cap does not move with S1 or A: the samples stay
    // put and their spatial slopes drop out
    if (R.s != 0.0f || R.a != 0.0f)
      fwd_taps<true>(pack, taps, ntap, n_taps, W, H, x, y, R, cpv, rp, dcs, inv_A, inv_ramp, nr, ng, nb, den);
    else
      fwd_taps<false>(pack, taps, ntap, n_taps, W, H, x, y, R, cpv, rp, dcs, inv_A, inv_ramp, nr, ng, nb, den);
    // composite backward per channel; post-filter transpose for the colour
    const float gq[3] = {g[p], g[N + p], g[2 * N + p]};
    const D3 num[3] = {nr, ng, nb};
    const float cr[3] = {cp4.x, cp4.y, cp4.z};
    const float iden = 1.0f / den.v;
    for (int c = 0; c < 3; ++c) {
      const float crt = h * cn[c * N + p] + (1.f - h) * cf[c * N + p];
      const D3 cpp = dquot(num[c], den);
      const D3 oof = crt * acoef + bcoef * cpp;
      const D3 out = (dc(1.f) - phi) * dc(cr[c]) + phi * oof;
      gs = fmaf(gq[c], out.s, gs);
      ga = fmaf(gq[c], out.a, ga);
      gpp[c] = gq[c] * phi.v * bcoef.v * iden;
      const float own = fmaf(gq[c], 1.f - phi.v, gpp[c] * w0.v);
      if (mode == 1)
        acc[(c * wd + ly + E) * wd + lx + E] += own;  // this pixel's own window texel
      else
        atomicAdd(&gcol[c * N + p], own);
    }
    area = R.v * R.v / (float)n_taps;
  }
  // pass 2: the weights again (value only) and the scatter of gpp * weight
  const bool scat = active && (gpp[0] != 0.f || gpp[1] != 0.f || gpp[2] != 0.f);
  const float rpv = 0.5f * fabsf(cp4.w);
  if (UNI && mode != 0) {
    // per tap: every pixel posts gpp * weight, then footprint texel (r, q)
    // collects the posts of pixels (r - dy, q - dx) with the block-uniform
    // bilinear weight of corner (dx, dy)
    // each tap's texel CoCs are requested one tap ahead (see fwd_taps)
    float4 cw = make_float4(0.f, 0.f, 0.f, 0.f);
    // blocks start at different taps, so neighbouring blocks' atomics land
    // on different texels at a time
    const int rot = ntap > 0 ? (int)((blk * 17u) % (unsigned)ntap) : 0;
    if (scat && ntap > 0) {
      const TapGeo t0 = tap_geo(Rv, taps[rot]);
      cw = cocs_clamped(pack, W, H, x + t0.ix, y + t0.iy);
    }
    for (int kk = 0; kk < ntap; ++kk) {
      const int ki = kk + rot < ntap ? kk + rot : kk + rot - ntap;
      const float4 u = taps[ki];
      const TapGeo tg = tap_geo(Rv, u);
      const float ax = tg.ax, ay = tg.ay, bx = 1.f - ax, by = 1.f - ay;
      float4 cwn = cw;
      if (scat && kk + 1 < ntap) {
        const int kn = ki + 1 < ntap ? ki + 1 : 0;
        const TapGeo tn = tap_geo(Rv, taps[kn]);
        cwn = cocs_clamped(pack, W, H, x + tn.ix, y + tn.iy);
      }
      float4 post = make_float4(0.f, 0.f, 0.f, 0.f);
      if (scat) {
        const float cq = bx * by * cw.x + ax * by * cw.y + bx * ay * cw.z + ax * ay * cw.w;
        const float rq = 0.5f * fabsf(cq);
        const float tk = clamp01((cq - cp4.w) * inv_ramp);
        const float a = clamp01(rq - tk * fmaxf(0.f, rq - rpv) - Rv * u.z + 0.5f);
        const float rq5 = fmaxf(rq, 0.5f);
        const float wv = a * area * __builtin_amdgcn_rcpf(rq5 * rq5);
        post = make_float4(gpp[0] * wv, gpp[1] * wv, gpp[2] * wv, 0.f);
      }
      cw = cwn;
      float4* kb = posts[kk & 1];
      kb[(ly + 1) * PPB_PAD + lx + 1] = post;
      __syncthreads();
      // footprint texel t of the 17x17 (two per thread for t < 33)
      const float w00 = bx * by, w10 = ax * by, w01 = bx * ay, w11 = ax * ay;
      if (mode == 1) {
        foot_texel<1>(kb, tid, w00, w10, w01, w11, tg, E, wd, acc, gcol, x0, y0, W, H, N);
        if (tid < PPB_FOOT - 256) foot_texel<1>(kb, tid + 256, w00, w10, w01, w11, tg, E, wd, acc, gcol, x0, y0, W, H, N);
      } else {
        foot_texel<2>(kb, tid, w00, w10, w01, w11, tg, E, wd, acc, gcol, x0, y0, W, H, N);
        if (tid < PPB_FOOT - 256) foot_texel<2>(kb, tid + 256, w00, w10, w01, w11, tg, E, wd, acc, gcol, x0, y0, W, H, N);
      }
    }
  } else if (scat) {
    for (int kk = 0; kk < ntap; ++kk) {
      const float4 u = taps[kk];
      const TapGeo tg = tap_geo(Rv, u);
      const float ax = tg.ax, ay = tg.ay, bx = 1.f - ax, by = 1.f - ay;
      const int xa = x + tg.ix, ya = y + tg.iy;
      const int xa_ = clampi(xa, 0, W - 1), xb_ = clampi(xa + 1, 0, W - 1);
      const int ya_ = clampi(ya, 0, H - 1), yb_ = clampi(ya + 1, 0, H - 1);
      const size_t i00 = (size_t)ya_ * W + xa_, i10 = (size_t)ya_ * W + xb_, i01 = (size_t)yb_ * W + xa_,
                   i11 = (size_t)yb_ * W + xb_;
      const float w00 = bx * by, w10 = ax * by, w01 = bx * ay, w11 = ax * ay;
      const float cq = w00 * pack[i00].w + w10 * pack[i10].w + w01 * pack[i01].w + w11 * pack[i11].w;
      const float rq = 0.5f * fabsf(cq);
      const float tk = clamp01((cq - cp4.w) * inv_ramp);
      const float a = clamp01(rq - tk * fmaxf(0.f, rq - rpv) - Rv * u.z + 0.5f);
      if (a == 0.f) continue;
      const float rq5 = fmaxf(rq, 0.5f);
      const float wv = a * area * __builtin_amdgcn_rcpf(rq5 * rq5);
      for (int c = 0; c < 3; ++c) {
        const float k = gpp[c] * wv;
        float* gc = gcol + c * N;
        atomicAdd(&gc[i00], k * w00);
        atomicAdd(&gc[i10], k * w10);
        atomicAdd(&gc[i01], k * w01);
        atomicAdd(&gc[i11], k * w11);
      }
    }
  }
  if (UNI && mode == 1) {
    __syncthreads();
    const int n2 = wd * wd;
    for (int i = tid; i < 3 * n2; i += 256) {
      const float v = acc[i];
      if (v != 0.f) {
        const int c = i / n2, t = i - c * n2, r = t / wd;
        const int gy = clampi(y0 - E + r, 0, H - 1), gx = clampi(x0 - E + t - r * wd, 0, W - 1);
        atomicAdd(&gcol[c * N + (size_t)gy * W + gx], v);
      }
    }
  }
  __syncthreads();  // the posts' last readers are done
  red[tid] = make_float2(gs, ga);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] = make_float2(red[tid].x + red[tid + o].x, red[tid].y + red[tid + o].y);
    __syncthreads();
  }
  if (tid == 0) partial[blockIdx.x] = red[0];
}

// block partials summed in a fixed order (deterministic), in double
__global__ void k_sum_partials(const float2* __restrict__ partial, int n, float* __restrict__ out) {
  __shared__ double sx[256], sy[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    a += partial[i].x;
    b += partial[i].y;
  }
  sx[threadIdx.x] = a;
  sy[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sx[threadIdx.x] += sx[threadIdx.x + o];
      sy[threadIdx.x] += sy[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = (float)sx[0];
    out[1] = (float)sy[0];
  }
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

hdof_status postfilter_reserve(hdof_ctx* ctx, const CamK& k, const LensK& l, const hdof_pp_params& pp,
                               hipStream_t st) {
  const int t = pp.tile;
  const size_t N = (size_t)k.W * k.H, NT = (size_t)cdiv(k.W, t) * cdiv(k.H, t);
  hdof_status s;
  if ((s = hdof_ensure(ctx->pp_pack, sizeof(float4) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_tile, sizeof(float) * NT)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_rad, sizeof(float) * NT)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_taps, sizeof(float4) * 256)) != HDOF_OK) return s;
  pp_taps_ensure(ctx, pp.n_taps, l, st);
  return HDOF_OK;
}

namespace {

// where one post-filter call keeps its intermediates
struct PPScratch {
  float4* pack;   // packed texels (rgb, signed CoC), one per pixel
  float* tile;    // per-tile maximum CoC radius
  float* rad;     // dilated tile radius (tiles other than 16 px)
  float4* taps;   // tap table, 256 entries
};

hdof_status postfilter_run(hdof_ctx* ctx, const PPScratch& S, const float* color, const float* depth,
                           const CamK& k, const LensK& l, const hdof_pp_params& pp, float* out, hipStream_t st,
                           bool packed, const PostFuse* fuse) {
  const int W = k.W, H = k.H, t = pp.tile;
  const int TW = cdiv(W, t), TH = cdiv(H, t);
  const int K = (int)ceil((double)pp.r_cap / t);
  if (!packed)
    hipLaunchKernelGGL(k_pp_pack, dim3(cdiv(W, 16) * cdiv(H, 16)), dim3(256), 0, st, color, depth, k, l, t,
                       S.pack, S.tile);
  if (t != 16)
    hipLaunchKernelGGL(k_pp_dilate, dim3(cdiv(TW, 64), TH), dim3(64), 0, st, (const float*)S.tile, TW,
                       TH, K, pp.r_cap, S.rad);
  hdof_prof_mark(ctx, 8, st);
  if (t == 16) {
    const bool sa = l.sa != 0.0f;
    FuseK fz{};
    if (fuse && fuse->untraced_only) {
      fz.out = fuse->out;
      // beside the trace (the overlapped frame) the four-wave form: the quad
      // form finishes sooner but takes the trace's issue slots on the way
      auto kern = sa ? k_pp_gather16<2, true> : k_pp_gather16<2, false>;
      if (fuse->done)
        hipExtLaunchKernelGGL(kern, dim3(TW * TH), dim3(256), 0, st, nullptr, fuse->done, 0,
                              (const float4*)S.pack, (const float*)S.tile, K, pp.r_cap, (const float4*)S.taps,
                              pp.n_taps, W, H, 1.0f / pp.bg_ramp_px, out, fz);
      else
        hipLaunchKernelGGL(kern, dim3(TW * TH), dim3(256), 0, st, (const float4*)S.pack,
                           (const float*)S.tile, K, pp.r_cap, (const float4*)S.taps, pp.n_taps, W, H,
                           1.0f / pp.bg_ramp_px, out, fz);
    } else if (fuse) {
      fz = FuseK{fuse->spp, fuse->rt.c_near, fuse->rt.c_far, fuse->rt.hit_ratio, 1.0f / fuse->cp.h_t,
                 fuse->cp.rt_override, fuse->out, fuse->pps,
                 fuse->pps && fuse->cp.spec_y > 0.0f ? 1.0f / fuse->cp.spec_y : 0.0f};
      auto kern = sa ? k_pp_gather16q<1, true> : k_pp_gather16q<1, false>;
      hipLaunchKernelGGL(kern, dim3((TW * TH + 3) / 4), dim3(256), 0, st, (const float4*)S.pack,
                         (const float*)S.tile, K, pp.r_cap, (const float4*)S.taps, pp.n_taps, W, H,
                         1.0f / pp.bg_ramp_px, out, fz);
    } else {
      auto kern = sa ? k_pp_gather16q<0, true> : k_pp_gather16q<0, false>;
      hipLaunchKernelGGL(kern, dim3((TW * TH + 3) / 4), dim3(256), 0, st, (const float4*)S.pack,
                         (const float*)S.tile, K, pp.r_cap, (const float4*)S.taps, pp.n_taps, W, H,
                         1.0f / pp.bg_ramp_px, out, fz);
    }
  } else {
    hipLaunchKernelGGL(k_pp_gather_any, dim3(cdiv(W, 16), cdiv(H, 16)), dim3(256), 0, st,
                       (const float4*)S.pack, (const float*)S.rad,
                       (const float4*)S.taps, pp.n_taps, W, H, t, 1.0f / pp.bg_ramp_px, out);
    if (fuse && !fuse->untraced_only) {
      HDOF_HIP(hipGetLastError());
      return launch_composite(ctx, color, out, depth, fuse->spp, fuse->rt, k, l, fuse->cp, fuse->out, st,
                              fuse->pps);
    }
  }
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

}  // namespace

hdof_status launch_postfilter(hdof_ctx* ctx, const float* color, const float* depth, const CamK& k,
                              const LensK& l, const hdof_pp_params& pp, float* out, hipStream_t st, bool packed,
                              const PostFuse* fuse) {
  hdof_status s;
  if ((s = postfilter_reserve(ctx, k, l, pp, st)) != HDOF_OK) return s;
  const PPScratch S{(float4*)ctx->pp_pack.p, (float*)ctx->pp_tile.p, (float*)ctx->pp_rad.p, (float4*)ctx->pp_taps.p};
  return postfilter_run(ctx, S, color, depth, k, l, pp, out, st, packed, fuse);
}

hdof_status launch_postfilter_batched(hdof_ctx* ctx, const float4* pack, const float* tile_r, int n_views,
                                      const BatchView* hviews, const void* views_dev, float* const* outs,
                                      const hdof_pp_params& pp, float* pp_out, hipStream_t st) {
  if (pp.tile != 16) return hdof_set_error(HDOF_ERR_INVALID_ARG, "batched gather: 16-pixel tiles only");
  PPBatch b{};
  b.n = n_views;
  const bool sa = hviews[0].l.sa != 0.0f;
  for (int v = 0; v < n_views; ++v) {
    if ((hviews[v].l.sa != 0.0f) != sa)
      return hdof_set_error(HDOF_ERR_UNSUPPORTED, "batched gather: one spherical aberration for every view");
    b.tile_base[v + 1] = b.tile_base[v] + cdiv(hviews[v].k.W, 16) * cdiv(hviews[v].k.H, 16);
    b.out[v] = outs[v];
  }
  const int K = (int)ceil((double)pp.r_cap / 16);
  auto kern = sa ? k_pp_gather16q_batch<true> : k_pp_gather16q_batch<false>;
  hipLaunchKernelGGL(kern, dim3((b.tile_base[n_views] + 3) / 4), dim3(256), 0, st, pack, tile_r, K, pp.r_cap,
                     (const float4*)ctx->pp_taps.p, pp.n_taps, 1.0f / pp.bg_ramp_px, pp_out,
                     (const BatchView*)views_dev, b);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

hdof_status launch_composite_traced_batched(hdof_ctx* ctx, const float* color, const float* pp, const float* depth,
                                            const uint8_t* spp, hdof_rt_bufs rt, int n_views,
                                            const BatchView* hviews, const void* views_dev, float* const* outs,
                                            const hdof_composite_params& cp, hipStream_t st) {
  (void)ctx;
  PPBatch b{};
  b.n = n_views;
  for (int v = 0; v < n_views; ++v) {
    b.blk_base[v + 1] = b.blk_base[v] + cdiv(hviews[v].k.W * hviews[v].k.H, HDOF_BATCH_PX_BLOCK);
    b.out[v] = outs[v];
  }
  const CompK a{color, pp, depth, spp, rt.c_near, rt.c_far, rt.hit_ratio, hviews[0].l, 0, 1.0f / cp.h_t,
                cp.rt_override, nullptr, 0.0f, nullptr};
  hipLaunchKernelGGL(k_composite_traced_batch, dim3(b.blk_base[n_views]), dim3(256), 0, st, a,
                     (const BatchView*)views_dev, b);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

// ---------------------------------------------------------------------------
// The post-filter without allocation: its intermediates live in `scratch`,
// one file-scope device array per device (tap table, tile radii, dilated
// tile radii, packed texels), sized for images of up to
// HDOF_POSTFILTER_NOALLOC_MAX_PX pixels.  In host code `scratch` names a
// host-side stand-in, never device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device when the library's first context on it is created.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t NA_TAPS_BYTES = 256 * sizeof(float4);
// tile radii at the smallest tile (4 px) of any W x H <= the maximum with
// W, H <= 16384: ceil(W/4) ceil(H/4) <= N/16 + (W + H)/4 + 1
constexpr size_t NA_TILES = (size_t)HDOF_POSTFILTER_NOALLOC_MAX_PX / 16 + 8193;
constexpr size_t NA_TILE_BYTES = (NA_TILES * sizeof(float) + 255) / 256 * 256;
constexpr size_t NA_BYTES = NA_TAPS_BYTES + 2 * NA_TILE_BYTES + sizeof(float4) * (size_t)HDOF_POSTFILTER_NOALLOC_MAX_PX;
static_assert(NA_BYTES == (size_t)HDOF_POSTFILTER_NOALLOC_BYTES, "header size of the no-alloc scratch");
constexpr int NA_MAX_DEVICES = 64;

std::mutex na_mu;
void* na_ptr[NA_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

hdof_status postfilter_noalloc_init(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= NA_MAX_DEVICES)
    return hdof_set_error(HDOF_ERR_UNSUPPORTED, "device %d beyond the %d the library tracks", device, NA_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(na_mu);
  if (!na_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return hdof_set_error(HDOF_ERR_HIP, "no-alloc scratch address on device %d: %s", device, hipGetErrorString(e));
    na_ptr[device] = p;
  }
  *out = na_ptr[device];
  return HDOF_OK;
}

hdof_status launch_postfilter_noalloc(hdof_ctx* ctx, const float* color, const float* depth, const CamK& k,
                                      const LensK& l, const hdof_pp_params& pp, float* out, hipStream_t st) {
  if ((size_t)k.W * (size_t)k.H > (size_t)HDOF_POSTFILTER_NOALLOC_MAX_PX)
    return hdof_set_error(HDOF_ERR_CAPACITY, "%dx%d exceeds the no-alloc post-filter's %d pixels", k.W, k.H,
                          HDOF_POSTFILTER_NOALLOC_MAX_PX);
  unsigned char* base = (unsigned char*)ctx->noalloc_scratch;
  if (!base) return hdof_set_error(HDOF_ERR_UNSUPPORTED, "the context holds no no-alloc scratch");
  const PPScratch S{(float4*)(base + NA_TAPS_BYTES + 2 * NA_TILE_BYTES), (float*)(base + NA_TAPS_BYTES),
                    (float*)(base + NA_TAPS_BYTES + NA_TILE_BYTES), (float4*)base};
  // the tap table is rebuilt every call: the array keeps whatever the last
  // call on this device left in it
  const int blades = l.blades >= 3 ? l.blades : 0;
  hipLaunchKernelGGL(k_pp_taps, dim3(1), dim3(256), 0, st, pp.n_taps, blades,
                     (double)l.rot_ht * 3.14159265358979323846, l.sa, S.taps);
  return postfilter_run(ctx, S, color, depth, k, l, pp, out, st, false, nullptr);
}

hdof_status launch_composite(hdof_ctx* ctx, const float* color, const float* pp, const float* depth,
                             const uint8_t* spp, hdof_rt_bufs rt, const CamK& k, const LensK& l,
                             const hdof_composite_params& cp, float* out, hipStream_t st, const float* pps,
                             bool sparse) {
  (void)ctx;
  const int N = k.W * k.H;
  const float inv_sy = pps && cp.spec_y > 0.0f ? 1.0f / cp.spec_y : 0.0f;
  const CompK a{color, pp, depth, spp, rt.c_near, rt.c_far, rt.hit_ratio, l, N, 1.0f / cp.h_t, cp.rt_override,
                pps, inv_sy, out};
  if (sparse)
    hipLaunchKernelGGL(k_composite_traced, dim3(cdiv(N, 256)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_composite, dim3(cdiv(N, 256)), dim3(256), 0, st, a);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

hdof_status launch_pp_spec(hdof_ctx* ctx, const float* ys, const uint8_t* spp, const CamK& k, const LensK& l,
                           const hdof_pp_params& pp, float* out, hipStream_t st) {
  const int W = k.W, H = k.H, t = pp.tile;
  const int K = (int)ceil((double)pp.r_cap / t);
  if (!ctx->pp_pack.p || !ctx->pp_tile.p || (t != 16 && !ctx->pp_rad.p))
    return hdof_set_error(HDOF_ERR_INVALID_ARG, "specular post-filter before the frame's post-filter preparation");
  hdof_status s;
  if ((s = hdof_ensure(ctx->pp_taps, sizeof(float4) * 256)) != HDOF_OK) return s;
  pp_taps_ensure(ctx, pp.n_taps, l, st);
  hipLaunchKernelGGL(k_pp_spec, dim3(cdiv(W, 8) * cdiv(H, 8)), dim3(256), 0, st, (const float4*)ctx->pp_pack.p, ys,
                     spp, (const float*)ctx->pp_tile.p, (const float*)ctx->pp_rad.p, t, K, pp.r_cap,
                     (const float4*)ctx->pp_taps.p, pp.n_taps, W, H, 1.0f / pp.bg_ramp_px, out);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

hdof_status launch_ppc_backward(hdof_ctx* ctx, const float* color, const float* depth, const uint8_t* spp,
                                hdof_rt_bufs rt, const CamK& k, const LensK& l, const hdof_pp_params& pp,
                                const hdof_composite_params& cp, const float* grad_out, float* grad_color,
                                float* grad_lens, hipStream_t st) {
  const int W = k.W, H = k.H, t = pp.tile;
  const size_t N = (size_t)W * H;
  const int TW = cdiv(W, t), TH = cdiv(H, t);
  const int K = (int)ceil((double)pp.r_cap / t);
  const dim3 grid(cdiv(W, 16), cdiv(H, 16));
  const int nblk = (int)(grid.x * grid.y);
  hdof_status s;
  if ((s = hdof_ensure(ctx->pp_pack, sizeof(float4) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_tile, sizeof(float) * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_rad, sizeof(float) * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_taps, sizeof(float4) * 256)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->ppb_args, sizeof(int) * 2 * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->ppb_partial, sizeof(float2) * (size_t)nblk)) != HDOF_OK) return s;
  pp_taps_ensure(ctx, pp.n_taps, l, st);
  int* tile_arg = (int*)ctx->ppb_args.p;
  int* rad_arg = tile_arg + (size_t)TW * TH;
  hipLaunchKernelGGL(k_ppb_pack, dim3(nblk), dim3(256), 0, st, color, depth, k, l, t, (float4*)ctx->pp_pack.p,
                     (float*)ctx->pp_tile.p, tile_arg);
  hipLaunchKernelGGL(k_ppb_dilate, dim3(cdiv(TW, 64), TH), dim3(64), 0, st, (const float*)ctx->pp_tile.p,
                     (const int*)tile_arg, TW, TH, K, pp.r_cap, (float*)ctx->pp_rad.p, rad_arg);
  hipLaunchKernelGGL(k_fill_f, dim3(cdiv(3 * (long)N, 256)), dim3(256), 0, st, grad_color, 3 * N, 0.0f);
  if (t == 16)
    hipLaunchKernelGGL(k_ppc_backward<true>, dim3(nblk), dim3(256), 0, st, (const float4*)ctx->pp_pack.p,
                       (const float*)ctx->pp_rad.p, (const int*)rad_arg, (const float4*)ctx->pp_taps.p, pp.n_taps,
                       W, H, t, 1.0f / pp.bg_ramp_px, l, k.spx, spp, (const float*)rt.c_near,
                       (const float*)rt.c_far, (const float*)rt.hit_ratio, 1.0f / cp.h_t, cp.rt_override,
                       grad_out, grad_color, (float2*)ctx->ppb_partial.p);
  else
    hipLaunchKernelGGL(k_ppc_backward<false>, dim3(nblk), dim3(256), 0, st, (const float4*)ctx->pp_pack.p,
                       (const float*)ctx->pp_rad.p, (const int*)rad_arg, (const float4*)ctx->pp_taps.p, pp.n_taps,
                       W, H, t, 1.0f / pp.bg_ramp_px, l, k.spx, spp, (const float*)rt.c_near,
                       (const float*)rt.c_far, (const float*)rt.hit_ratio, 1.0f / cp.h_t, cp.rt_override,
                       grad_out, grad_color, (float2*)ctx->ppb_partial.p);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const float2*)ctx->ppb_partial.p, nblk,
                     grad_lens);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}
