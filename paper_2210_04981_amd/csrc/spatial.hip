// spatial.hip -- spatial reconstruction of the near and far ray-traced
// colours (paper, Reconstruction, last paragraph).
//
// The near and far CoC sizes of a traced pixel, blended by its accumulated
// hit ratio, give the radius of a circular gather and the level of detail
// it samples; a sample whose CoC radius is smaller than its distance is
// rejected (with the post-filter's half-pixel ramp); a clamped variance
// estimate sets how far the gathered colour replaces the pixel's own.
//
// Levels 1..5 of a box pyramid over the traced pixels hold, per texel of
// 2^L x 2^L pixels, the sums of the near-ray-weighted near colour s h C_tn
// and its weight s h, the far pair s (1 - h) C_tf and s (1 - h), and the
// traced pixels' blended radii and count: 3 float4 per texel, levels
// concatenated.  k_sp_levels builds all five in one pass (a block reduces
// one 32 x 32 region through LDS); k_sp_gather runs one thread per pixel:
// untraced pixels copy their colours, traced ones gather N golden-angle
// taps from their level (level 0 reads the pixels themselves).
#include "hdof_internal.h"

#include <cmath>

#define SP_LMAX 5

namespace {

struct SpIn {
  const uint8_t* spp;
  const float *cn, *cf, *h, *hacc, *coc;  // hacc nullable: the latest hit ratio stands in
  float r_cap;
  int W, H;
};

__device__ inline float sp_radius(const SpIn& I, size_t q, size_t N) {
  const float Hq = I.hacc ? I.hacc[q] : I.h[q];
  return fminf(I.r_cap, 0.5f * fmaf(Hq, I.coc[q], (1.0f - Hq) * I.coc[N + q]));
}

// first texel of level L (>= 1) in the concatenated pyramid
__host__ __device__ inline size_t sp_level_offset(int W, int H, int L) {
  size_t off = 0;
  for (int l = 1; l < L; ++l) off += (size_t)((W + (1 << l) - 1) >> l) * (size_t)((H + (1 << l) - 1) >> l);
  return off;
}

__device__ inline void sp_emit(float4* __restrict__ lv, int W, int H, int L, int X, int Y, const float* a) {
  const int WL = (W + (1 << L) - 1) >> L, HL = (H + (1 << L) - 1) >> L;
  if (X >= WL || Y >= HL) return;
  float4* t = lv + 3 * (sp_level_offset(W, H, L) + (size_t)Y * WL + X);
  t[0] = make_float4(a[0], a[1], a[2], a[3]);
  t[1] = make_float4(a[4], a[5], a[6], a[7]);
  t[2] = make_float4(a[8], a[9], 0.0f, 0.0f);
}

// one 32x32-pixel region per block: thread t sums the 2x2 pixels of its
// level-1 texel, then levels 2..5 are 2x2 sums of the level below in LDS
__global__ __launch_bounds__(256) void k_sp_levels(SpIn I, float4* __restrict__ lv) {
  __shared__ float red[10][256];
  const int RW = (I.W + 31) >> 5;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int rx = b % RW, ry = b / RW;
  const int t = threadIdx.x, qx = t & 15, qy = t >> 4;
  const size_t N = (size_t)I.W * I.H;
  float a[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) a[i] = 0.0f;
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const int x = rx * 32 + qx * 2 + dx, y = ry * 32 + qy * 2 + dy;
      if (x >= I.W || y >= I.H) continue;
      const size_t q = (size_t)y * I.W + x;
      const int s = I.spp[q];
      if (s == 0) continue;
      const float hq = I.h[q], wn = (float)s * hq, wf = (float)s * (1.0f - hq);
      a[0] = fmaf(wn, I.cn[q], a[0]);
      a[1] = fmaf(wn, I.cn[N + q], a[1]);
      a[2] = fmaf(wn, I.cn[2 * N + q], a[2]);
      a[3] += wn;
      a[4] = fmaf(wf, I.cf[q], a[4]);
      a[5] = fmaf(wf, I.cf[N + q], a[5]);
      a[6] = fmaf(wf, I.cf[2 * N + q], a[6]);
      a[7] += wf;
      a[8] += sp_radius(I, q, N);
      a[9] += 1.0f;
    }
  sp_emit(lv, I.W, I.H, 1, rx * 16 + qx, ry * 16 + qy, a);
#pragma unroll
  for (int i = 0; i < 10; ++i) red[i][t] = a[i];
  int side = 16;
  for (int L = 2; L <= SP_LMAX; ++L) {
    __syncthreads();
    const int ns = side >> 1;
    const bool act = t < ns * ns;
    const int ix = t % ns, iy = t / ns;
    float c[10];
    if (act) {
      const int i00 = (2 * iy) * side + 2 * ix;
#pragma unroll
      for (int i = 0; i < 10; ++i) c[i] = (red[i][i00] + red[i][i00 + 1]) + (red[i][i00 + side] + red[i][i00 + side + 1]);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int i = 0; i < 10; ++i) red[i][t] = c[i];
      sp_emit(lv, I.W, I.H, L, rx * ns + ix, ry * ns + iy, c);
    }
    side = ns;
  }
}

// golden-angle taps u_k = sqrt((k - 0.5)/n) (cos k g, sin k g), g = pi (3 - sqrt 5),
// evaluated in double and stored as (ux, uy, |u|, 0)
__global__ void k_sp_taps(int n, float4* __restrict__ taps) {
  const int k = threadIdx.x + 1;
  if (k > n) return;
  const double g = 3.14159265358979323846 * (3.0 - sqrt(5.0));
  const double rr = sqrt((k - 0.5) / n);
  taps[k - 1] = make_float4((float)(rr * cos(k * g)), (float)(rr * sin(k * g)), (float)rr, 0.0f);
}

// variance source of the clamp weight
enum { SP_VAR_NONE = 0, SP_VAR_PLANE = 1, SP_VAR_HIST = 2 };
struct SpVar {
  const float* v;                // SP_VAR_PLANE: +inf = no estimate yet
  const float *m1, *m2;          // SP_VAR_HIST: luminance moments and flags
  const uint8_t* fl;
  float v_clamp;
};

// spc = float(sqrt(pi / n_taps)), formed on the host in double
template <int VSRC>
__global__ __launch_bounds__(256) void k_sp_gather(SpIn I, const float4* __restrict__ lv,
                                                   const float4* __restrict__ taps, int n_taps, float spc,
                                                   SpVar var, float* __restrict__ cn_out,
                                                   float* __restrict__ cf_out) {
  const int W = I.W, H = I.H;
  const size_t N = (size_t)W * H;
  const size_t p = (size_t)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (p >= N) return;
  const float cn0 = I.cn[p], cn1 = I.cn[N + p], cn2 = I.cn[2 * N + p];
  const float cf0 = I.cf[p], cf1 = I.cf[N + p], cf2 = I.cf[2 * N + p];
  const int s = I.spp[p];
  if (s == 0) {
    cn_out[p] = cn0;
    cn_out[N + p] = cn1;
    cn_out[2 * N + p] = cn2;
    cf_out[p] = cf0;
    cf_out[N + p] = cf1;
    cf_out[2 * N + p] = cf2;
    return;
  }
  const int x = (int)(p % W), y = (int)(p / W);
  const float rp = sp_radius(I, p, N);
  // level: texels no wider than the taps' mean spacing r sqrt(pi / n)
  const float spacing = rp * spc;
  int L = 0;
  while (L < SP_LMAX && spacing >= (float)(2 << L)) ++L;
  const float hp = I.h[p], wn0 = (float)s * hp, wf0 = (float)s * (1.0f - hp);
  float An0 = wn0 * cn0, An1 = wn0 * cn1, An2 = wn0 * cn2, Bn = wn0;
  float Af0 = wf0 * cf0, Af1 = wf0 * cf1, Af2 = wf0 * cf2, Bf = wf0;
  const float fx0 = (float)x + 0.5f, fy0 = (float)y + 0.5f;
  if (L == 0) {
    for (int k = 0; k < n_taps; ++k) {
      const float4 u = taps[k];
      const int px = min(max((int)floorf(fmaf(rp, u.x, fx0)), 0), W - 1);
      const int py = min(max((int)floorf(fmaf(rp, u.y, fy0)), 0), H - 1);
      const size_t q = (size_t)py * W + px;
      const int sq = I.spp[q];
      if (sq == 0) continue;
      const float a = clamp01(sp_radius(I, q, N) - rp * u.z + 0.5f);
      const float hq = I.h[q], wn = a * (float)sq * hq, wf = a * (float)sq * (1.0f - hq);
      An0 = fmaf(wn, I.cn[q], An0);
      An1 = fmaf(wn, I.cn[N + q], An1);
      An2 = fmaf(wn, I.cn[2 * N + q], An2);
      Bn += wn;
      Af0 = fmaf(wf, I.cf[q], Af0);
      Af1 = fmaf(wf, I.cf[N + q], Af1);
      Af2 = fmaf(wf, I.cf[2 * N + q], Af2);
      Bf += wf;
    }
  } else {
    const int WL = (W + (1 << L) - 1) >> L;
    const float4* lvl = lv + 3 * sp_level_offset(W, H, L);
    for (int k = 0; k < n_taps; ++k) {
      const float4 u = taps[k];
      const int px = min(max((int)floorf(fmaf(rp, u.x, fx0)), 0), W - 1);
      const int py = min(max((int)floorf(fmaf(rp, u.y, fy0)), 0), H - 1);
      const float4* tx = lvl + 3 * ((size_t)(py >> L) * WL + (px >> L));
      const float4 t2 = tx[2];
      if (!(t2.y > 0.0f)) continue;
      const float4 t0 = tx[0], t1 = tx[1];
      const float a = clamp01(t2.x / t2.y - rp * u.z + 0.5f);
      An0 = fmaf(a, t0.x, An0);
      An1 = fmaf(a, t0.y, An1);
      An2 = fmaf(a, t0.z, An2);
      Bn = fmaf(a, t0.w, Bn);
      Af0 = fmaf(a, t1.x, Af0);
      Af1 = fmaf(a, t1.y, Af1);
      Af2 = fmaf(a, t1.z, Af2);
      Bf = fmaf(a, t1.w, Bf);
    }
  }
  float lam = 1.0f;
  if (VSRC == SP_VAR_PLANE) {
    const float v = var.v[p];
    if (!isinf(v)) lam = clamp01(v / var.v_clamp);
  } else if (VSRC == SP_VAR_HIST) {
    const uint8_t f = var.fl[p];
    if (!(f & HDOF_HIST_NEW)) {
      const float m1 = var.m1[p];
      const float v = (f & HDOF_HIST_VALID) ? fmaxf(0.0f, fmaf(-m1, m1, var.m2[p])) : 0.0f;
      lam = clamp01(v / var.v_clamp);
    }
  }
  const float in_ = Bn > 0.0f ? 1.0f / Bn : 0.0f, if_ = Bf > 0.0f ? 1.0f / Bf : 0.0f;
  const float gn0 = Bn > 0.0f ? An0 * in_ : cn0, gn1 = Bn > 0.0f ? An1 * in_ : cn1, gn2 = Bn > 0.0f ? An2 * in_ : cn2;
  const float gf0 = Bf > 0.0f ? Af0 * if_ : cf0, gf1 = Bf > 0.0f ? Af1 * if_ : cf1, gf2 = Bf > 0.0f ? Af2 * if_ : cf2;
  cn_out[p] = fmaf(lam, gn0 - cn0, cn0);
  cn_out[N + p] = fmaf(lam, gn1 - cn1, cn1);
  cn_out[2 * N + p] = fmaf(lam, gn2 - cn2, cn2);
  cf_out[p] = fmaf(lam, gf0 - cf0, cf0);
  cf_out[N + p] = fmaf(lam, gf1 - cf1, cf1);
  cf_out[2 * N + p] = fmaf(lam, gf2 - cf2, cf2);
}

inline int cdiv(size_t a, int b) { return (int)((a + b - 1) / b); }

}  // namespace

size_t spatial_level_bytes(int W, int H) { return sizeof(float4) * 3 * sp_level_offset(W, H, SP_LMAX + 1); }

hdof_status spatial_reserve(hdof_ctx* ctx, int W, int H) {
  hdof_status s;
  if ((s = hdof_ensure(ctx->sp_levels, spatial_level_bytes(W, H))) != HDOF_OK) return s;
  return hdof_ensure(ctx->sp_taps, sizeof(float4) * 256);
}

hdof_status launch_spatial(hdof_ctx* ctx, int W, int H, const uint8_t* spp, hdof_rt_bufs in, const float* hacc,
                           const float* coc_nf, const float* variance, bool var_from_history,
                           const hdof_spatial_params& sp, float* cn_out, float* cf_out, hipStream_t st) {
  hdof_status s;
  if ((s = spatial_reserve(ctx, W, H)) != HDOF_OK) return s;
  if (ctx->sp_taps_n != sp.n_taps) {  // the table depends on the tap count only
    hipLaunchKernelGGL(k_sp_taps, dim3(1), dim3(256), 0, st, sp.n_taps, (float4*)ctx->sp_taps.p);
    ctx->sp_taps_n = sp.n_taps;
  }
  const SpIn I{spp, in.c_near, in.c_far, in.hit_ratio, hacc, coc_nf, sp.r_cap, W, H};
  float4* lv = (float4*)ctx->sp_levels.p;
  const int regions = ((W + 31) >> 5) * ((H + 31) >> 5);
  hipLaunchKernelGGL(k_sp_levels, dim3(regions), dim3(256), 0, st, I, lv);
  SpVar var{variance, nullptr, nullptr, nullptr, sp.v_clamp};
  const float spc = (float)std::sqrt(3.14159265358979323846 / (double)sp.n_taps);
  const size_t N = (size_t)W * H;
  const float4* taps = (const float4*)ctx->sp_taps.p;
  if (var_from_history) {
    var.m1 = (const float*)ctx->hist_m1.p;
    var.m2 = (const float*)ctx->hist_m2.p;
    var.fl = (const uint8_t*)ctx->hist_flags.p;
    hipLaunchKernelGGL(k_sp_gather<SP_VAR_HIST>, dim3(cdiv(N, 256)), dim3(256), 0, st, I, (const float4*)lv, taps,
                       sp.n_taps, spc, var, cn_out, cf_out);
  } else if (variance) {
    hipLaunchKernelGGL(k_sp_gather<SP_VAR_PLANE>, dim3(cdiv(N, 256)), dim3(256), 0, st, I, (const float4*)lv, taps,
                       sp.n_taps, spc, var, cn_out, cf_out);
  } else {
    hipLaunchKernelGGL(k_sp_gather<SP_VAR_NONE>, dim3(cdiv(N, 256)), dim3(256), 0, st, I, (const float4*)lv, taps,
                       sp.n_taps, spc, var, cn_out, cf_out);
  }
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}
