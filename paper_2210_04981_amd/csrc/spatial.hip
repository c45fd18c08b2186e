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
#define SP_G 4  // taps per load group of the gather

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
  // the quad's counts first, then all of its values at once (a frame's ray
  // mask is uniform over its tiles, so a quad is traced wholly or not at all)
  size_t q[4];
  int sv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int x = rx * 32 + qx * 2 + (i & 1), y = ry * 32 + qy * 2 + (i >> 1);
    const bool in = x < I.W && y < I.H;
    q[i] = in ? (size_t)y * I.W + x : 0;
    sv[i] = in ? (int)I.spp[q[i]] : 0;
  }
  if ((sv[0] | sv[1] | sv[2] | sv[3]) != 0) {
    float hq[4], r[4], c[4][6];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      hq[i] = I.h[q[i]];
      r[i] = sp_radius(I, q[i], N);
      c[i][0] = I.cn[q[i]], c[i][1] = I.cn[N + q[i]], c[i][2] = I.cn[2 * N + q[i]];
      c[i][3] = I.cf[q[i]], c[i][4] = I.cf[N + q[i]], c[i][5] = I.cf[2 * N + q[i]];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (sv[i] == 0) continue;
      const float wn = (float)sv[i] * hq[i], wf = (float)sv[i] * (1.0f - hq[i]);
      a[0] = fmaf(wn, c[i][0], a[0]);
      a[1] = fmaf(wn, c[i][1], a[1]);
      a[2] = fmaf(wn, c[i][2], a[2]);
      a[3] += wn;
      a[4] = fmaf(wf, c[i][3], a[4]);
      a[5] = fmaf(wf, c[i][4], a[5]);
      a[6] = fmaf(wf, c[i][5], a[6]);
      a[7] += wf;
      a[8] += r[i];
      a[9] += 1.0f;
    }
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

// One 16x16-pixel block per 256 threads, each wave an 8x8 quadrant: the
// ray mask is uniform over its 8x8 tiles, so a wave is wholly traced or
// wholly untraced and the gather's lanes do not idle beside copying ones.
// spc = float(sqrt(pi / n_taps)), formed on the host in double.
// zero_untraced: write 0 for untraced pixels without reading them (the
// whole-frame path, whose untraced inputs are 0 by construction).
template <int VSRC>
__global__ __launch_bounds__(256) void k_sp_gather(SpIn I, const float4* __restrict__ lv,
                                                   const float4* __restrict__ taps, int n_taps, float spc,
                                                   SpVar var, float* __restrict__ cn_out,
                                                   float* __restrict__ cf_out, int zero_untraced) {
  const int W = I.W, H = I.H;
  const size_t N = (size_t)W * H;
  // blocks in launch order, round-robin over the XCDs: the traced pixels
  // cluster along a few silhouettes, and XCD-contiguous ranges would give
  // most of them to one XCD
  const int b = blockIdx.x, BW = (W + 15) >> 4;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int x = (b % BW) * 16 + (w & 1) * 8 + (l & 7), y = (b / BW) * 16 + (w >> 1) * 8 + (l >> 3);
  if (x >= W || y >= H) return;
  const size_t p = (size_t)y * W + x;
  const int s = I.spp[p];
  if (s == 0) {
    float c[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (!zero_untraced) {
      c[0] = I.cn[p], c[1] = I.cn[N + p], c[2] = I.cn[2 * N + p];
      c[3] = I.cf[p], c[4] = I.cf[N + p], c[5] = I.cf[2 * N + p];
    }
    cn_out[p] = c[0];
    cn_out[N + p] = c[1];
    cn_out[2 * N + p] = c[2];
    cf_out[p] = c[3];
    cf_out[N + p] = c[4];
    cf_out[2 * N + p] = c[5];
    return;
  }
  const float cn0 = I.cn[p], cn1 = I.cn[N + p], cn2 = I.cn[2 * N + p];
  const float cf0 = I.cf[p], cf1 = I.cf[N + p], cf2 = I.cf[2 * N + p];
  const float rp = sp_radius(I, p, N);
  // level: texels no wider than the taps' mean spacing r sqrt(pi / n)
  const float spacing = rp * spc;
  int L = 0;
  while (L < SP_LMAX && spacing >= (float)(2 << L)) ++L;
  const float hp = I.h[p], wn0 = (float)s * hp, wf0 = (float)s * (1.0f - hp);
  float An0 = wn0 * cn0, An1 = wn0 * cn1, An2 = wn0 * cn2, Bn = wn0;
  float Af0 = wf0 * cf0, Af1 = wf0 * cf1, Af2 = wf0 * cf2, Bf = wf0;
  const float fx0 = (float)x + 0.5f, fy0 = (float)y + 0.5f;
  // taps in groups of SP_G: every load of a group is issued before any of
  // its sums, so a wave waits once per group rather than once per tap
  if (L == 0) {
    for (int k0 = 0; k0 < n_taps; k0 += SP_G) {
      size_t q[SP_G];
      int sq[SP_G];
      float d[SP_G];
#pragma unroll
      for (int g = 0; g < SP_G; ++g) {
        const int k = min(k0 + g, n_taps - 1);
        const float4 u = taps[k];
        const int px = min(max((int)floorf(fmaf(rp, u.x, fx0)), 0), W - 1);
        const int py = min(max((int)floorf(fmaf(rp, u.y, fy0)), 0), H - 1);
        q[g] = (size_t)py * W + px;
        d[g] = rp * u.z;
        sq[g] = k0 + g < n_taps ? (int)I.spp[q[g]] : 0;
      }
      float r[SP_G], hq[SP_G], c[SP_G][6];
#pragma unroll
      for (int g = 0; g < SP_G; ++g) {
        r[g] = sp_radius(I, q[g], N);
        hq[g] = I.h[q[g]];
        c[g][0] = I.cn[q[g]], c[g][1] = I.cn[N + q[g]], c[g][2] = I.cn[2 * N + q[g]];
        c[g][3] = I.cf[q[g]], c[g][4] = I.cf[N + q[g]], c[g][5] = I.cf[2 * N + q[g]];
      }
#pragma unroll
      for (int g = 0; g < SP_G; ++g) {
        const float a = sq[g] > 0 ? clamp01(r[g] - d[g] + 0.5f) : 0.0f;
        const float wn = a * (float)sq[g] * hq[g], wf = a * (float)sq[g] * (1.0f - hq[g]);
        An0 = fmaf(wn, c[g][0], An0);
        An1 = fmaf(wn, c[g][1], An1);
        An2 = fmaf(wn, c[g][2], An2);
        Bn += wn;
        Af0 = fmaf(wf, c[g][3], Af0);
        Af1 = fmaf(wf, c[g][4], Af1);
        Af2 = fmaf(wf, c[g][5], Af2);
        Bf += wf;
      }
    }
  } else {
    const int WL = (W + (1 << L) - 1) >> L;
    const float4* lvl = lv + 3 * sp_level_offset(W, H, L);
    for (int k0 = 0; k0 < n_taps; k0 += SP_G) {
      float4 t0[SP_G], t1[SP_G], t2[SP_G];
      float d[SP_G];
#pragma unroll
      for (int g = 0; g < SP_G; ++g) {
        const int k = min(k0 + g, n_taps - 1);
        const float4 u = taps[k];
        const int px = min(max((int)floorf(fmaf(rp, u.x, fx0)), 0), W - 1);
        const int py = min(max((int)floorf(fmaf(rp, u.y, fy0)), 0), H - 1);
        const float4* tx = lvl + 3 * ((size_t)(py >> L) * WL + (px >> L));
        t0[g] = tx[0];
        t1[g] = tx[1];
        t2[g] = tx[2];
        d[g] = k0 + g < n_taps ? rp * u.z : INFINITY;  // a tap past the end accepts nothing
      }
#pragma unroll
      for (int g = 0; g < SP_G; ++g) {
        const bool any = t2[g].y > 0.0f;
        const float a = any ? clamp01(t2[g].x / t2[g].y - d[g] + 0.5f) : 0.0f;
        An0 = fmaf(a, t0[g].x, An0);
        An1 = fmaf(a, t0[g].y, An1);
        An2 = fmaf(a, t0[g].z, An2);
        Bn = fmaf(a, t0[g].w, Bn);
        Af0 = fmaf(a, t1[g].x, Af0);
        Af1 = fmaf(a, t1[g].y, Af1);
        Af2 = fmaf(a, t1[g].z, Af2);
        Bf = fmaf(a, t1[g].w, Bf);
      }
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

}  // namespace

size_t spatial_level_bytes(int W, int H) { return sizeof(float4) * 3 * sp_level_offset(W, H, SP_LMAX + 1); }

hdof_status spatial_reserve(hdof_ctx* ctx, int W, int H) {
  hdof_status s;
  if ((s = hdof_ensure(ctx->sp_levels, spatial_level_bytes(W, H))) != HDOF_OK) return s;
  return hdof_ensure(ctx->sp_taps, sizeof(float4) * 256);
}

hdof_status launch_spatial(hdof_ctx* ctx, int W, int H, const uint8_t* spp, hdof_rt_bufs in, const float* hacc,
                           const float* coc_nf, const float* variance, bool var_from_history,
                           const hdof_spatial_params& sp, float* cn_out, float* cf_out, hipStream_t st,
                           bool zero_untraced) {
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
  const int blocks = ((W + 15) >> 4) * ((H + 15) >> 4);
  const int zu = zero_untraced ? 1 : 0;
  const float4* taps = (const float4*)ctx->sp_taps.p;
  if (var_from_history) {
    var.m1 = (const float*)ctx->hist_m1.p;
    var.m2 = (const float*)ctx->hist_m2.p;
    var.fl = (const uint8_t*)ctx->hist_flags.p;
    hipLaunchKernelGGL(k_sp_gather<SP_VAR_HIST>, dim3(blocks), dim3(256), 0, st, I, (const float4*)lv, taps,
                       sp.n_taps, spc, var, cn_out, cf_out, zu);
  } else if (variance) {
    hipLaunchKernelGGL(k_sp_gather<SP_VAR_PLANE>, dim3(blocks), dim3(256), 0, st, I, (const float4*)lv, taps,
                       sp.n_taps, spc, var, cn_out, cf_out, zu);
  } else {
    hipLaunchKernelGGL(k_sp_gather<SP_VAR_NONE>, dim3(blocks), dim3(256), 0, st, I, (const float4*)lv, taps,
                       sp.n_taps, spc, var, cn_out, cf_out, zu);
  }
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}
