// postfilter.hip -- post-process gather DoF filter and the composite.
//
// k_pp_pack: colour + signed CoC packed into one float4 per pixel (one
//   16-byte load per bilinear texel in the gather) and the per-tile maximum
//   CoC radius.
// k_pp_dilate: gather radius per tile = min(r_cap, max radius over the tiles
//   within ceil(r_cap / tile) tiles).
// k_pp_gather: 16x4-pixel waves; golden-angle taps from a small table read
//   with wave-uniform loads; four float4 texels per tap from L1/L2 (the
//   packed image is written just before, so it is cache-resident); weights
//   recomputed per tap, nothing stored.
// k_composite: focus zone / near / far rules, one pass over the pixels.
#include "hdof_internal.h"

namespace {

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__global__ __launch_bounds__(256) void k_pp_pack(const float* __restrict__ color,
                                                 const float* __restrict__ depth, CamK k, LensK l,
                                                 int tile, float4* __restrict__ pack,
                                                 float* __restrict__ tile_r) {
  __shared__ float red[256];
  const int tid = threadIdx.x;
  const int x = blockIdx.x * 16 + (tid & 15), y = blockIdx.y * 16 + (tid >> 4);
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
// evaluated in double and stored as (ux, uy, |u|, 0)
__global__ void k_pp_taps(int n, float4* __restrict__ taps) {
  int k = threadIdx.x + 1;
  if (k > n) return;
  const double g = 3.14159265358979323846 * (3.0 - sqrt(5.0));
  double rr = sqrt((k - 0.5) / n);
  taps[k - 1] = make_float4((float)(rr * cos(k * g)), (float)(rr * sin(k * g)), (float)rr, 0.0f);
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


// UNI: the post-filter tile equals the 16x16 block, so the gather radius and
// with it every tap's integer offset and bilinear weights are uniform over
// the block (computed once per tap in scalar registers); only the four
// texel loads and the per-tap weight are per lane.  Blocks whose reach stays
// inside the image skip the clamp-to-edge.
template <bool UNI>
__global__ __launch_bounds__(256) void k_pp_gather(const float4* __restrict__ pack,
                                                   const float* __restrict__ rad,
                                                   const float4* __restrict__ taps, int n_taps,
                                                   int W, int H, int tile, float inv_ramp,
                                                   float* __restrict__ out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x0 = blockIdx.x * 16, y0 = blockIdx.y * 16;
  const int x = x0 + (lane & 15), y = y0 + wave * 4 + (lane >> 4);
  if (x >= W || y >= H) return;
  const size_t N = (size_t)W * H, p = (size_t)y * W + x;
  const int TW = (W + tile - 1) / tile;
  const float R = UNI ? rad[blockIdx.y * TW + blockIdx.x] : rad[(y / tile) * TW + x / tile];
  const float4 cp4 = pack[p];
  const float cp = cp4.w, rp = 0.5f * fabsf(cp);
  const float rp5 = fmaxf(rp, 0.5f);
  const float w0 = 1.0f / (rp5 * rp5);
  float ar = w0 * cp4.x, ag = w0 * cp4.y, ab = w0 * cp4.z, ws = w0;
  if (R > 0.0f) {
    const float area = R * R / (float)n_taps;
    const int reach = (int)ceilf(R) + 1;
    const bool interior = UNI && x0 - reach >= 0 && x0 + 15 + reach < W && y0 - reach >= 0 && y0 + 15 + reach < H;
    for (int kk = 0; kk < n_taps; ++kk) {
      const float4 u = taps[kk];  // (ux, uy, |u|, 0)
      // tap position relative to this pixel's texel grid: x + R u.x (the
      // +0.5 pixel centre and the -0.5 texel centre cancel)
      const float ox = R * u.x, oy = R * u.y;
      const float fx = floorf(ox), fy = floorf(oy);
      const float ax = ox - fx, ay = oy - fy;
      int xa = x + (int)fx, ya = y + (int)fy;
      int xb = xa + 1, yb = ya + 1;
      if (!interior) {
        xa = clampi(xa, 0, W - 1);
        xb = clampi(xb, 0, W - 1);
        ya = clampi(ya, 0, H - 1);
        yb = clampi(yb, 0, H - 1);
      }
      const float4 v00 = pack[(size_t)ya * W + xa], v10 = pack[(size_t)ya * W + xb];
      const float4 v01 = pack[(size_t)yb * W + xa], v11 = pack[(size_t)yb * W + xb];
      const float bx = 1.0f - ax, by = 1.0f - ay;
      const float w00 = bx * by, w10 = ax * by, w01 = bx * ay, w11 = ax * ay;
      const float sr = fmaf(w11, v11.x, fmaf(w01, v01.x, fmaf(w10, v10.x, w00 * v00.x)));
      const float sg = fmaf(w11, v11.y, fmaf(w01, v01.y, fmaf(w10, v10.y, w00 * v00.y)));
      const float sb = fmaf(w11, v11.z, fmaf(w01, v01.z, fmaf(w10, v10.z, w00 * v00.z)));
      const float cq = fmaf(w11, v11.w, fmaf(w01, v01.w, fmaf(w10, v10.w, w00 * v00.w)));
      const float rq = 0.5f * fabsf(cq);
      const float tk = clamp01((cq - cp) * inv_ramp);
      const float reff = rq - tk * fmaxf(0.0f, rq - rp);
      const float a = clamp01(reff + (0.5f - R * u.z));
      const float rq5 = fmaxf(rq, 0.5f);
      const float w = a * area * __frcp_rn(rq5 * rq5);
      ar = fmaf(w, sr, ar);
      ag = fmaf(w, sg, ag);
      ab = fmaf(w, sb, ab);
      ws += w;
    }
  }
  const float iw = 1.0f / ws;
  out[p] = ar * iw;
  out[N + p] = ag * iw;
  out[2 * N + p] = ab * iw;
}

__global__ void k_composite(const float* __restrict__ color, const float* __restrict__ pp,
                            const float* __restrict__ depth, const uint8_t* __restrict__ spp,
                            const float* __restrict__ cn, const float* __restrict__ cf,
                            const float* __restrict__ hr, LensK l, int N, float inv_ht, int rt_override,
                            float* __restrict__ out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const float c = coc_px(l, depth[p]);
  const float phi = clamp01(fabsf(c) - HDOF_SQRT2);
  const float nu = clamp01(fmaf(-c, 0.35355339059327376f, 0.5f));
  const bool traced = spp[p] > 0;
  const float h = hr[p];
  const float rho = traced ? 1.0f : 0.0f;
  const float beta = traced ? clamp01(1.0f - h * inv_ht) : 0.0f;
  for (int q = 0; q < 3; ++q) {
    size_t i = (size_t)q * N + p;
    float crt = h * cn[i] + (1.0f - h) * cf[i];
    float cpp = pp[i];
    float oof = nu * (rho * crt + (1.0f - rho) * cpp) + (1.0f - nu) * (beta * crt + (1.0f - beta) * cpp);
    float o = (1.0f - phi) * color[i] + phi * oof;
    if (rt_override && traced) o = crt;
    out[i] = o;
  }
}

// ---------------------------------------------------------------------------
// Adjoint of post-filter + composite (differentiable form).
// Reverse mode for the colour (the gather's transpose: every tap scatters
// its share back to its four bilinear texels with atomics), forward mode for
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
  float q = x.v / y.v, iy = 1.0f / y.v;
  return D3{q, (x.s - q * y.s) * iy, (x.a - q * y.a) * iy};
}
// clamp with zero slope outside the open interval (lo, hi)
__device__ inline D3 dclamp(D3 x, float lo, float hi) { return x.v <= lo ? dc(lo) : (x.v >= hi ? dc(hi) : x); }
__device__ inline D3 dmaxc(D3 x, float c) { return x.v > c ? x : dc(c); }
__device__ inline D3 dabs(D3 x) { return x.v >= 0.f ? x : D3{-x.v, -x.s, -x.a}; }

// pack (rgb, c) plus the CoC per unit aperture, tile max with its pixel
__global__ __launch_bounds__(256) void k_ppb_pack(const float* __restrict__ color, const float* __restrict__ depth,
                                                  CamK k, LensK l, int tile, float4* __restrict__ pack,
                                                  float* __restrict__ unit_coc, float* __restrict__ tile_r,
                                                  int* __restrict__ tile_arg) {
  __shared__ float red[256];
  __shared__ int redi[256];
  const int tid = threadIdx.x;
  const int x = blockIdx.x * 16 + (tid & 15), y = blockIdx.y * 16 + (tid >> 4);
  const size_t N = (size_t)k.W * k.H;
  float r = -1.0f;
  int idx = 0x7fffffff;
  if (x < k.W && y < k.H) {
    size_t p = (size_t)y * k.W + x;
    float u = (l.invS1 - 1.0f / depth[p]) * k.spx;
    float c = l.A * u;
    pack[p] = make_float4(color[p], color[N + p], color[2 * N + p], c);
    unit_coc[p] = u;
    r = 0.5f * fabsf(c);
    idx = (int)p;
  }
  red[tid] = r;
  redi[tid] = idx;
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;
  if ((tx % tile) == 0 && (ty % tile) == 0 && x < k.W && y < k.H) {
    float m = -1.0f;
    int mi = 0x7fffffff;
    for (int dy = 0; dy < tile; ++dy)
      for (int dx = 0; dx < tile; ++dx) {
        float v = red[(ty + dy) * 16 + tx + dx];
        int vi = redi[(ty + dy) * 16 + tx + dx];
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

__global__ __launch_bounds__(256) void k_ppc_backward(
    const float4* __restrict__ pack, const float* __restrict__ unit_coc, const float* __restrict__ rad,
    const int* __restrict__ rad_arg, const float4* __restrict__ taps, int n_taps, int W, int H, int tile,
    float inv_ramp, LensK l, float spx, const uint8_t* __restrict__ spp, const float* __restrict__ cn,
    const float* __restrict__ cf, const float* __restrict__ hr, float inv_ht, int rt_override,
    const float* __restrict__ g, float* __restrict__ gcol, float2* __restrict__ partial) {
  __shared__ float2 red[256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x = blockIdx.x * 16 + (lane & 15), y = blockIdx.y * 16 + wave * 4 + (lane >> 4);
  float gs = 0.0f, ga = 0.0f;
  const size_t N = (size_t)W * H;
  const float dcs = -l.A * spx * l.invS1 * l.invS1;  // dc/dS1 (every pixel)
  const bool inside = x < W && y < H;
  const size_t p = inside ? (size_t)y * W + x : 0;
  const bool traced = inside && spp[p] > 0;
  if (inside && !(rt_override && traced)) {
    const int TW = (W + tile - 1) / tile;
    const int ti = (y / tile) * TW + x / tile;
    const float4 cp4 = pack[p];
    const D3 cpv = dk(cp4.w, dcs, unit_coc[p]);
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
    D3 R = dc(rad[ti]);
    const int m = rad_arg[ti];
    if (m >= 0) {
      const float sg = pack[m].w >= 0.f ? 0.5f : -0.5f;
      R = dk(R.v, sg * dcs, sg * unit_coc[m]);
    }
    D3 nr = w0 * dc(cp4.x), ng = w0 * dc(cp4.y), nb = w0 * dc(cp4.z), den = w0;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const int ntap = R.v > 0.f ? n_taps : 0;
    for (int kk = 0; kk < ntap; ++kk) {
      const float4 u = taps[kk];
      const float gx = fmaf(R.v, u.x, px) - 0.5f, gy = fmaf(R.v, u.y, py) - 0.5f;
      const float fx0 = floorf(gx), fy0 = floorf(gy);
      const float ax = gx - fx0, ay = gy - fy0, bx = 1.f - ax, by = 1.f - ay;
      const int ix = (int)fx0, iy = (int)fy0;
      const int xa = min(max(ix, 0), W - 1), xb = min(max(ix + 1, 0), W - 1);
      const int ya = min(max(iy, 0), H - 1), yb = min(max(iy + 1, 0), H - 1);
      const size_t i00 = (size_t)ya * W + xa, i10 = (size_t)ya * W + xb, i01 = (size_t)yb * W + xa,
                   i11 = (size_t)yb * W + xb;
      const float4 v00 = pack[i00], v10 = pack[i10], v01 = pack[i01], v11 = pack[i11];
      const float w00 = bx * by, w10 = ax * by, w01 = bx * ay, w11 = ax * ay;
      // samples, their spatial slopes, and their motion with R
      const float dxs = u.x * R.s, dxa = u.x * R.a, dys = u.y * R.s, dya = u.y * R.a;
#define SAMPLE(c)                                                                       \
  const float s_##c = w00 * v00.c + w10 * v10.c + w01 * v01.c + w11 * v11.c;            \
  const float sx_##c = by * (v10.c - v00.c) + ay * (v11.c - v01.c);                      \
  const float sy_##c = bx * (v01.c - v00.c) + ax * (v11.c - v10.c);
      SAMPLE(x) SAMPLE(y) SAMPLE(z) SAMPLE(w)
#undef SAMPLE
      const float uq = w00 * unit_coc[i00] + w10 * unit_coc[i10] + w01 * unit_coc[i01] + w11 * unit_coc[i11];
      const D3 cq = dk(s_w, dcs + sx_w * dxs + sy_w * dys, uq + sx_w * dxa + sy_w * dya);
      const D3 rq = 0.5f * dabs(cq);
      const D3 tk = dclamp(inv_ramp * (cq - cpv), 0.f, 1.f);
      const D3 dpos = dmaxc(rq - rp, 0.f);
      const D3 reff = rq - tk * dpos;
      const D3 a = dclamp(reff - u.z * R + dc(0.5f), 0.f, 1.f);
      const D3 rq5 = dmaxc(rq, 0.5f);
      const D3 w = dquot(a * ((1.0f / (float)n_taps) * (R * R)), rq5 * rq5);
      nr = nr + w * dk(s_x, sx_x * dxs + sy_x * dys, sx_x * dxa + sy_x * dya);
      ng = ng + w * dk(s_y, sx_y * dxs + sy_y * dys, sx_y * dxa + sy_y * dya);
      nb = nb + w * dk(s_z, sx_z * dxs + sy_z * dys, sx_z * dxa + sy_z * dya);
      den = den + w;
    }
    // composite backward per channel; post-filter transpose for the colour
    const float gq[3] = {g[p], g[N + p], g[2 * N + p]};
    const D3 num[3] = {nr, ng, nb};
    const float cr[3] = {cp4.x, cp4.y, cp4.z};
    float gpp[3];
    const float iden = 1.0f / den.v;
    for (int c = 0; c < 3; ++c) {
      const float crt = h * cn[c * N + p] + (1.f - h) * cf[c * N + p];
      const D3 cpp = dquot(num[c], den);
      const D3 oof = crt * acoef + bcoef * cpp;
      const D3 out = (dc(1.f) - phi) * dc(cr[c]) + phi * oof;
      gs = fmaf(gq[c], out.s, gs);
      ga = fmaf(gq[c], out.a, ga);
      gpp[c] = gq[c] * phi.v * bcoef.v * iden;
      atomicAdd(&gcol[c * N + p], fmaf(gq[c], 1.f - phi.v, gpp[c] * w0.v));
    }
    if (gpp[0] != 0.f || gpp[1] != 0.f || gpp[2] != 0.f) {
      // second pass over the taps: the weights again (value only) and the scatter
      const float rpv = rp.v, area = R.v * R.v / (float)n_taps;
      for (int kk = 0; kk < ntap; ++kk) {
        const float4 u = taps[kk];
        const float gx = fmaf(R.v, u.x, px) - 0.5f, gy = fmaf(R.v, u.y, py) - 0.5f;
        const float fx0 = floorf(gx), fy0 = floorf(gy);
        const float ax = gx - fx0, ay = gy - fy0, bx = 1.f - ax, by = 1.f - ay;
        const int ix = (int)fx0, iy = (int)fy0;
        const int xa = min(max(ix, 0), W - 1), xb = min(max(ix + 1, 0), W - 1);
        const int ya = min(max(iy, 0), H - 1), yb = min(max(iy + 1, 0), H - 1);
        const size_t i00 = (size_t)ya * W + xa, i10 = (size_t)ya * W + xb, i01 = (size_t)yb * W + xa,
                     i11 = (size_t)yb * W + xb;
        const float w00 = bx * by, w10 = ax * by, w01 = bx * ay, w11 = ax * ay;
        const float cq = w00 * pack[i00].w + w10 * pack[i10].w + w01 * pack[i01].w + w11 * pack[i11].w;
        const float rq = 0.5f * fabsf(cq);
        const float tk = clamp01((cq - cp4.w) * inv_ramp);
        const float reff = rq - tk * fmaxf(0.f, rq - rpv);
        const float a = clamp01(reff - R.v * u.z + 0.5f);
        if (a == 0.f) continue;
        const float rq5 = fmaxf(rq, 0.5f);
        const float wv = a * area / (rq5 * rq5);
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
  }
  red[tid] = make_float2(gs, ga);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] = make_float2(red[tid].x + red[tid + o].x, red[tid].y + red[tid + o].y);
    __syncthreads();
  }
  if (tid == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
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

hdof_status launch_postfilter(hdof_ctx* ctx, const float* color, const float* depth, const CamK& k,
                              const LensK& l, const hdof_pp_params& pp, float* out, hipStream_t st) {
  const int W = k.W, H = k.H, t = pp.tile;
  const size_t N = (size_t)W * H;
  const int TW = cdiv(W, t), TH = cdiv(H, t);
  const int K = (int)ceil((double)pp.r_cap / t);
  hdof_status s;
  if ((s = hdof_ensure(ctx->pp_pack, sizeof(float4) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_tile, sizeof(float) * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_rad, sizeof(float) * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_taps, sizeof(float4) * 256)) != HDOF_OK) return s;
  if (ctx->pp_taps_n != pp.n_taps) {  // the table depends on the tap count only
    hipLaunchKernelGGL(k_pp_taps, dim3(1), dim3(256), 0, st, pp.n_taps, (float4*)ctx->pp_taps.p);
    ctx->pp_taps_n = pp.n_taps;
  }
  hipLaunchKernelGGL(k_pp_pack, dim3(cdiv(W, 16), cdiv(H, 16)), dim3(256), 0, st, color, depth, k, l, t,
                     (float4*)ctx->pp_pack.p, (float*)ctx->pp_tile.p);
  hipLaunchKernelGGL(k_pp_dilate, dim3(cdiv(TW, 64), TH), dim3(64), 0, st, (const float*)ctx->pp_tile.p, TW,
                     TH, K, pp.r_cap, (float*)ctx->pp_rad.p);
  hdof_prof_mark(ctx, 7, st);
  if (t == 16)
    hipLaunchKernelGGL(k_pp_gather<true>, dim3(cdiv(W, 16), cdiv(H, 16)), dim3(256), 0, st,
                       (const float4*)ctx->pp_pack.p, (const float*)ctx->pp_rad.p,
                       (const float4*)ctx->pp_taps.p, pp.n_taps, W, H, t, 1.0f / pp.bg_ramp_px, out);
  else
    hipLaunchKernelGGL(k_pp_gather<false>, dim3(cdiv(W, 16), cdiv(H, 16)), dim3(256), 0, st,
                       (const float4*)ctx->pp_pack.p, (const float*)ctx->pp_rad.p,
                       (const float4*)ctx->pp_taps.p, pp.n_taps, W, H, t, 1.0f / pp.bg_ramp_px, out);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

hdof_status launch_composite(hdof_ctx* ctx, const float* color, const float* pp, const float* depth,
                             const uint8_t* spp, hdof_rt_bufs rt, const CamK& k, const LensK& l,
                             const hdof_composite_params& cp, float* out, hipStream_t st) {
  (void)ctx;
  const int N = k.W * k.H;
  hipLaunchKernelGGL(k_composite, dim3(cdiv(N, 256)), dim3(256), 0, st, color, pp, depth, spp, rt.c_near,
                     rt.c_far, rt.hit_ratio, l, N, 1.0f / cp.h_t, cp.rt_override, out);
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
  hdof_status s;
  if ((s = hdof_ensure(ctx->pp_pack, sizeof(float4) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_tile, sizeof(float) * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_rad, sizeof(float) * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->pp_taps, sizeof(float4) * 256)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->ppb_unit, sizeof(float) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->ppb_args, sizeof(int) * 2 * (size_t)TW * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->ppb_partial, sizeof(float2) * (size_t)grid.x * grid.y)) != HDOF_OK) return s;
  if (ctx->pp_taps_n != pp.n_taps) {
    hipLaunchKernelGGL(k_pp_taps, dim3(1), dim3(256), 0, st, pp.n_taps, (float4*)ctx->pp_taps.p);
    ctx->pp_taps_n = pp.n_taps;
  }
  int* tile_arg = (int*)ctx->ppb_args.p;
  int* rad_arg = tile_arg + (size_t)TW * TH;
  hipLaunchKernelGGL(k_ppb_pack, grid, dim3(256), 0, st, color, depth, k, l, t, (float4*)ctx->pp_pack.p,
                     (float*)ctx->ppb_unit.p, (float*)ctx->pp_tile.p, tile_arg);
  hipLaunchKernelGGL(k_ppb_dilate, dim3(cdiv(TW, 64), TH), dim3(64), 0, st, (const float*)ctx->pp_tile.p,
                     (const int*)tile_arg, TW, TH, K, pp.r_cap, (float*)ctx->pp_rad.p, rad_arg);
  hipLaunchKernelGGL(k_fill_f, dim3(cdiv(3 * (long)N, 256)), dim3(256), 0, st, grad_color, 3 * N, 0.0f);
  hipLaunchKernelGGL(k_ppc_backward, grid, dim3(256), 0, st, (const float4*)ctx->pp_pack.p,
                     (const float*)ctx->ppb_unit.p, (const float*)ctx->pp_rad.p, (const int*)rad_arg,
                     (const float4*)ctx->pp_taps.p, pp.n_taps, W, H, t, 1.0f / pp.bg_ramp_px, l, k.spx, spp,
                     (const float*)rt.c_near, (const float*)rt.c_far, (const float*)rt.hit_ratio, 1.0f / cp.h_t,
                     cp.rt_override, grad_out, grad_color, (float2*)ctx->ppb_partial.p);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, (const float2*)ctx->ppb_partial.p,
                     (int)(grid.x * grid.y), grad_lens);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}
