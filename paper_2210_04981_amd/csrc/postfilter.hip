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
