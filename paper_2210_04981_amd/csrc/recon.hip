// recon.hip -- temporal reconstruction of the near and far ray-traced
// colours (paper, Reconstruction).
//
// Per traced pixel, an exponential moving average of the premultiplied near
// colour h C_tn with its hit ratio h, reprojected through the pixel's
// G-buffer surface point (screen-space motion) with a 1 % depth test, and of
// the premultiplied far colour (1 - h) C_tf with the hit ratio accumulated
// along the far path, reprojected through the far-weighted mean hit point of
// the pixel's rays (or the mean of its 8 neighbours' when it has no far
// hit).  The outputs replace c_near and c_far: near = N / Hn, far =
// F / (1 - Hf); the composite mixes them with the latest hit ratio.
// Untraced pixels keep their colours and leave no history.  One thread per
// pixel; the history is a ping-pong pair of 9-plane images in the context.
#include "hdof_internal.h"

namespace {

struct RecHist {
  const float* h;      // 9 planes of the previous frame
  const uint8_t* v;    // valid bytes
  CamK pk;             // previous camera (same size as the current frame)
  int valid;
};

// nearest pixel of world point X in camera pk (W x H), and its axial depth
__device__ inline bool reproj_nearest(const CamK& pk, V3 X, size_t& q, float& zc) {
  const V3 d = X - pk.e;
  zc = dot3(d, pk.w);
  if (!(zc > 0.0f)) return false;
  const float sxp = dot3(d, pk.r) / zc, syp = dot3(d, pk.u) / zc;
  const float fx = (sxp / pk.tx + 1.0f) * 0.5f * (float)pk.W;
  const float fy = (1.0f - syp / pk.ty) * 0.5f * (float)pk.H;
  const float px = floorf(fx), py = floorf(fy);
  if (!(px >= 0.0f && px < (float)pk.W && py >= 0.0f && py < (float)pk.H)) return false;
  q = (size_t)py * pk.W + (size_t)px;
  return true;
}

__global__ __launch_bounds__(256) void k_recon(CamK k, RecHist hi, const float* __restrict__ depth,
                                               const uint8_t* __restrict__ spp, const float* __restrict__ far_pos,
                                               const float* __restrict__ hit, float* __restrict__ cn,
                                               float* __restrict__ cf, float alpha, float* __restrict__ hout,
                                               uint8_t* __restrict__ vout) {
  const int W = k.W, H = k.H;
  const size_t N = (size_t)W * H;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int x = (int)(p % W), y = (int)(p / W);
  const float z = depth[p];
  hout[8 * N + p] = z;
  if (spp[p] == 0) {
    for (int c = 0; c < 8; ++c) hout[c * N + p] = 0.0f;
    vout[p] = 0;
    return;
  }
  const float h = hit[p];
  bool okn = false, okf = false;
  size_t qn = 0, qf = 0;
  if (hi.valid) {
    // near path: the G-buffer surface point
    const V3 v = pixel_dir(k, x, y);
    const V3 X = V3{fmaf(z, v.x, k.e.x), fmaf(z, v.y, k.e.y), fmaf(z, v.z, k.e.z)};
    float zc;
    if (reproj_nearest(hi.pk, X, qn, zc) && hi.v[qn]) okn = fabsf(hi.h[8 * N + qn] - zc) / zc <= 0.01f;
    // far path: the pixel's far-hit mean, else its neighbours'
    V3 Xf = V3{0.0f, 0.0f, 0.0f};
    bool have = false;
    if (far_pos[3 * N + p] > 0.0f) {
      Xf = V3{far_pos[p], far_pos[N + p], far_pos[2 * N + p]};
      have = true;
    } else {
      int cnt = 0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int xx = x + dx, yy = y + dy;
          if ((dx == 0 && dy == 0) || xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
          const size_t o = (size_t)yy * W + xx;
          if (spp[o] > 0 && far_pos[3 * N + o] > 0.0f) {
            Xf = Xf + V3{far_pos[o], far_pos[N + o], far_pos[2 * N + o]};
            ++cnt;
          }
        }
      if (cnt > 0) {
        const float ic = 1.0f / (float)cnt;
        Xf = V3{Xf.x * ic, Xf.y * ic, Xf.z * ic};
        have = true;
      }
    }
    float zf;
    if (have && reproj_nearest(hi.pk, Xf, qf, zf) && hi.v[qf]) okf = true;
  }
  const float a = alpha, b = 1.0f - alpha;
  const float Hn = okn ? fmaf(b, hi.h[3 * N + qn], a * h) : h;
  const float Hf = okf ? fmaf(b, hi.h[7 * N + qf], a * h) : h;
  for (int c = 0; c < 3; ++c) {
    const float cnc = cn[c * N + p], cfc = cf[c * N + p];
    const float Np = okn ? fmaf(b, hi.h[c * N + qn], a * h * cnc) : h * cnc;
    const float Fp = okf ? fmaf(b, hi.h[(4 + c) * N + qf], a * (1.0f - h) * cfc) : (1.0f - h) * cfc;
    cn[c * N + p] = Hn > 0.0f ? Np / Hn : cnc;
    cf[c * N + p] = 1.0f - Hf > 0.0f ? Fp / (1.0f - Hf) : cfc;
    hout[c * N + p] = Np;
    hout[(4 + c) * N + p] = Fp;
  }
  hout[3 * N + p] = Hn;
  hout[7 * N + p] = Hf;
  vout[p] = 1;
}

inline int cdiv(size_t a, int b) { return (int)((a + b - 1) / b); }

}  // namespace

hdof_status launch_recon(hdof_ctx* ctx, const CamK& k, const CamK* prev, const float* depth, const uint8_t* spp,
                         const float* far_pos, hdof_rt_bufs rt, float alpha, hipStream_t st) {
  const size_t N = (size_t)k.W * k.H;
  hdof_status s;
  for (int i = 0; i < 2; ++i) {
    if ((s = hdof_ensure(ctx->rec_hist[i], sizeof(float) * 9 * N)) != HDOF_OK) return s;
    if ((s = hdof_ensure(ctx->rec_valid[i], N)) != HDOF_OK) return s;
  }
  RecHist hi{};
  const int cur = ctx->rec_cur, nxt = 1 - cur;
  if (prev && ctx->rec_any && ctx->rec_w == prev->W && ctx->rec_h == prev->H && prev->W == k.W && prev->H == k.H) {
    hi.valid = 1;
    hi.h = (const float*)ctx->rec_hist[cur].p;
    hi.v = (const uint8_t*)ctx->rec_valid[cur].p;
    hi.pk = *prev;
  }
  hipLaunchKernelGGL(k_recon, dim3(cdiv(N, 256)), dim3(256), 0, st, k, hi, depth, spp, far_pos, rt.hit_ratio,
                     rt.c_near, rt.c_far, alpha, (float*)ctx->rec_hist[nxt].p, (uint8_t*)ctx->rec_valid[nxt].p);
  HDOF_HIP(hipGetLastError());
  ctx->rec_cur = nxt;
  ctx->rec_any = true;
  ctx->rec_w = k.W;
  ctx->rec_h = k.H;
  return HDOF_OK;
}
