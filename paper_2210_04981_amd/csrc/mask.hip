// mask.hip -- adaptive ray mask and temporally accumulated luminance variance.
//
// k_mask_score: one block per 16x16 pixel tile.  The tile plus an apron of
// (Gaussian radius + 1) pixels of depth and normal is staged in LDS with
// clamp-to-edge, blurred separably (x then y), Sobel-filtered, scored, and
// the per-pixel count reduced to the mask-tile maxima (mask tiles divide 16,
// so no mask tile straddles a block).  The variance history is reprojected
// in the same pass when a previous camera is given.
// k_mask_rows / k_mask_rowscan / k_mask_write: per-pixel counts are constant
// over a mask tile, so the row-major exclusive scan over pixels reduces to a
// scan over tile rows; the device-side total is written last.
// Tile 0 scales the mask resolution with the frame's maximum CoC: the score
// pass also forms the tile maxima for 4-, 8- and 16-pixel tiles and each
// block's largest CoC radius, k_mask_pick reduces those to the frame's
// maximum R and picks the tile edge (4 below 16 px, 8 below 32 px, else
// 16: about R / 2), and the later passes read it from device memory, so the
// choice never reaches the host.
#include <utility>

#include "hdof_internal.h"

#define MT 16          // pixels per block edge
#define MAX_GR 6       // max Gaussian radius (sigma <= 2)
#define MAX_AP (MAX_GR + 1)
#define MAX_IN (MT + 2 * MAX_AP)
#define BL (MT + 2)    // blurred region edge (Sobel apron 1)

namespace {

struct MaskK {
  float taps[2 * MAX_GR + 1];
  int gr;
  float inv_tz, inv_tn, inv_tv;
  int spp_max, tile, dilate;
  float coc_scale, inv_s1;  // tile 0: the CoC of a depth, coc_scale (inv_s1 - 1/z)
};

// tile 0: the tile-maximum grids of the three candidate tile edges and each
// score block's largest CoC radius
struct MaskAuto {
  int *tm4, *tm8, *tm16;
  float* blk_r;
};

__device__ inline void emit_tile_max(int t, const int (*sr)[MT], int tx, int ty, int x, int y, int W,
                                     int* __restrict__ tile_max) {
  if ((tx % t) == 0 && (ty % t) == 0) {
    int mx = 0;
    for (int dy = 0; dy < t; ++dy)
      for (int dx = 0; dx < t; ++dx) mx = max(mx, sr[ty + dy][tx + dx]);
    const int TW = (W + t - 1) / t;
    tile_max[(y / t) * TW + x / t] = mx;
  }
}

struct HistIn {
  const float* m1;
  const float* m2;
  const uint8_t* flags;
  const float* z;
  int PW, PH;
  int valid;  // 0: no history (first frame, camera cut, size change)
  CamK pk;
};

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <int GR>
__device__ __forceinline__ void mask_score_block(const float* __restrict__ depth, const float* __restrict__ normal,
                                                 const CamK& k, const MaskK& mk, const HistIn& hi,
                                                 float* __restrict__ rep_m1, float* __restrict__ rep_m2,
                                                 uint8_t* __restrict__ rep_flags, float* __restrict__ rep_z,
                                                 int* __restrict__ tile_max, const MaskAuto& au, int lb) {
  // (depth, nx, ny, nz) of one pixel per float4; all extents compile-time
  constexpr int AP = GR + 1, NIN = MT + 2 * AP;
  __shared__ float4 in[NIN][NIN];
  __shared__ float4 xb[NIN][BL];
  __shared__ float4 yb[BL][BL];
  __shared__ int sr[MT][MT];
  const int W = k.W, H = k.H;
  const size_t N = (size_t)W * H;
  const int BX = (W + MT - 1) / MT;
  const int x0 = (lb % BX) * MT, y0 = (lb / BX) * MT;
  const int tid = threadIdx.x;
  // stage depth (clamped to zmax) and normal with clamp-to-edge
  for (int i = tid; i < NIN * NIN; i += 256) {
    const int ly = i / NIN, lx = i - ly * NIN;
    const int gx = clampi(x0 - AP + lx, 0, W - 1), gy = clampi(y0 - AP + ly, 0, H - 1);
    const size_t p = (size_t)gy * W + gx;
    in[ly][lx] = make_float4(fminf(depth[p], HDOF_ZMAX), normal[p], normal[N + p], normal[2 * N + p]);
  }
  __syncthreads();
  // x pass on every staged row for the 18 columns the Sobel needs; a column
  // outside the image takes the value of the clamped column
  for (int i = tid; i < NIN * BL; i += 256) {
    const int ly = i / BL, ox = i - ly * BL;
    const int lx0 = clampi(x0 - 1 + ox, 0, W - 1) - x0 + 1;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int t = 0; t <= 2 * GR; ++t) {
      const float4 v = in[ly][lx0 + t];
      const float w = mk.taps[t];
      a.x = fmaf(w, v.x, a.x);
      a.y = fmaf(w, v.y, a.y);
      a.z = fmaf(w, v.z, a.z);
      a.w = fmaf(w, v.w, a.w);
    }
    xb[ly][ox] = a;
  }
  __syncthreads();
  for (int i = tid; i < BL * BL; i += 256) {
    const int oy = i / BL, ox = i - oy * BL;
    const int ly0 = clampi(y0 - 1 + oy, 0, H - 1) - y0 + 1;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int t = 0; t <= 2 * GR; ++t) {
      const float4 v = xb[ly0 + t][ox];
      const float w = mk.taps[t];
      a.x = fmaf(w, v.x, a.x);
      a.y = fmaf(w, v.y, a.y);
      a.z = fmaf(w, v.z, a.z);
      a.w = fmaf(w, v.w, a.w);
    }
    yb[oy][ox] = a;
  }
  __syncthreads();
  const int tx = tid & 15, ty = tid >> 4;
  const int x = x0 + tx, y = y0 + ty;
  int s_raw = 0;
  float rc = 0.0f;  // CoC radius (tile 0)
  if (x < W && y < H) {
    // Sobel: yb index = local + 1
    const float4 a00 = yb[ty][tx], a10 = yb[ty][tx + 1], a20 = yb[ty][tx + 2];
    const float4 a01 = yb[ty + 1][tx], a21 = yb[ty + 1][tx + 2];
    const float4 a02 = yb[ty + 2][tx], a12 = yb[ty + 2][tx + 1], a22 = yb[ty + 2][tx + 2];
    const float zb = yb[ty + 1][tx + 1].x;
#define SOBEL(c)                                                                      \
  const float gx_##c = (a20.c - a00.c) + 2.0f * (a21.c - a01.c) + (a22.c - a02.c);    \
  const float gy_##c = (a02.c - a00.c) + 2.0f * (a12.c - a10.c) + (a22.c - a20.c);    \
  const float g2_##c = fmaf(gx_##c, gx_##c, gy_##c * gy_##c);
    SOBEL(x) SOBEL(y) SOBEL(z) SOBEL(w)
#undef SOBEL
    const float gz = sqrtf(g2_x) / (8.0f * fmaxf(zb, 1e-3f));
    const float gn = sqrtf(g2_y + g2_z + g2_w) * 0.125f;
    // reprojected variance
    const size_t p = (size_t)y * W + x;
    float V = 0.0f, a1 = 0.0f, a2 = 0.0f;
    uint8_t fl = 0;
    if (hi.valid) {
      float z = depth[p];
      V3 v = pixel_dir(k, x, y);
      V3 X = V3{fmaf(z, v.x, k.e.x), fmaf(z, v.y, k.e.y), fmaf(z, v.z, k.e.z)};
      V3 d = X - hi.pk.e;
      float zc = dot3(d, hi.pk.w);
      if (zc > 0.0f) {
        float sxp = dot3(d, hi.pk.r) / zc, syp = dot3(d, hi.pk.u) / zc;
        float fx = (sxp / hi.pk.tx + 1.0f) * 0.5f * (float)hi.PW;
        float fy = (1.0f - syp / hi.pk.ty) * 0.5f * (float)hi.PH;
        float px = floorf(fx), py = floorf(fy);
        if (px >= 0.0f && px < (float)hi.PW && py >= 0.0f && py < (float)hi.PH) {
          size_t q = (size_t)py * hi.PW + (size_t)px;
          uint8_t pf = hi.flags[q];
          if (pf & HDOF_HIST_VALID) {
            float rel = fabsf(hi.z[q] - zc) / zc;
            if (rel <= 0.01f) {
              a1 = hi.m1[q];
              a2 = hi.m2[q];
              fl = pf;
            }
          }
        }
      }
      if (fl & HDOF_HIST_VALID) V = (fl & HDOF_HIST_NEW) ? INFINITY : fmaxf(0.0f, fmaf(-a1, a1, a2));
    }
    if (rep_m1) {  // NULL: nothing will read the reprojected history
      rep_m1[p] = a1;
      rep_m2[p] = a2;
      rep_flags[p] = fl;
      rep_z[p] = depth[p];  // the history depth, should these planes become the history
    }
    float m = fmaxf(gz * mk.inv_tz, fmaxf(gn * mk.inv_tn, V * mk.inv_tv));
    if (m >= 1.0f) s_raw = (int)ceilf(fminf(m, (float)mk.spp_max));
    if (mk.tile == 0) rc = 0.5f * fabsf(mk.coc_scale * (mk.inv_s1 - 1.0f / depth[p]));
  }
  sr[ty][tx] = s_raw;
  __syncthreads();
  if (x >= W || y >= H) {
    // nothing to emit; the CoC reduction below still needs every lane
  } else if (mk.tile > 0) {
    emit_tile_max(mk.tile, sr, tx, ty, x, y, W, tile_max);
  } else {
    emit_tile_max(4, sr, tx, ty, x, y, W, au.tm4);
    emit_tile_max(8, sr, tx, ty, x, y, W, au.tm8);
    emit_tile_max(16, sr, tx, ty, x, y, W, au.tm16);
  }
  if (mk.tile == 0) {
    __shared__ float wr[4];
    for (int o = 32; o > 0; o >>= 1) rc = fmaxf(rc, __shfl_xor(rc, o));
    if ((tid & 63) == 0) wr[tid >> 6] = rc;
    __syncthreads();
    if (tid == 0) au.blk_r[lb] = fmaxf(fmaxf(wr[0], wr[1]), fmaxf(wr[2], wr[3]));
  }
}

// blocks in XCD-contiguous order: the halo rows a block stages are mostly
// in the L2 of its own XCD already
template <int GR>
__global__ __launch_bounds__(256) void k_mask_score(const float* __restrict__ depth,
                                                    const float* __restrict__ normal, CamK k, MaskK mk,
                                                    HistIn hi, float* __restrict__ rep_m1,
                                                    float* __restrict__ rep_m2,
                                                    uint8_t* __restrict__ rep_flags, float* __restrict__ rep_z,
                                                    int* __restrict__ tile_max, MaskAuto au) {
  const int nb = ((k.W + MT - 1) / MT) * ((k.H + MT - 1) / MT);
  mask_score_block<GR>(depth, normal, k, mk, hi, rep_m1, rep_m2, rep_flags, rep_z, tile_max, au,
                       xcd_block(blockIdx.x, nb));
}

// The batched form's masks (fixed mask tiles), one launch per pass over
// every view: view v's 16x16 score blocks start at blk[v], its tiles at
// tile[v], its tile rows at row[v] and its blocks of HDOF_BATCH_PX_BLOCK
// pixels at pix[v] ([n] the totals); its planes at its px_base.  No view
// carries a history.
struct MaskBatch {
  int n;
  int blk[HDOF_MAX_VIEWS + 1], tile[HDOF_MAX_VIEWS + 1], row[HDOF_MAX_VIEWS + 1], pix[HDOF_MAX_VIEWS + 1];
};

template <int GR>
__global__ __launch_bounds__(256) void k_mask_score_batch(const float* __restrict__ depth,
                                                          const float* __restrict__ normal,
                                                          const BatchView* __restrict__ views, MaskK mk,
                                                          int* __restrict__ tile_max, MaskBatch mb) {
  const int g = xcd_block(blockIdx.x, mb.blk[mb.n]);
  const int v = batch_view_of(mb.blk, mb.n, g);
  const size_t pb = (size_t)views[v].px_base;
  HistIn hi{};
  hi.valid = 0;
  mask_score_block<GR>(depth + pb, normal + 3 * pb, views[v].k, mk, hi, nullptr, nullptr, nullptr, nullptr,
                       tile_max + mb.tile[v], MaskAuto{}, g - mb.blk[v]);
}

// tile 0: the frame's largest CoC radius R over the score blocks' maxima,
// tile edge 4 (R < 16), 8 (R < 32) or 16
__global__ __launch_bounds__(1024) void k_mask_pick(const float* __restrict__ blk_r, int nb, int* __restrict__ tsel) {
  __shared__ float wr[16];
  const int tid = threadIdx.x;
  float r = 0.0f;
  for (int i = tid; i < nb; i += 1024) r = fmaxf(r, blk_r[i]);
  for (int o = 32; o > 0; o >>= 1) r = fmaxf(r, __shfl_xor(r, o));
  if ((tid & 63) == 0) wr[tid >> 6] = r;
  __syncthreads();
  if (tid == 0) {
    float R = 0.0f;
    for (int i = 0; i < 16; ++i) R = fmaxf(R, wr[i]);
    tsel[0] = R < 16.0f ? 4 : (R < 32.0f ? 8 : 16);
  }
}

// the tile edge in force: the launch's, or the one k_mask_pick chose
__device__ inline int mask_tile_of(int t, const int* __restrict__ tsel) { return tsel ? *tsel : t; }

// per tile row: dilated tile values, x-prefix of (value * tile width), row sum
// (tile 0: launched for the rows of 4-pixel tiles; rows past the chosen
// tile edge's grid exit)
__device__ __forceinline__ void mask_rows_block(const int* __restrict__ tile_max, int W, int H, int t, int dil,
                                                int* __restrict__ tile_dil, int* __restrict__ xpref,
                                                int* __restrict__ rowsum, int* __restrict__ rowtot, int ty) {
  __shared__ int part[4];
  const int TW = (W + t - 1) / t, TH = (H + t - 1) / t;
  const int tid = threadIdx.x;
  const int chunk = (TW + 255) / 256;
  const int lo = tid * chunk, hi = min(TW, lo + chunk);
  int local = 0;
  for (int tx = lo; tx < hi; ++tx) {
    int m = 0;
    for (int dy = -dil; dy <= dil; ++dy) {
      int yy = ty + dy;
      if (yy < 0 || yy >= TH) continue;
      for (int dx = -dil; dx <= dil; ++dx) {
        int xx = tx + dx;
        if (xx < 0 || xx >= TW) continue;
        m = max(m, tile_max[yy * TW + xx]);
      }
    }
    tile_dil[ty * TW + tx] = m;
    local += m * min(t, W - tx * t);
  }
  // inclusive scan of the threads' sums: within each wave by shuffles,
  // then the four wave totals
  const int lane = tid & 63, wave = tid >> 6;
  int incl = local;
  for (int o = 1; o < 64; o <<= 1) {
    const int n = __shfl_up(incl, o);
    if (lane >= o) incl += n;
  }
  if (lane == 63) part[wave] = incl;
  __syncthreads();
  for (int w = 0; w < wave; ++w) incl += part[w];
  const int row = part[0] + part[1] + part[2] + part[3];
  int run = incl - local;
  for (int tx = lo; tx < hi; ++tx) {
    xpref[ty * TW + tx] = run;
    run += tile_dil[ty * TW + tx] * min(t, W - tx * t);
  }
  if (tid == 255) {
    rowsum[ty] = row;
    rowtot[ty] = row * min(t, H - ty * t);
  }
}

__global__ __launch_bounds__(256) void k_mask_rows(const int* __restrict__ tile_max, int W, int H,
                                                   int t, int dil, int* __restrict__ tile_dil,
                                                   int* __restrict__ xpref, int* __restrict__ rowsum,
                                                   int* __restrict__ rowtot, const int* __restrict__ tsel,
                                                   MaskAuto au) {
  t = mask_tile_of(t, tsel);
  if (tsel) tile_max = t == 4 ? au.tm4 : (t == 8 ? au.tm8 : au.tm16);
  if ((int)blockIdx.x >= (H + t - 1) / t) return;
  mask_rows_block(tile_max, W, H, t, dil, tile_dil, xpref, rowsum, rowtot, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_mask_rows_batch(const int* __restrict__ tile_max,
                                                         const BatchView* __restrict__ views, int t, int dil,
                                                         int* __restrict__ tile_dil, int* __restrict__ xpref,
                                                         int* __restrict__ rowsum, int* __restrict__ rowtot,
                                                         MaskBatch mb) {
  const int v = batch_view_of(mb.row, mb.n, blockIdx.x);
  const int tb = mb.tile[v], rb = mb.row[v];
  mask_rows_block(tile_max + tb, views[v].k.W, views[v].k.H, t, dil, tile_dil + tb, xpref + tb, rowsum + rb,
                  rowtot + rb, blockIdx.x - rb);
}

// exclusive scan over tile rows (one block), total to the caller's buffer
__device__ __forceinline__ void mask_rowscan_block(const int* __restrict__ rowtot, int TH, int* __restrict__ ybase,
                                                   int* __restrict__ total) {
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  const int chunk = (TH + 1023) / 1024;
  const int lo = tid * chunk, hi = min(TH, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += rowtot[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - s;
  for (int i = lo; i < hi; ++i) {
    ybase[i] = run;
    run += rowtot[i];
  }
  if (tid == 1023) *total = part[1023];
}

__global__ void k_mask_rowscan(const int* __restrict__ rowtot, int TH, int* __restrict__ ybase,
                               int* __restrict__ total, int H, int t, const int* __restrict__ tsel) {
  if (tsel) TH = (H + *tsel - 1) / *tsel;
  mask_rowscan_block(rowtot, TH, ybase, total);
}

// one block per view
__global__ void k_mask_rowscan_batch(const int* __restrict__ rowtot, int* __restrict__ ybase,
                                     int* __restrict__ totals, MaskBatch mb) {
  const int v = blockIdx.x, rb = mb.row[v];
  mask_rowscan_block(rowtot + rb, mb.row[v + 1] - rb, ybase + rb, totals + v);
}

__global__ void k_mask_write(int W, int H, int t, const int* __restrict__ tile_dil,
                             const int* __restrict__ xpref, const int* __restrict__ rowsum,
                             const int* __restrict__ ybase, uint8_t* __restrict__ spp,
                             int* __restrict__ offsets, const int* __restrict__ tsel) {
  int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W) return;
  t = mask_tile_of(t, tsel);
  const int TW = (W + t - 1) / t;
  int tx = x / t, ty = y / t;
  int S = tile_dil[ty * TW + tx];
  size_t p = (size_t)y * W + x;
  spp[p] = (uint8_t)S;
  offsets[p] = ybase[ty] + (y - ty * t) * rowsum[ty] + xpref[ty * TW + tx] + (x - tx * t) * S;
}

// the batched form's counts and offsets, HDOF_BATCH_PX_BLOCK pixels per block
__global__ __launch_bounds__(256) void k_mask_write_batch(const BatchView* __restrict__ views, int t,
                                                          const int* __restrict__ tile_dil,
                                                          const int* __restrict__ xpref,
                                                          const int* __restrict__ rowsum,
                                                          const int* __restrict__ ybase, uint8_t* __restrict__ spp,
                                                          int* __restrict__ offsets, MaskBatch mb) {
  const int v = batch_view_of(mb.pix, mb.n, blockIdx.x);
  const int W = views[v].k.W, N = W * views[v].k.H;
  const size_t pb = (size_t)views[v].px_base;
  const int TW = (W + t - 1) / t, tb = mb.tile[v], rb = mb.row[v];
  const int p0 = (blockIdx.x - mb.pix[v]) * HDOF_BATCH_PX_BLOCK;
  for (int i = threadIdx.x; i < HDOF_BATCH_PX_BLOCK; i += blockDim.x) {
    const int p = p0 + i;
    if (p >= N) break;
    const int x = p % W, y = p / W, tx = x / t, ty = y / t;
    const int S = tile_dil[tb + ty * TW + tx];
    spp[pb + p] = (uint8_t)S;
    offsets[pb + p] = ybase[rb + ty] + (y - ty * t) * rowsum[rb + ty] + xpref[tb + ty * TW + tx] + (x - tx * t) * S;
  }
}

// Whole frames: the same write with the tile-row scan done per block, one
// block per 256 columns of one tile row (the block sums the row totals
// before its tile row; the last tile row's first block also writes the
// total), and the ray queue written here instead of by the trace's queue
// fill (pixel index per entry, entries outside [0, cap) dropped; the
// trace's work counters cleared).  Launched over the tile rows of the
// launch's tile edge t (tile 0: 4, the smallest); with the edge chosen on
// the device, blocks past its tile rows exit.
__global__ __launch_bounds__(256) void k_mask_write_queue(int W, int H, int t, int TH,
                                                          const int* __restrict__ tile_dil,
                                                          const int* __restrict__ xpref,
                                                          const int* __restrict__ rowsum,
                                                          const int* __restrict__ rowtot, uint8_t* __restrict__ spp,
                                                          int* __restrict__ offsets, int* __restrict__ total,
                                                          int* __restrict__ queue, long cap, int* __restrict__ counter,
                                                          const int* __restrict__ tsel) {
  __shared__ int2 red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tsel) {
    t = *tsel;
    TH = (H + t - 1) / t;
  }
  const int ty = blockIdx.y;
  if (ty >= TH) return;
  if (blockIdx.x == 0 && ty == 0)
    for (int i = tid; i < 8 * HDOF_SEG_STRIDE; i += 256) counter[i] = 0;
  int before = 0, all = 0;
  for (int i = tid; i < TH; i += 256) {
    const int v = rowtot[i];
    if (i < ty) before += v;
    all += v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    before += __shfl_xor(before, o);
    all += __shfl_xor(all, o);
  }
  if (lane == 0) red[wave] = make_int2(before, all);
  __syncthreads();
  const int ybase = red[0].x + red[1].x + red[2].x + red[3].x;
  if (blockIdx.x == 0 && ty == TH - 1 && tid == 0) *total = red[0].y + red[1].y + red[2].y + red[3].y;
  const int x = blockIdx.x * blockDim.x + tid;
  if (x >= W) return;
  const int TW = (W + t - 1) / t, tx = x / t;
  const int S = tile_dil[ty * TW + tx];
  const int rs = rowsum[ty];
  const int o0 = ybase + xpref[ty * TW + tx] + (x - tx * t) * S;
  const int y1 = min(H, (ty + 1) * t);
  for (int y = ty * t; y < y1; ++y) {
    const size_t p = (size_t)y * W + x;
    const int o = o0 + (y - ty * t) * rs;
    spp[p] = (uint8_t)S;
    offsets[p] = o;
    for (int j = 0; j < S; ++j)
      if ((long)o + j >= 0 && (long)o + j < cap) queue[o + j] = (int)p;
  }
}

// history update after the trace
__global__ void k_var_update(int N, float alpha, const uint8_t* __restrict__ spp,
                             const float* __restrict__ depth, const float* __restrict__ ybar,
                             const float* __restrict__ y2bar, const float* __restrict__ rm1,
                             const float* __restrict__ rm2, const uint8_t* __restrict__ rfl,
                             float* __restrict__ m1, float* __restrict__ m2, uint8_t* __restrict__ fl,
                             float* __restrict__ hz) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  float a1 = rm1[p], a2 = rm2[p];
  uint8_t f = rfl[p];
  if (spp[p] > 0) {
    if (f & HDOF_HIST_VALID) {
      a1 = fmaf(alpha, ybar[p], (1.0f - alpha) * a1);
      a2 = fmaf(alpha, y2bar[p], (1.0f - alpha) * a2);
      f = HDOF_HIST_VALID;
    } else {
      a1 = ybar[p];
      a2 = y2bar[p];
      f = HDOF_HIST_VALID | HDOF_HIST_NEW;
    }
  }
  m1[p] = a1;
  m2[p] = a2;
  fl[p] = f;
  hz[p] = depth[p];
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

// tile-grid sizes of a frame: tile 0 reserves for the 4-pixel grid (the
// largest) plus the 8- and 16-pixel maxima grids
static size_t grid_tiles(int W, int H, int t) { return (size_t)cdiv(W, t) * cdiv(H, t); }

hdof_status mask_reserve(hdof_ctx* ctx, int W, int H, const hdof_mask_params& mp) {
  const size_t N = (size_t)W * H;
  const int t = mp.tile > 0 ? mp.tile : 4;
  const size_t tiles = grid_tiles(W, H, t), TH = cdiv(H, t);
  const size_t extra = mp.tile > 0 ? 0 : grid_tiles(W, H, 8) + grid_tiles(W, H, 16);
  const size_t blocks = (size_t)cdiv(W, MT) * cdiv(H, MT);
  hdof_status s;
  if ((s = hdof_ensure(ctx->mask_tile, sizeof(int) * (tiles + extra))) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_tile_dil, sizeof(int) * tiles)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_xpref, sizeof(int) * tiles)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_rowsum, sizeof(int) * 2 * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_ybase, sizeof(int) * TH)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_auto, sizeof(float) * (blocks + 1))) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->rep_m1, sizeof(float) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->rep_m2, sizeof(float) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->rep_z, sizeof(float) * N)) != HDOF_OK) return s;
  return hdof_ensure(ctx->rep_flags, N);
}

// the score pass's constants; Gaussian taps exp(-i^2 / 2 sigma^2), radius
// floor(3 sigma + 0.5), normalised
static MaskK make_maskk(const hdof_mask_params& mp, const LensK* lens) {
  MaskK mk;
  const int gr = (int)floor(3.0 * mp.sigma + 0.5);
  mk.gr = gr;  // above MAX_GR the launchers refuse the parameters
  if (gr <= MAX_GR) {
    double tw[2 * MAX_GR + 1], sum = 0.0;
    for (int i = -gr; i <= gr; ++i) sum += (tw[i + gr] = exp(-(double)(i * i) / (2.0 * mp.sigma * mp.sigma)));
    for (int i = 0; i <= 2 * gr; ++i) mk.taps[i] = (float)(tw[i] / sum);
  }
  mk.inv_tz = 1.0f / mp.tau_depth;
  mk.inv_tn = 1.0f / mp.tau_normal;
  mk.inv_tv = 1.0f / mp.tau_var;
  mk.spp_max = mp.spp_max;
  mk.tile = mp.tile;
  mk.dilate = mp.dilate;
  mk.coc_scale = lens ? lens->coc_scale : 0.0f;
  mk.inv_s1 = lens ? lens->invS1 : 0.0f;
  return mk;
}

hdof_status launch_mask(hdof_ctx* ctx, const float* depth, const float* normal, const CamK& k,
                        const CamK* prev, const hdof_mask_params& mp, uint8_t* spp, int32_t* offsets,
                        int32_t* total, hipStream_t st, int* queue, long cap, int* counter, const LensK* lens,
                        bool write_rep) {
  const int W = k.W, H = k.H;
  const bool scaled = mp.tile == 0;
  if (scaled && !lens) return hdof_set_error(HDOF_ERR_INVALID_ARG, "mask tile 0 (scaled by the CoC) needs the lens");
  const int t = scaled ? 4 : mp.tile;  // the grid the launches are sized for
  const int TH = cdiv(H, t);
  const MaskK mk = make_maskk(mp, lens);
  const int gr = mk.gr;
  hdof_status s;
  if ((s = mask_reserve(ctx, W, H, mp)) != HDOF_OK) return s;
  HistIn hi{};
  hi.valid = 0;
  if (prev && ctx->hist_any && ctx->hist_w == prev->W && ctx->hist_h == prev->H) {
    hi.valid = 1;
    hi.m1 = (const float*)ctx->hist_m1.p;
    hi.m2 = (const float*)ctx->hist_m2.p;
    hi.flags = (const uint8_t*)ctx->hist_flags.p;
    hi.z = (const float*)ctx->hist_z.p;
    hi.PW = prev->W;
    hi.PH = prev->H;
    hi.pk = *prev;
  }
  ctx->rep_w = W;
  ctx->rep_h = H;
  ctx->rep_valid = write_rep;
  int* rowsum = (int*)ctx->mask_rowsum.p;
  int* rowtot = rowsum + TH;
  const int nblk = cdiv(W, MT) * cdiv(H, MT);
  MaskAuto au{};
  const int* tsel = nullptr;
  if (scaled) {
    au.tm4 = (int*)ctx->mask_tile.p;
    au.tm8 = au.tm4 + grid_tiles(W, H, 4);
    au.tm16 = au.tm8 + grid_tiles(W, H, 8);
    au.blk_r = (float*)ctx->mask_auto.p;
    tsel = (const int*)(au.blk_r + nblk);
  }
  {
    const dim3 g(nblk), b(256);
    float* r1 = write_rep ? (float*)ctx->rep_m1.p : nullptr;
    float* r2 = write_rep ? (float*)ctx->rep_m2.p : nullptr;
    uint8_t* rf = write_rep ? (uint8_t*)ctx->rep_flags.p : nullptr;
    float* rz = write_rep ? (float*)ctx->rep_z.p : nullptr;
    int* tm = (int*)ctx->mask_tile.p;
    switch (gr) {
#define CASE(R) \
  case R: hipLaunchKernelGGL(k_mask_score<R>, g, b, 0, st, depth, normal, k, mk, hi, r1, r2, rf, rz, tm, au); break;
      CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
      default: return hdof_set_error(HDOF_ERR_INVALID_ARG, "Gaussian radius %d above %d", gr, MAX_GR);
    }
  }
  if (scaled) hipLaunchKernelGGL(k_mask_pick, dim3(1), dim3(1024), 0, st, (const float*)au.blk_r, nblk, (int*)tsel);
  hipLaunchKernelGGL(k_mask_rows, dim3(TH), dim3(256), 0, st, (const int*)ctx->mask_tile.p, W, H, t,
                     mp.dilate, (int*)ctx->mask_tile_dil.p, (int*)ctx->mask_xpref.p, rowsum, rowtot, tsel, au);
  if (queue) {
    hipLaunchKernelGGL(k_mask_write_queue, dim3(cdiv(W, 256), TH), dim3(256), 0, st, W, H, t, TH,
                       (const int*)ctx->mask_tile_dil.p, (const int*)ctx->mask_xpref.p, (const int*)rowsum,
                       (const int*)rowtot, spp, offsets, total, queue, cap, counter, tsel);
  } else {
    hipLaunchKernelGGL(k_mask_rowscan, dim3(1), dim3(1024), 0, st, (const int*)rowtot, TH,
                       (int*)ctx->mask_ybase.p, total, H, t, tsel);
    hipLaunchKernelGGL(k_mask_write, dim3(cdiv(W, 256), H), dim3(256), 0, st, W, H, t,
                       (const int*)ctx->mask_tile_dil.p, (const int*)ctx->mask_xpref.p,
                       (const int*)rowsum, (const int*)ctx->mask_ybase.p, spp, offsets, tsel);
  }
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

static MaskBatch mask_batch_of(int n_views, const BatchView* hv, int t) {
  MaskBatch mb{};
  mb.n = n_views;
  for (int v = 0; v < n_views; ++v) {
    const int W = hv[v].k.W, H = hv[v].k.H;
    mb.blk[v + 1] = mb.blk[v] + cdiv(W, MT) * cdiv(H, MT);
    mb.tile[v + 1] = mb.tile[v] + cdiv(W, t) * cdiv(H, t);
    mb.row[v + 1] = mb.row[v] + cdiv(H, t);
    mb.pix[v + 1] = mb.pix[v] + cdiv((long)W * H, HDOF_BATCH_PX_BLOCK);
  }
  return mb;
}

hdof_status mask_reserve_batched(hdof_ctx* ctx, int n_views, const BatchView* hviews, const hdof_mask_params& mp) {
  if (mp.tile <= 0) return HDOF_OK;
  const MaskBatch mb = mask_batch_of(n_views, hviews, mp.tile);
  const size_t tiles = (size_t)mb.tile[n_views], rows = (size_t)mb.row[n_views];
  hdof_status s;
  if ((s = hdof_ensure(ctx->mask_tile, sizeof(int) * tiles)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_tile_dil, sizeof(int) * tiles)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_xpref, sizeof(int) * tiles)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->mask_rowsum, sizeof(int) * 2 * rows)) != HDOF_OK) return s;
  return hdof_ensure(ctx->mask_ybase, sizeof(int) * rows);
}

hdof_status launch_mask_batched(hdof_ctx* ctx, const float* depth, const float* normal, int n_views,
                                const BatchView* hviews, const void* views_dev, const hdof_mask_params& mp,
                                uint8_t* spp, int32_t* offsets, int32_t* totals, hipStream_t st) {
  if (mp.tile <= 0) return hdof_set_error(HDOF_ERR_INVALID_ARG, "batched masks: fixed mask tiles only");
  const int t = mp.tile;
  const MaskK mk = make_maskk(mp, nullptr);
  const MaskBatch mb = mask_batch_of(n_views, hviews, t);
  hdof_status s;
  if ((s = mask_reserve_batched(ctx, n_views, hviews, mp)) != HDOF_OK) return s;
  const BatchView* vd = (const BatchView*)views_dev;
  int* rowsum = (int*)ctx->mask_rowsum.p;
  int* rowtot = rowsum + mb.row[n_views];
  switch (mk.gr) {
#define CASE(R)                                                                                                  \
  case R:                                                                                                        \
    hipLaunchKernelGGL(k_mask_score_batch<R>, dim3(mb.blk[n_views]), dim3(256), 0, st, depth, normal, vd, mk,   \
                       (int*)ctx->mask_tile.p, mb);                                                             \
    break;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
    default: return hdof_set_error(HDOF_ERR_INVALID_ARG, "Gaussian radius %d above %d", mk.gr, MAX_GR);
  }
  hipLaunchKernelGGL(k_mask_rows_batch, dim3(mb.row[n_views]), dim3(256), 0, st, (const int*)ctx->mask_tile.p, vd,
                     t, mp.dilate, (int*)ctx->mask_tile_dil.p, (int*)ctx->mask_xpref.p, rowsum, rowtot, mb);
  hipLaunchKernelGGL(k_mask_rowscan_batch, dim3(n_views), dim3(1024), 0, st, (const int*)rowtot,
                     (int*)ctx->mask_ybase.p, totals, mb);
  hipLaunchKernelGGL(k_mask_write_batch, dim3(mb.pix[n_views]), dim3(256), 0, st, vd, t,
                     (const int*)ctx->mask_tile_dil.p, (const int*)ctx->mask_xpref.p, (const int*)rowsum,
                     (const int*)ctx->mask_ybase.p, spp, offsets, mb);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

hdof_status var_update_prepare(hdof_ctx* ctx, const CamK& k, float alpha, const float* depth, VarFuse* vf,
                               bool in_place) {
  const size_t N = (size_t)k.W * k.H;
  hdof_status s;
  if (!ctx->rep_valid || ctx->rep_w != k.W || ctx->rep_h != k.H)
    return hdof_set_error(HDOF_ERR_INVALID_ARG,
                          "variance update without a ray mask of the same frame size");
  if (in_place) {
    float* r1 = (float*)ctx->rep_m1.p;
    float* r2 = (float*)ctx->rep_m2.p;
    uint8_t* rf = (uint8_t*)ctx->rep_flags.p;
    *vf = VarFuse{alpha, depth, r1, r2, rf, r1, r2, rf, (float*)ctx->rep_z.p, 0, 1};
    return HDOF_OK;
  }
  if ((s = hdof_ensure(ctx->hist_m1, sizeof(float) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->hist_m2, sizeof(float) * N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->hist_flags, N)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->hist_z, sizeof(float) * N)) != HDOF_OK) return s;
  *vf = VarFuse{alpha, depth, (const float*)ctx->rep_m1.p, (const float*)ctx->rep_m2.p,
                (const uint8_t*)ctx->rep_flags.p, (float*)ctx->hist_m1.p, (float*)ctx->hist_m2.p,
                (uint8_t*)ctx->hist_flags.p, (float*)ctx->hist_z.p};
  ctx->hist_w = k.W;
  ctx->hist_h = k.H;
  ctx->hist_any = true;
  return HDOF_OK;
}

void history_swap(hdof_ctx* ctx) {
  std::swap(ctx->hist_m1, ctx->rep_m1);
  std::swap(ctx->hist_m2, ctx->rep_m2);
  std::swap(ctx->hist_flags, ctx->rep_flags);
  std::swap(ctx->hist_z, ctx->rep_z);
  ctx->hist_w = ctx->rep_w;
  ctx->hist_h = ctx->rep_h;
  ctx->hist_any = true;
  ctx->rep_valid = false;  // these planes now hold the old history, no reprojection
}

hdof_status launch_var_update(hdof_ctx* ctx, const CamK& k, float alpha, const uint8_t* spp,
                              const float* depth, const float* m1, const float* m2, hipStream_t st) {
  const size_t N = (size_t)k.W * k.H;
  VarFuse vf;
  hdof_status s;
  if ((s = var_update_prepare(ctx, k, alpha, depth, &vf)) != HDOF_OK) return s;
  hipLaunchKernelGGL(k_var_update, dim3(cdiv((long)N, 256)), dim3(256), 0, st, (int)N, alpha, spp, depth,
                     m1, m2, vf.rm1, vf.rm2, vf.rfl, vf.m1, vf.m2, vf.fl, vf.hz);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}
