// bvh.hip -- linear BVH build on the GPU (per scene, outside the frame).
//
// The paper traces through the driver's hardware BVH; CDNA4 has no ray
// tracing units, so the acceleration structure is built here:
//   centroid bounds -> 63-bit Morton codes -> LSD radix sort (8 x 8 bits)
//   -> Karras (HPG 2012) binary radix hierarchy over the sorted codes
//   -> bottom-up box refit with one arrival counter per internal node
//   -> traversal layout: per internal node the boxes of both children
//      (64 B), triangles as 3 float4 in leaf order.
// Subtrees of at most HDOF_BVH_LEAF triangles become one leaf (their
// triangles are contiguous in Morton order).
#include "hdof_internal.h"

#define RS_THREADS 256
#define RS_ITEMS 8
#define RS_TILE (RS_THREADS * RS_ITEMS)
#define HDOF_BVH_LEAF 2

namespace {

__global__ void k_centroid_bounds(const float* __restrict__ v, int n, float* __restrict__ part) {
  __shared__ float red[6][RS_THREADS];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = blockIdx.x * RS_THREADS + threadIdx.x; i < n; i += gridDim.x * RS_THREADS) {
    const float* t = v + 9 * (size_t)i;
    for (int a = 0; a < 3; ++a) {
      float c = (t[a] + t[3 + a] + t[6 + a]) * (1.0f / 3.0f);
      lo[a] = fminf(lo[a], c);
      hi[a] = fmaxf(hi[a], c);
    }
  }
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = lo[a];
    red[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int s = RS_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_reduce_bounds(float* __restrict__ part, int nb) {
  // single thread: nb is small (<= 1024)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int b = 1; b < nb; ++b)
    for (int a = 0; a < 3; ++a) {
      part[a] = fminf(part[a], part[6 * b + a]);
      part[3 + a] = fmaxf(part[3 + a], part[6 * b + 3 + a]);
    }
}

__device__ inline uint64_t spread21(uint64_t x) {
  x &= 0x1FFFFF;
  x = (x | (x << 32)) & 0x1F00000000FFFFull;
  x = (x | (x << 16)) & 0x1F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__global__ void k_morton(const float* __restrict__ v, int n, const float* __restrict__ bounds,
                         uint64_t* __restrict__ keys, int* __restrict__ vals) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* t = v + 9 * (size_t)i;
  uint64_t q[3];
  for (int a = 0; a < 3; ++a) {
    float c = (t[a] + t[3 + a] + t[6 + a]) * (1.0f / 3.0f);
    float ext = bounds[3 + a] - bounds[a];
    float u = ext > 0.0f ? (c - bounds[a]) / ext : 0.5f;
    u = fminf(fmaxf(u, 0.0f), 1.0f);
    q[a] = (uint64_t)fminf(u * 2097152.0f, 2097151.0f);
  }
  keys[i] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
  vals[i] = i;
}

// ---- LSD radix sort: histogram, scan, stable scatter ----------------------
__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int n, int shift, int nblocks,
                          int* __restrict__ hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  int base = blockIdx.x * RS_TILE;
  for (int k = 0; k < RS_ITEMS; ++k) {
    int i = base + k * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of m ints by one block of 1024 threads (chunked)
__global__ void k_scan_single(int* __restrict__ a, int m, int* __restrict__ total) {
  __shared__ int part[1024];
  int t = threadIdx.x;
  int chunk = (m + 1023) / 1024;
  int lo = t * chunk, hi = min(m, lo + chunk);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    int x = a[i];
    a[i] = run;
    run += x;
  }
  if (total && t == 1023) *total = part[1023];
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const int* __restrict__ vin, int n,
                                                           int shift, int nblocks,
                                                           const int* __restrict__ hist,
                                                           uint64_t* __restrict__ kout,
                                                           int* __restrict__ vout) {
  __shared__ int gbase[256];
  __shared__ int running[256];
  __shared__ int wcount[RS_THREADS / 64][256];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  gbase[t] = hist[t * nblocks + blockIdx.x];
  running[t] = 0;
  for (int w = 0; w < RS_THREADS / 64; ++w) wcount[w][t] = 0;
  __syncthreads();
  int base = blockIdx.x * RS_TILE;
  for (int k = 0; k < RS_ITEMS; ++k) {
    int i = base + k * RS_THREADS + t;
    bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    int val = valid ? vin[i] : 0;
    int d = valid ? (int)((key >> shift) & 255) : 256;
    // lanes of this wave holding the same digit
    uint64_t same = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      uint64_t bits = __ballot(valid && ((d >> b) & 1));
      same &= ((d >> b) & 1) ? bits : ~bits;
    }
    if (!valid) same = 0;
    uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int rank = __popcll(same & lt);
    int leader = valid && rank == 0;
    if (leader) wcount[wave][d] = __popcll(same);
    __syncthreads();
    if (valid) {
      int off = running[d] + rank;
      for (int w = 0; w < wave; ++w) off += wcount[w][d];
      int dst = gbase[d] + off;
      kout[dst] = key;
      vout[dst] = val;
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < RS_THREADS / 64; ++w) {
      add += wcount[w][t];
      wcount[w][t] = 0;
    }
    running[t] += add;
    __syncthreads();
  }
}

// ---- Karras hierarchy ------------------------------------------------------
__device__ inline int delta(const uint64_t* __restrict__ k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = k[i], b = k[j];
  if (a == b) return 64 + __clz((unsigned)(i ^ j));
  return __clzll((long long)(a ^ b));
}

// child encoding while building: >= 0 internal index, else ~leaf (sorted position)
__global__ void k_karras(const uint64_t* __restrict__ keys, int n, int* __restrict__ left,
                         int* __restrict__ right, int* __restrict__ rlo, int* __restrict__ rhi,
                         int* __restrict__ parent_int, int* __restrict__ parent_leaf) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
  int dmin = delta(keys, n, i, i - d);
  int lmax = 2;
  while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
  int j = i + l * d;
  int dnode = delta(keys, n, i, j);
  int s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  int g = i + s * d + min(d, 0);
  int lo = min(i, j), hi = max(i, j);
  int cl = (lo == g) ? ~g : g;
  int cr = (hi == g + 1) ? ~(g + 1) : g + 1;
  left[i] = cl;
  right[i] = cr;
  rlo[i] = lo;
  rhi[i] = hi;
  if (cl < 0) parent_leaf[~cl] = i; else parent_int[cl] = i;
  if (cr < 0) parent_leaf[~cr] = i; else parent_int[cr] = i;
}

// triangles in leaf order + leaf boxes
__global__ void k_write_tris(const float* __restrict__ v, const int* __restrict__ order, int n,
                             float4* __restrict__ tris, float* __restrict__ lbox) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int t = order[i];
  const float* p = v + 9 * (size_t)t;
  tris[3 * (size_t)i + 0] = make_float4(p[0], p[1], p[2], __int_as_float(t));
  tris[3 * (size_t)i + 1] = make_float4(p[3], p[4], p[5], 0.0f);
  tris[3 * (size_t)i + 2] = make_float4(p[6], p[7], p[8], 0.0f);
  for (int a = 0; a < 3; ++a) {
    lbox[6 * (size_t)i + a] = fminf(p[a], fminf(p[3 + a], p[6 + a]));
    lbox[6 * (size_t)i + 3 + a] = fmaxf(p[a], fmaxf(p[3 + a], p[6 + a]));
  }
}

__device__ inline float ld_coherent(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// bottom-up refit: the second thread to reach an internal node computes it
__global__ void k_refit(int n, const int* __restrict__ left, const int* __restrict__ right,
                        const int* __restrict__ parent_int, const int* __restrict__ parent_leaf,
                        const float* __restrict__ lbox, float* ibox, int* arrive) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int node = parent_leaf[i];
  for (int guard = 0; node >= 0 && guard < n; ++guard) {
    __threadfence();
    int old = atomicAdd(&arrive[node], 1);
    if (old == 0) return;
    __threadfence();
    float b[6];
    for (int a = 0; a < 3; ++a) { b[a] = INFINITY; b[3 + a] = -INFINITY; }
    int ch[2] = {left[node], right[node]};
    for (int c = 0; c < 2; ++c) {
      const float* src = ch[c] < 0 ? lbox + 6 * (size_t)(~ch[c]) : ibox + 6 * (size_t)ch[c];
      for (int a = 0; a < 3; ++a) {
        b[a] = fminf(b[a], ld_coherent(src + a));
        b[3 + a] = fmaxf(b[3 + a], ld_coherent(src + 3 + a));
      }
    }
    for (int a = 0; a < 6; ++a) ibox[6 * (size_t)node + a] = b[a];
    node = node == 0 ? -1 : parent_int[node];
  }
}

__global__ void k_depth(int n, const int* __restrict__ parent_int, const int* __restrict__ parent_leaf,
                        int* depth) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int d = 1, node = parent_leaf[i];
  while (node > 0 && d <= n) {
    node = parent_int[node];
    ++d;
  }
  atomicMax(depth, d + 1);
}

__device__ inline unsigned leaf_code(int first, int count) {
  return HDOF_LEAF_BIT | ((unsigned)(count - 1) << 27) | (unsigned)first;
}

__global__ void k_write_nodes(int n, const int* __restrict__ left, const int* __restrict__ right,
                              const int* __restrict__ rlo, const int* __restrict__ rhi,
                              const float* __restrict__ lbox, const float* __restrict__ ibox,
                              float4* __restrict__ nodes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  int ch[2] = {left[i], right[i]};
  float b[2][6];
  unsigned code[2];
  for (int c = 0; c < 2; ++c) {
    const float* src;
    if (ch[c] < 0) {
      src = lbox + 6 * (size_t)(~ch[c]);
      code[c] = leaf_code(~ch[c], 1);
    } else {
      src = ibox + 6 * (size_t)ch[c];
      int cnt = rhi[ch[c]] - rlo[ch[c]] + 1;
      code[c] = cnt <= HDOF_BVH_LEAF ? leaf_code(rlo[ch[c]], cnt) : (unsigned)ch[c];
    }
    for (int a = 0; a < 6; ++a) b[c][a] = src[a];
  }
  float4* o = nodes + 4 * (size_t)i;
  o[0] = make_float4(b[0][0], b[0][3], b[0][1], b[0][4]);
  o[1] = make_float4(b[1][0], b[1][3], b[1][1], b[1][4]);
  o[2] = make_float4(b[0][2], b[0][5], b[1][2], b[1][5]);
  o[3] = make_float4(__uint_as_float(code[0]), __uint_as_float(code[1]), 0.0f, 0.0f);
}

// one triangle: a root whose second child box is empty
__global__ void k_single_root(const float* __restrict__ lbox, float4* __restrict__ nodes) {
  float4* o = nodes;
  o[0] = make_float4(lbox[0], lbox[3], lbox[1], lbox[4]);
  o[1] = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
  o[2] = make_float4(lbox[2], lbox[5], INFINITY, -INFINITY);
  o[3] = make_float4(__uint_as_float(leaf_code(0, 1)), __uint_as_float(leaf_code(0, 1)), 0.0f, 0.0f);
}

__global__ void k_fill_int(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_copy_albedo(const float* __restrict__ a, int n3, float* __restrict__ o) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) o[i] = a[i];
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

hdof_status launch_bvh_build(hdof_ctx* ctx, const float* verts, const float* albedo, int n,
                             hdof_scene* sc, hipStream_t st) {
  (void)ctx;
  const int nint = n > 1 ? n - 1 : 1;
  const int nb = cdiv(n, RS_TILE);
  const int nbounds = min(1024, max(1, cdiv(n, RS_THREADS)));
  // permanent storage
  HDOF_HIP(hipMalloc(&sc->nodes, sizeof(float4) * 4 * (size_t)nint));
  HDOF_HIP(hipMalloc(&sc->tris, sizeof(float4) * 3 * (size_t)n));
  HDOF_HIP(hipMalloc(&sc->albedo, sizeof(float) * 3 * (size_t)n));
  HDOF_HIP(hipMalloc(&sc->depth_out, sizeof(int)));
  sc->n_nodes = nint;
  sc->bytes = (int64_t)sizeof(float4) * (4 * (int64_t)nint + 3 * (int64_t)n) + 12 * (int64_t)n;
  // build scratch, one allocation
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  size_t o_bounds = carve(sizeof(float) * 6 * nbounds);
  size_t o_k0 = carve(sizeof(uint64_t) * n), o_k1 = carve(sizeof(uint64_t) * n);
  size_t o_v0 = carve(sizeof(int) * n), o_v1 = carve(sizeof(int) * n);
  size_t o_hist = carve(sizeof(int) * 256 * (size_t)nb);
  size_t o_left = carve(sizeof(int) * nint), o_right = carve(sizeof(int) * nint);
  size_t o_rlo = carve(sizeof(int) * nint), o_rhi = carve(sizeof(int) * nint);
  size_t o_pint = carve(sizeof(int) * nint), o_pleaf = carve(sizeof(int) * n);
  size_t o_lbox = carve(sizeof(float) * 6 * (size_t)n), o_ibox = carve(sizeof(float) * 6 * (size_t)nint);
  size_t o_arr = carve(sizeof(int) * nint);
  char* s = nullptr;
  HDOF_HIP(hipMalloc(&s, off));
  float* bounds = (float*)(s + o_bounds);
  uint64_t* k0 = (uint64_t*)(s + o_k0);
  uint64_t* k1 = (uint64_t*)(s + o_k1);
  int* v0 = (int*)(s + o_v0);
  int* v1 = (int*)(s + o_v1);
  int* hist = (int*)(s + o_hist);
  int *left = (int*)(s + o_left), *right = (int*)(s + o_right);
  int *rlo = (int*)(s + o_rlo), *rhi = (int*)(s + o_rhi);
  int *pint = (int*)(s + o_pint), *pleaf = (int*)(s + o_pleaf);
  float *lbox = (float*)(s + o_lbox), *ibox = (float*)(s + o_ibox);
  int* arrive = (int*)(s + o_arr);

  hipLaunchKernelGGL(k_copy_albedo, dim3(cdiv(3L * n, 256)), dim3(256), 0, st, albedo, 3 * n, sc->albedo);
  hipLaunchKernelGGL(k_centroid_bounds, dim3(nbounds), dim3(RS_THREADS), 0, st, verts, n, bounds);
  hipLaunchKernelGGL(k_reduce_bounds, dim3(1), dim3(64), 0, st, bounds, nbounds);
  hipLaunchKernelGGL(k_morton, dim3(cdiv(n, 256)), dim3(256), 0, st, verts, n, bounds, k0, v0);
  for (int pass = 0; pass < 8; ++pass) {
    int shift = 8 * pass;
    hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(RS_THREADS), 0, st, k0, n, shift, nb, hist);
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, st, hist, 256 * nb, (int*)nullptr);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(RS_THREADS), 0, st, k0, v0, n, shift, nb, hist, k1, v1);
    uint64_t* tk = k0; k0 = k1; k1 = tk;
    int* tv = v0; v0 = v1; v1 = tv;
  }
  hipLaunchKernelGGL(k_write_tris, dim3(cdiv(n, 256)), dim3(256), 0, st, verts, v0, n, sc->tris, lbox);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, sc->depth_out, 1, 1);
  if (n == 1) {
    hipLaunchKernelGGL(k_single_root, dim3(1), dim3(1), 0, st, lbox, sc->nodes);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, sc->depth_out, 1, 2);
  } else {
    hipLaunchKernelGGL(k_fill_int, dim3(cdiv(nint, 256)), dim3(256), 0, st, arrive, nint, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(cdiv(nint, 256)), dim3(256), 0, st, pint, nint, -1);
    hipLaunchKernelGGL(k_karras, dim3(cdiv(nint, 256)), dim3(256), 0, st, k0, n, left, right, rlo, rhi, pint, pleaf);
    hipLaunchKernelGGL(k_refit, dim3(cdiv(n, 256)), dim3(256), 0, st, n, left, right, pint, pleaf, lbox, ibox, arrive);
    hipLaunchKernelGGL(k_depth, dim3(cdiv(n, 256)), dim3(256), 0, st, n, pint, pleaf, sc->depth_out);
    hipLaunchKernelGGL(k_write_nodes, dim3(cdiv(nint, 256)), dim3(256), 0, st, n, left, right, rlo, rhi, lbox, ibox, sc->nodes);
  }
  HDOF_HIP(hipGetLastError());
  // scratch is released once the stream has consumed it
  HDOF_HIP(hipStreamSynchronize(st));
  HDOF_HIP(hipFree(s));
  return HDOF_OK;
}
