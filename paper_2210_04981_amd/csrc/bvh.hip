// bvh.hip -- BVH build on the GPU (per scene, outside the frame).
//
// The paper traces through the driver's hardware BVH; CDNA4 has no ray
// tracing units, so the acceleration structure is built here:
//   centroid bounds -> 63-bit Morton codes -> LSD radix sort (8 x 8 bits)
//   -> PLOC clustering (Meister & Bittner, TVCG 2018): each cluster finds
//      its nearest neighbour by merged-box surface area within a window of
//      the Morton order, mutual pairs merge, clusters are compacted, until
//      one remains (a surface-area-aware tree rather than a pure Morton
//      split, which large triangles such as room walls would inflate)
//   -> depth-first numbering from subtree sizes; subtrees of at most
//      HDOF_BVH_LEAF triangles become leaves whose triangles are contiguous
//   -> traversal layout: per internal node the boxes of both children
//      (64 B), triangles as 3 float4 in leaf order.
#include "hdof_internal.h"

#define RS_THREADS 256
#define RS_ITEMS 8
#define RS_TILE (RS_THREADS * RS_ITEMS)
#define HDOF_BVH_LEAF 4
#define PLOC_R 16

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

// ---- leaves ------------------------------------------------------------------
__global__ void k_leaf_boxes(const float* __restrict__ v, const int* __restrict__ order, int n,
                             float* __restrict__ lbox) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* p = v + 9 * (size_t)order[i];
  for (int a = 0; a < 3; ++a) {
    lbox[6 * (size_t)i + a] = fminf(p[a], fminf(p[3 + a], p[6 + a]));
    lbox[6 * (size_t)i + 3 + a] = fmaxf(p[a], fmaxf(p[3 + a], p[6 + a]));
  }
}

// ---- PLOC clustering -----------------------------------------------------------
// cluster codes: >= 0 internal node (build numbering), < 0 ~leaf (Morton position)
__device__ inline float half_area(float4 lo, float4 hi) {
  float dx = hi.x - lo.x, dy = hi.y - lo.y, dz = hi.z - lo.z;
  return dx * dy + dy * dz + dz * dx;
}

__global__ void k_leaf_clusters(const float* __restrict__ lbox, int n, int* __restrict__ cid,
                                float4* __restrict__ cbox, int2* __restrict__ csz) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* b = lbox + 6 * (size_t)i;
  cid[i] = ~i;
  cbox[2 * (size_t)i] = make_float4(b[0], b[1], b[2], 0.0f);
  cbox[2 * (size_t)i + 1] = make_float4(b[3], b[4], b[5], 0.0f);
  csz[i] = make_int2(1, 0);  // (triangles, kept internal nodes) of the subtree
}

// nearest neighbour within +-PLOC_R positions by merged-box area; ties go to
// the lower index (j runs upwards with a strict comparison)
__global__ __launch_bounds__(256) void k_ploc_nn(const float4* __restrict__ cbox, int m, int* __restrict__ nn) {
  __shared__ float4 blo[256 + 2 * PLOC_R], bhi[256 + 2 * PLOC_R];
  const int base = blockIdx.x * 256 - PLOC_R;
  for (int t = threadIdx.x; t < 256 + 2 * PLOC_R; t += 256) {
    int g = base + t;
    if (g >= 0 && g < m) {
      blo[t] = cbox[2 * (size_t)g];
      bhi[t] = cbox[2 * (size_t)g + 1];
    }
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int li = i - base;
  const float4 lo = blo[li], hi = bhi[li];
  float best = INFINITY;
  int bj = -1;
  for (int d = -PLOC_R; d <= PLOC_R; ++d) {
    int j = i + d;
    if (d == 0 || j < 0 || j >= m) continue;
    const float4 l2 = blo[li + d], h2 = bhi[li + d];
    float a = half_area(make_float4(fminf(lo.x, l2.x), fminf(lo.y, l2.y), fminf(lo.z, l2.z), 0.f),
                        make_float4(fmaxf(hi.x, h2.x), fmaxf(hi.y, h2.y), fmaxf(hi.z, h2.z), 0.f));
    if (a < best) {
      best = a;
      bj = j;
    }
  }
  nn[i] = bj;
}

// bits 0..31: the cluster survives; bits 32..63: it leads a merge
__global__ void k_ploc_flags(const int* __restrict__ nn, int m, unsigned long long* __restrict__ fl) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int j = nn[i];
  bool mutual = j >= 0 && nn[j] == i;
  fl[i] = (unsigned long long)((mutual && i > j) ? 0 : 1) | ((unsigned long long)((mutual && i < j) ? 1 : 0) << 32);
}

// exclusive scan of m uint64 by one block of 1024 threads; total to *tot
__global__ void k_scan64(unsigned long long* __restrict__ a, int m, unsigned long long* __restrict__ tot) {
  __shared__ unsigned long long part[1024];
  int t = threadIdx.x;
  int chunk = (m + 1023) / 1024;
  int lo = min(m, t * chunk), hi = min(m, lo + chunk);
  unsigned long long s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    unsigned long long v = t >= off ? part[t - off] : 0ull;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned long long run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    unsigned long long x = a[i];
    a[i] = run;
    run += x;
  }
  if (t == 1023) *tot = part[1023];
}

// merged clusters take internal node indices counting down from `next`, so
// the last merge (the root) gets index 0
__global__ void k_ploc_merge(const int* __restrict__ nn, int m, const unsigned long long* __restrict__ pre,
                             const int* __restrict__ cid, const float4* __restrict__ cbox,
                             const int2* __restrict__ csz, int next, int* __restrict__ oid,
                             float4* __restrict__ obox, int2* __restrict__ osz, int* __restrict__ bl,
                             int* __restrict__ br, float* __restrict__ bbox, int2* __restrict__ bsz) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int j = nn[i];
  bool mutual = j >= 0 && nn[j] == i;
  if (mutual && i > j) return;
  unsigned long long p = pre[i];
  int pos = (int)(p & 0xffffffffull);
  if (mutual) {
    int node = next - (int)(p >> 32);
    float4 l1 = cbox[2 * (size_t)i], h1 = cbox[2 * (size_t)i + 1];
    float4 l2 = cbox[2 * (size_t)j], h2 = cbox[2 * (size_t)j + 1];
    float4 lo = make_float4(fminf(l1.x, l2.x), fminf(l1.y, l2.y), fminf(l1.z, l2.z), 0.f);
    float4 hi = make_float4(fmaxf(h1.x, h2.x), fmaxf(h1.y, h2.y), fmaxf(h1.z, h2.z), 0.f);
    int2 s1 = csz[i], s2 = csz[j];
    int cnt = s1.x + s2.x;
    int2 sz = make_int2(cnt, s1.y + s2.y + (cnt > HDOF_BVH_LEAF ? 1 : 0));
    bl[node] = cid[i];
    br[node] = cid[j];
    float* bb = bbox + 6 * (size_t)node;
    bb[0] = lo.x;
    bb[1] = lo.y;
    bb[2] = lo.z;
    bb[3] = hi.x;
    bb[4] = hi.y;
    bb[5] = hi.z;
    bsz[node] = sz;
    oid[pos] = node;
    obox[2 * (size_t)pos] = lo;
    obox[2 * (size_t)pos + 1] = hi;
    osz[pos] = sz;
  } else {
    oid[pos] = cid[i];
    obox[2 * (size_t)pos] = cbox[2 * (size_t)i];
    obox[2 * (size_t)pos + 1] = cbox[2 * (size_t)i + 1];
    osz[pos] = csz[i];
  }
}

__global__ void k_parents(int nint, const int* __restrict__ bl, const int* __restrict__ br,
                          int* __restrict__ pint, int* __restrict__ pleaf) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nint) return;
  int c[2] = {bl[a], br[a]};
  for (int k = 0; k < 2; ++k) {
    if (c[k] < 0) pleaf[~c[k]] = a;
    else pint[c[k]] = a;
  }
}

// depth-first placement by walking to the root: the first triangle slot of a
// subtree (sum of left-sibling sizes on the way up) and a kept internal
// node's index (one per level, plus the kept nodes of left siblings)
__device__ inline void dfs_place(int code, int n, const int* __restrict__ bl, const int* __restrict__ pint,
                                 const int* __restrict__ pleaf, const int2* __restrict__ bsz, int& off,
                                 int& idx, int& depth) {
  off = 0;
  idx = 0;
  depth = 0;
  int a = code < 0 ? pleaf[~code] : pint[code];
  for (int guard = 0; a >= 0 && guard < n; ++guard) {
    int left = bl[a];
    if (code != left) {  // right child
      int2 ls = left < 0 ? make_int2(1, 0) : bsz[left];
      off += ls.x;
      idx += 1 + ls.y;
    } else {
      idx += 1;
    }
    ++depth;
    code = a;
    a = a == 0 ? -1 : pint[a];
  }
}

__global__ void k_place_leaves(int n, const int* __restrict__ bl, const int* __restrict__ pint,
                               const int* __restrict__ pleaf, const int2* __restrict__ bsz,
                               int* __restrict__ leaf_off, int* __restrict__ depth_out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int off, idx, d;
  dfs_place(~i, n, bl, pint, pleaf, bsz, off, idx, d);
  leaf_off[i] = off;
  atomicMax(depth_out, d + 1);
}

__global__ void k_place_nodes(int nint, int n, const int* __restrict__ bl, const int* __restrict__ pint,
                              const int* __restrict__ pleaf, const int2* __restrict__ bsz,
                              int* __restrict__ node_off, int* __restrict__ node_idx) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nint) return;
  int off = 0, idx = 0, d = 0;
  if (a != 0) dfs_place(a, n, bl, pint, pleaf, bsz, off, idx, d);
  node_off[a] = off;
  node_idx[a] = idx;
}

__global__ void k_place_tris(const float* __restrict__ v, const int* __restrict__ order,
                             const int* __restrict__ leaf_off, int n, float4* __restrict__ tris) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int t = order[i], o = leaf_off ? leaf_off[i] : i;
  const float* p = v + 9 * (size_t)t;
  tris[3 * (size_t)o + 0] = make_float4(p[0], p[1], p[2], __int_as_float(t));
  tris[3 * (size_t)o + 1] = make_float4(p[3], p[4], p[5], 0.0f);
  tris[3 * (size_t)o + 2] = make_float4(p[6], p[7], p[8], 0.0f);
}

__device__ inline unsigned leaf_code(int first, int count) {
  return HDOF_LEAF_BIT | ((unsigned)(count - 1) << 27) | (unsigned)first;
}

// kept internal nodes (more than HDOF_BVH_LEAF triangles, or the root) are
// written at their depth-first index; smaller subtrees become leaf ranges
__global__ void k_emit_nodes(int nint, const int* __restrict__ bl, const int* __restrict__ br,
                             const int2* __restrict__ bsz, const float* __restrict__ bbox,
                             const float* __restrict__ lbox, const int* __restrict__ leaf_off,
                             const int* __restrict__ node_off, const int* __restrict__ node_idx,
                             float4* __restrict__ nodes) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nint) return;
  if (a != 0 && bsz[a].x <= HDOF_BVH_LEAF) return;
  int ch[2] = {bl[a], br[a]};
  float b[2][6];
  unsigned code[2];
  for (int k = 0; k < 2; ++k) {
    int c = ch[k];
    const float* src;
    if (c < 0) {
      src = lbox + 6 * (size_t)(~c);
      code[k] = leaf_code(leaf_off[~c], 1);
    } else {
      src = bbox + 6 * (size_t)c;
      int cnt = bsz[c].x;
      code[k] = cnt <= HDOF_BVH_LEAF ? leaf_code(node_off[c], cnt) : (unsigned)node_idx[c];
    }
    for (int q = 0; q < 6; ++q) b[k][q] = src[q];
  }
  float4* o = nodes + 4 * (size_t)node_idx[a];
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
  // permanent storage (node slots for every internal node; collapsed
  // subtrees leave the tail unused)
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
  size_t o_lbox = carve(sizeof(float) * 6 * (size_t)n);
  size_t o_cid0 = carve(sizeof(int) * n), o_cid1 = carve(sizeof(int) * n);
  size_t o_cb0 = carve(sizeof(float4) * 2 * (size_t)n), o_cb1 = carve(sizeof(float4) * 2 * (size_t)n);
  size_t o_cs0 = carve(sizeof(int2) * n), o_cs1 = carve(sizeof(int2) * n);
  size_t o_nn = carve(sizeof(int) * n), o_fl = carve(sizeof(unsigned long long) * n);
  size_t o_tot = carve(sizeof(unsigned long long));
  size_t o_bl = carve(sizeof(int) * nint), o_br = carve(sizeof(int) * nint);
  size_t o_bbox = carve(sizeof(float) * 6 * (size_t)nint), o_bsz = carve(sizeof(int2) * nint);
  size_t o_pint = carve(sizeof(int) * nint), o_pleaf = carve(sizeof(int) * n);
  size_t o_loff = carve(sizeof(int) * n), o_noff = carve(sizeof(int) * nint), o_nidx = carve(sizeof(int) * nint);
  char* s = nullptr;
  HDOF_HIP(hipMalloc(&s, off));
  float* bounds = (float*)(s + o_bounds);
  uint64_t* k0 = (uint64_t*)(s + o_k0);
  uint64_t* k1 = (uint64_t*)(s + o_k1);
  int* v0 = (int*)(s + o_v0);
  int* v1 = (int*)(s + o_v1);
  int* hist = (int*)(s + o_hist);
  float* lbox = (float*)(s + o_lbox);
  int* cid[2] = {(int*)(s + o_cid0), (int*)(s + o_cid1)};
  float4* cbox[2] = {(float4*)(s + o_cb0), (float4*)(s + o_cb1)};
  int2* csz[2] = {(int2*)(s + o_cs0), (int2*)(s + o_cs1)};
  int* nn = (int*)(s + o_nn);
  unsigned long long* fl = (unsigned long long*)(s + o_fl);
  unsigned long long* tot = (unsigned long long*)(s + o_tot);
  int *bl = (int*)(s + o_bl), *br = (int*)(s + o_br);
  float* bbox = (float*)(s + o_bbox);
  int2* bsz = (int2*)(s + o_bsz);
  int *pint = (int*)(s + o_pint), *pleaf = (int*)(s + o_pleaf);
  int *loff = (int*)(s + o_loff), *noff = (int*)(s + o_noff), *nidx = (int*)(s + o_nidx);

  hdof_status status = HDOF_OK;
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
  hipLaunchKernelGGL(k_leaf_boxes, dim3(cdiv(n, 256)), dim3(256), 0, st, verts, v0, n, lbox);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, sc->depth_out, 1, 1);
  if (n == 1) {
    hipLaunchKernelGGL(k_place_tris, dim3(1), dim3(64), 0, st, verts, v0, (const int*)nullptr, n, sc->tris);
    hipLaunchKernelGGL(k_single_root, dim3(1), dim3(1), 0, st, lbox, sc->nodes);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, sc->depth_out, 1, 2);
  } else {
    hipLaunchKernelGGL(k_leaf_clusters, dim3(cdiv(n, 256)), dim3(256), 0, st, lbox, n, cid[0], cbox[0], csz[0]);
    int m = n, next = n - 2, cur = 0;
    for (int iter = 0; m > 1 && iter < 4 * 64 + n; ++iter) {
      hipLaunchKernelGGL(k_ploc_nn, dim3(cdiv(m, 256)), dim3(256), 0, st, (const float4*)cbox[cur], m, nn);
      hipLaunchKernelGGL(k_ploc_flags, dim3(cdiv(m, 256)), dim3(256), 0, st, (const int*)nn, m, fl);
      hipLaunchKernelGGL(k_scan64, dim3(1), dim3(1024), 0, st, fl, m, tot);
      hipLaunchKernelGGL(k_ploc_merge, dim3(cdiv(m, 256)), dim3(256), 0, st, (const int*)nn, m,
                         (const unsigned long long*)fl, (const int*)cid[cur], (const float4*)cbox[cur],
                         (const int2*)csz[cur], next, cid[cur ^ 1], cbox[cur ^ 1], csz[cur ^ 1], bl, br, bbox, bsz);
      unsigned long long t = 0;
      hipError_t e = hipMemcpyAsync(&t, tot, sizeof t, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        status = hdof_set_error(HDOF_ERR_HIP, "BVH clustering: %s", hipGetErrorString(e));
        break;
      }
      int m_new = (int)(t & 0xffffffffull), merges = (int)(t >> 32);
      if (merges <= 0 || m_new != m - merges) {
        status = hdof_set_error(HDOF_ERR_HIP, "BVH clustering made no progress (%d clusters)", m);
        break;
      }
      next -= merges;
      m = m_new;
      cur ^= 1;
    }
    if (status == HDOF_OK && (m != 1 || next != -1))
      status = hdof_set_error(HDOF_ERR_HIP, "BVH clustering ended with %d clusters", m);
    if (status == HDOF_OK) {
      hipLaunchKernelGGL(k_fill_int, dim3(cdiv(nint, 256)), dim3(256), 0, st, pint, nint, -1);
      hipLaunchKernelGGL(k_parents, dim3(cdiv(nint, 256)), dim3(256), 0, st, nint, (const int*)bl, (const int*)br,
                         pint, pleaf);
      hipLaunchKernelGGL(k_place_leaves, dim3(cdiv(n, 256)), dim3(256), 0, st, n, (const int*)bl,
                         (const int*)pint, (const int*)pleaf, (const int2*)bsz, loff, sc->depth_out);
      hipLaunchKernelGGL(k_place_nodes, dim3(cdiv(nint, 256)), dim3(256), 0, st, nint, n, (const int*)bl,
                         (const int*)pint, (const int*)pleaf, (const int2*)bsz, noff, nidx);
      hipLaunchKernelGGL(k_place_tris, dim3(cdiv(n, 256)), dim3(256), 0, st, verts, (const int*)v0,
                         (const int*)loff, n, sc->tris);
      hipLaunchKernelGGL(k_emit_nodes, dim3(cdiv(nint, 256)), dim3(256), 0, st, nint, (const int*)bl,
                         (const int*)br, (const int2*)bsz, (const float*)bbox, (const float*)lbox,
                         (const int*)loff, (const int*)noff, (const int*)nidx, sc->nodes);
    }
  }
  hipError_t e = hipGetLastError();
  if (status == HDOF_OK && e != hipSuccess)
    status = hdof_set_error(HDOF_ERR_HIP, "BVH build launch: %s", hipGetErrorString(e));
  // scratch is released once the stream has consumed it
  e = hipStreamSynchronize(st);
  if (status == HDOF_OK && e != hipSuccess) status = hdof_set_error(HDOF_ERR_HIP, "BVH build: %s", hipGetErrorString(e));
  hipFree(s);
  return status;
}
