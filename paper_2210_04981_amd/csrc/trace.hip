// trace.hip -- BVH traversal, G-buffer and thin-lens distributed ray trace.
//
// Traversal: per-lane stack whose first HDOF_LDS_STACK entries live in LDS
// (entry i of lane t at stk[i * BLOCK + t], so a wave's pushes hit 64
// distinct banks) and the rest in a short private spill array; both children
// of a node are box-tested from one 64-byte node record, leaves are tested
// in the same step, the nearer internal child is visited first.
// Triangles: watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013),
// ties broken towards the lowest input triangle index.
//
// G-buffer: 16x16-pixel blocks, each wave an 8x8 quadrant (coherent primary
// rays); blocks remapped so each XCD works on a contiguous band of the image
// and keeps its part of the BVH in its own L2.
// Thin-lens trace: queue of (pixel, sample) entries built from the mask's
// counts and offsets; a persistent grid pops 64 entries per wave from a
// device counter, so the host never reads the ray count; results per entry,
// then a per-pixel reduction in fixed sample order (deterministic).
#include "hdof_internal.h"

#include <hip/hip_ext.h>

namespace {

struct Ray {
  V3 O, D;
  V3 inv, oinv;  // 1/D and -O/D for the slab test
  // watertight test in the ray's sheared frame (Woop, Benthin, Wald): rows
  // of the map v -> ((v-O)[kx] - Sx (v-O)[kz], (v-O)[ky] - Sy (v-O)[kz],
  // Sz (v-O)[kz]) as dense 3-vectors, with the origin term folded in
  V3 mx, my, mz;
  float ox, oy, oz;
};

__device__ inline float safe_inv(float d) {
  float a = fabsf(d) > 1e-30f ? d : copysignf(1e-30f, d);
  return 1.0f / a;
}

__device__ inline V3 unit(int k) { return V3{k == 0 ? 1.0f : 0.0f, k == 1 ? 1.0f : 0.0f, k == 2 ? 1.0f : 0.0f}; }

__device__ inline Ray make_ray(V3 O, V3 D) {
  Ray r;
  r.O = O;
  r.D = D;
  r.inv = V3{safe_inv(D.x), safe_inv(D.y), safe_inv(D.z)};
  r.oinv = V3{-O.x * r.inv.x, -O.y * r.inv.y, -O.z * r.inv.z};
  float ax = fabsf(D.x), ay = fabsf(D.y), az = fabsf(D.z);
  int kz = ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  float dz = comp(D, kz);
  if (dz < 0.0f) {
    int t = kx;
    kx = ky;
    ky = t;
  }
  const float Sx = comp(D, kx) / dz, Sy = comp(D, ky) / dz, Sz = 1.0f / dz;
  const V3 ex = unit(kx), ey = unit(ky), ez = unit(kz);
  r.mx = V3{ex.x - Sx * ez.x, ex.y - Sx * ez.y, ex.z - Sx * ez.z};
  r.my = V3{ey.x - Sy * ez.x, ey.y - Sy * ez.y, ey.z - Sy * ez.z};
  r.mz = V3{Sz * ez.x, Sz * ez.y, Sz * ez.z};
  r.ox = dot3(r.mx, O);
  r.oy = dot3(r.my, O);
  r.oz = dot3(r.mz, O);
  return r;
}

// slab test of one child box against [0, tmax]; conservative by 2 gamma(3)
__device__ inline bool box_hit(const Ray& r, float lox, float hix, float loy, float hiy, float loz,
                               float hiz, float tmax, float& tnear) {
  float tx0 = fmaf(lox, r.inv.x, r.oinv.x), tx1 = fmaf(hix, r.inv.x, r.oinv.x);
  float ty0 = fmaf(loy, r.inv.y, r.oinv.y), ty1 = fmaf(hiy, r.inv.y, r.oinv.y);
  float tz0 = fmaf(loz, r.inv.z, r.oinv.z), tz1 = fmaf(hiz, r.inv.z, r.oinv.z);
  float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
  float tmx = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
  tnear = tmin;
  return tmin <= tmx * 1.0000004f;
}

// The same test when the signs of the ray's direction are known: (nx, ny,
// nz) are the box's planes the ray enters through and (fx, fy, fz) those it
// leaves through, so the per-axis min and max of box_hit are decided in
// advance.  For a box with lo <= hi on every axis the entry and exit
// distances equal box_hit's bit for bit (an fma with a fixed multiplier and
// addend is monotonic in its first operand).
__device__ inline bool box_hit_signed(const Ray& r, float nx, float fx, float ny, float fy, float nz, float fz,
                                      float tmax, float& tnear) {
  const float tx0 = fmaf(nx, r.inv.x, r.oinv.x), tx1 = fmaf(fx, r.inv.x, r.oinv.x);
  const float ty0 = fmaf(ny, r.inv.y, r.oinv.y), ty1 = fmaf(fy, r.inv.y, r.oinv.y);
  const float tz0 = fmaf(nz, r.inv.z, r.oinv.z), tz1 = fmaf(fz, r.inv.z, r.oinv.z);
  const float tmin = fmaxf(fmaxf(tx0, ty0), fmaxf(tz0, 0.0f));
  const float tmx = fminf(fminf(tx1, ty1), fminf(tz1, tmax));
  tnear = tmin;
  return tmin <= tmx * 1.0000004f;
}

struct Best {
  float t;
  int tri;   // leaf-order index, -1 = none
  int id;    // input index
};

// Woop-Benthin-Wald watertight test; updates best on a closer (or tied,
// lower input index) hit with t > 0.  Each vertex is mapped by the ray's
// shear exactly once per test, so two triangles sharing an edge evaluate
// the same 2D edge function for it (watertight); the z row is only needed
// for a triangle the ray passes through.
__device__ inline float shear(V3 m, float o, float4 v) { return fmaf(m.z, v.z, fmaf(m.y, v.y, m.x * v.x)) - o; }

__device__ inline void tri_test(const Ray& r, const float4* __restrict__ tris, int i, Best& b) {
  const float4 a = tris[3 * i], q = tris[3 * i + 1], c = tris[3 * i + 2];
  const float Ax = shear(r.mx, r.ox, a), Ay = shear(r.my, r.oy, a);
  const float Bx = shear(r.mx, r.ox, q), By = shear(r.my, r.oy, q);
  const float Cx = shear(r.mx, r.ox, c), Cy = shear(r.my, r.oy, c);
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return;
  const float det = U + V + W;
  if (det == 0.0f) return;
  const float T = U * shear(r.mz, r.oz, a) + V * shear(r.mz, r.oz, q) + W * shear(r.mz, r.oz, c);
  const float t = T * __builtin_amdgcn_rcpf(det);
  if (!(t > 0.0f)) return;
  const int id = __float_as_int(a.w);
  if (t < b.t || (t == b.t && id < b.id)) {
    b.t = t;
    b.tri = i;
    b.id = id;
  }
}

__device__ inline void test_leaf(const Ray& r, const float4* __restrict__ tris, unsigned code, Best& b) {
  int first = (int)(code & HDOF_LEAF_FIRST_MASK);
  int cnt = (int)((code >> 27) & 0xF) + 1;
  for (int k = 0; k < cnt; ++k) tri_test(r, tris, first + k, b);
}

// Each internal node is entered at most once per ray, so more than n_nodes
// steps means a malformed tree: the ray stops and raises the device flag
// instead of looping.
struct Work {
  int visits, tests;
};

// Traversal state of one ray between steps.
struct Trav {
  Best b;
  unsigned cur;  // entry to visit next: an internal node, or a leaf code (leaf bit set)
  int sp;        // stack depth
};

__device__ inline void trav_init(Trav& s) {
  s.b = Best{INFINITY, -1, 0x7fffffff};
  s.cur = 0;  // root (internal)
  s.sp = 0;
}

// Per-lane traversal in two kinds of step.  A box step enters the lane's
// current entry, an internal node: of its two children whose boxes the ray
// reaches within the closest hit so far, the nearer (internal node or
// leaf) becomes the entry and the farther is pushed; with neither, the
// entry is popped.  A leaf step tests the entry's triangles and pops.  The
// caller takes box steps until the entry is a leaf, so the lanes of a wave
// test their leaves together; testing a leaf child as soon as it is met
// costs the whole wave its triangle loop in nearly every box step, since
// some lane nearly always meets one.
template <int BLOCK>
__device__ inline void trav_push(int* __restrict__ stk, int* __restrict__ spill, Trav& s, unsigned code,
                                 int* __restrict__ flags) {
  if (s.sp < HDOF_LDS_STACK) {
    stk[s.sp * BLOCK] = (int)code;
    ++s.sp;
  } else if (s.sp < HDOF_LDS_STACK + HDOF_SPILL_STACK) {
    spill[s.sp - HDOF_LDS_STACK] = (int)code;
    ++s.sp;
  } else {
    atomicOr(flags, HDOF_FLAG_STACK_OVERFLOW);
  }
}

// Pop the next entry; true when the stack is empty (the ray is done).
template <int BLOCK>
__device__ inline bool trav_pop(const int* __restrict__ stk, const int* __restrict__ spill, Trav& s) {
  if (s.sp == 0) return true;
  --s.sp;
  s.cur = (unsigned)(s.sp < HDOF_LDS_STACK ? stk[s.sp * BLOCK] : spill[s.sp - HDOF_LDS_STACK]);
  return false;
}

template <int BLOCK, bool COUNT>
__device__ inline bool box_step(const float4* __restrict__ nodes, const Ray& r, int* __restrict__ stk,
                                int* __restrict__ spill, Trav& s, int* __restrict__ flags, Work& wk) {
  if (COUNT) wk.visits++;
  const float4* nd = nodes + 4 * (size_t)s.cur;
  const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
  float t0, t1;
  const bool h0 = box_hit(r, n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, s.b.t, t0);
  const bool h1 = box_hit(r, n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, s.b.t, t1);
  const unsigned c0 = __float_as_uint(n3.x), c1 = __float_as_uint(n3.y);
  if (h0 && h1) {
    trav_push<BLOCK>(stk, spill, s, t0 <= t1 ? c1 : c0, flags);
    s.cur = t0 <= t1 ? c0 : c1;
  } else if (h0) {
    s.cur = c0;
  } else if (h1) {
    s.cur = c1;
  } else {
    return trav_pop<BLOCK>(stk, spill, s);
  }
  return false;
}

template <int BLOCK, bool COUNT>
__device__ inline bool leaf_step(const float4* __restrict__ tris, const Ray& r, const int* __restrict__ stk,
                                 const int* __restrict__ spill, Trav& s, Work& wk) {
  test_leaf(r, tris, s.cur, s.b);
  if (COUNT) wk.tests += (int)((s.cur >> 27) & 0xF) + 1;
  return trav_pop<BLOCK>(stk, spill, s);
}

// Wave-coherent traversal: the lanes of a wave walk one node sequence, the
// union of their own paths (primary rays of an 8x8 pixel quadrant are
// coherent).  Node records and leaf triangles are then wave-uniform loads,
// served by the scalar data cache instead of 64 vector fetches per node;
// the node stack is one VGPR holding entry i in lane i; a lane tests the
// boxes of every node the wave enters against its own closest hit, and the
// wave enters a child when any lane's ray reaches it.  Of two such
// children the one the wave's first lane reaches first is entered first.
// Each node is entered at most once per wave, so more than n_nodes steps
// raises the device flag and stops.
// FLIP >= 0: every live lane's direction has the signs FLIP gives (bit k
// set: axis k negative), so each slab's entry and exit planes are known at
// compile time (one copy of the loop per sign octant) and the box test
// needs no per-lane min and max of the two slab distances.  FLIP < 0: the
// general test.
template <bool COUNT, int FLIP>
__device__ inline Best traverse_wave(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                     int n_nodes, const Ray& r, bool live, int* __restrict__ flags, Work& wk) {
  // a lane without a ray starts with a negative closest-hit distance: every
  // box test then fails for it (entry distances are >= 0), so its results
  // need no masking
  Best b = Best{live ? INFINITY : -1.0f, -1, 0x7fffffff};
  const int lane = (int)(threadIdx.x & 63);
  int stackv = 0;  // entry i in lane i
  int sp = 0;
  unsigned cur = 0;  // root (internal)
  for (int steps = 0;; ++steps) {
    if (steps > n_nodes) {
      if (live) atomicOr(flags, HDOF_FLAG_STACK_OVERFLOW);
      break;
    }
    if (COUNT && live) wk.visits++;
    const float4* nd = nodes + 4 * (size_t)cur;
    const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2], n3 = nd[3];
    float t0, t1;
    bool h0, h1;
    if (FLIP >= 0) {
      constexpr bool fx = (FLIP & 1) != 0, fy = (FLIP & 2) != 0, fz = (FLIP & 4) != 0;
      h0 = box_hit_signed(r, fx ? n0.y : n0.x, fx ? n0.x : n0.y, fy ? n0.w : n0.z, fy ? n0.z : n0.w,
                          fz ? n2.y : n2.x, fz ? n2.x : n2.y, b.t, t0);
      h1 = box_hit_signed(r, fx ? n1.y : n1.x, fx ? n1.x : n1.y, fy ? n1.w : n1.z, fy ? n1.z : n1.w,
                          fz ? n2.w : n2.z, fz ? n2.z : n2.w, b.t, t1);
    } else {
      h0 = box_hit(r, n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, b.t, t0);
      h1 = box_hit(r, n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, b.t, t1);
    }
    const unsigned c0 = __float_as_uint(n3.x), c1 = __float_as_uint(n3.y);
    const unsigned long long m0 = __builtin_amdgcn_ballot_w64(h0), m1 = __builtin_amdgcn_ballot_w64(h1);
    const bool l0 = (c0 & HDOF_LEAF_BIT) != 0, l1 = (c1 & HDOF_LEAF_BIT) != 0;
    if (l0 && m0 != 0ull) {
      if (h0) {
        test_leaf(r, tris, c0, b);
        if (COUNT) wk.tests += (int)((c0 >> 27) & 0xF) + 1;
      }
    }
    if (l1 && m1 != 0ull) {
      if (h1) {
        test_leaf(r, tris, c1, b);
        if (COUNT) wk.tests += (int)((c1 >> 27) & 0xF) + 1;
      }
    }
    const bool v0 = !l0 && m0 != 0ull, v1 = !l1 && m1 != 0ull;
    if (v0 && v1) {
      const bool first0 = __builtin_amdgcn_readfirstlane((int)(t0 <= t1)) != 0;
      const unsigned nearc = first0 ? c0 : c1, farc = first0 ? c1 : c0;
      if (sp < 64) {
        stackv = lane == sp ? (int)farc : stackv;
        ++sp;
      } else if (live) {
        atomicOr(flags, HDOF_FLAG_STACK_OVERFLOW);
      }
      cur = nearc;
    } else if (v0) {
      cur = c0;
    } else if (v1) {
      cur = c1;
    } else {
      if (sp == 0) break;
      --sp;
      cur = (unsigned)__builtin_amdgcn_readlane(stackv, sp);
    }
  }
  return b;
}

// The wave's traversal: the signed form when the live lanes' directions
// share their signs on every axis (nearly every wave of pixel-adjacent
// rays), else the general one.  Both return the same closest hit.
template <bool COUNT>
__device__ inline Best traverse_wave_any(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                         int n_nodes, const Ray& r, bool live, int* __restrict__ flags, Work& wk) {
  const unsigned long long lm = __ballot(live);
  const unsigned long long sx = __ballot(live && signbit(r.inv.x)), sy = __ballot(live && signbit(r.inv.y)),
                           sz = __ballot(live && signbit(r.inv.z));
  if ((sx == 0ull || sx == lm) && (sy == 0ull || sy == lm) && (sz == 0ull || sz == lm)) {
    const int flip = (sx != 0ull ? 1 : 0) | (sy != 0ull ? 2 : 0) | (sz != 0ull ? 4 : 0);
    switch (flip) {
      case 0: return traverse_wave<COUNT, 0>(nodes, tris, n_nodes, r, live, flags, wk);
      case 1: return traverse_wave<COUNT, 1>(nodes, tris, n_nodes, r, live, flags, wk);
      case 2: return traverse_wave<COUNT, 2>(nodes, tris, n_nodes, r, live, flags, wk);
      case 3: return traverse_wave<COUNT, 3>(nodes, tris, n_nodes, r, live, flags, wk);
      case 4: return traverse_wave<COUNT, 4>(nodes, tris, n_nodes, r, live, flags, wk);
      case 5: return traverse_wave<COUNT, 5>(nodes, tris, n_nodes, r, live, flags, wk);
      case 6: return traverse_wave<COUNT, 6>(nodes, tris, n_nodes, r, live, flags, wk);
      default: return traverse_wave<COUNT, 7>(nodes, tris, n_nodes, r, live, flags, wk);
    }
  }
  return traverse_wave<COUNT, -1>(nodes, tris, n_nodes, r, live, flags, wk);
}

// Two-sided Lambertian face normal + point light, no shadow ray; with a
// specular table (k_s, shininess per input triangle) a Blinn-Phong lobe
// k_s I max(0, n.h)^shininess / max(d^2, 1e-4) is added while the light is
// on the viewer's side, h the unit half vector of the light direction and
// the direction back along the ray; ys = the lobe's luminance.
__device__ inline void shade(const float4* __restrict__ tris, const float* __restrict__ albedo,
                             const float2* __restrict__ spec, const LightK& li, const Ray& r, const Best& b, V3& L,
                             V3& n, V3& alb, float& ys) {
  float4 a = tris[3 * b.tri], q = tris[3 * b.tri + 1], c = tris[3 * b.tri + 2];
  V3 e1 = V3{q.x - a.x, q.y - a.y, q.z - a.z};
  V3 e2 = V3{c.x - a.x, c.y - a.y, c.z - a.z};
  V3 nn = cross3(e1, e2);
  float il = rsqrtf(dot3(nn, nn));
  nn = il * nn;
  if (dot3(nn, r.D) > 0.0f) nn = V3{-nn.x, -nn.y, -nn.z};
  V3 P = V3{fmaf(b.t, r.D.x, r.O.x), fmaf(b.t, r.D.y, r.O.y), fmaf(b.t, r.D.z, r.O.z)};
  V3 l = li.p - P;
  float d2 = dot3(l, l);
  float cosv = d2 > 0.0f ? dot3(nn, l) * rsqrtf(d2) : 0.0f;
  float irr = fmaxf(0.0f, cosv) / fmaxf(d2, 1e-4f);
  const float* al = albedo + 3 * (size_t)b.id;
  alb = V3{al[0], al[1], al[2]};
  L = V3{alb.x * fmaf(li.I.x, irr, li.ka.x), alb.y * fmaf(li.I.y, irr, li.ka.y),
         alb.z * fmaf(li.I.z, irr, li.ka.z)};
  n = nn;
  ys = 0.0f;
  if (spec) {
    const float2 m = spec[b.id];
    if (m.x > 0.0f && cosv > 0.0f) {
      const float il2 = rsqrtf(d2), iD = rsqrtf(dot3(r.D, r.D));
      const V3 h = V3{fmaf(l.x, il2, -r.D.x * iD), fmaf(l.y, il2, -r.D.y * iD), fmaf(l.z, il2, -r.D.z * iD)};
      const float hh = dot3(h, h);
      const float nh = hh > 0.0f ? fmaxf(0.0f, dot3(nn, h) * rsqrtf(hh)) : 0.0f;
      const float f = m.x * powf(nh, m.y) / fmaxf(d2, 1e-4f);
      L = V3{fmaf(f, li.I.x, L.x), fmaf(f, li.I.y, L.y), fmaf(f, li.I.z, L.z)};
      ys = f * fmaf(0.2126f, li.I.x, fmaf(0.7152f, li.I.y, 0.0722f * li.I.z));
    }
  }
}

// PACK (frames with 16-pixel post-filter tiles): also the post-filter's
// packed texel (shaded rgb, signed CoC of the stored depth) and the block's
// maximum CoC radius, the block being the post-filter tile.
// spec_out (nullable): the specular luminance plane.
// One 16x16-pixel block lb of the image of camera k (its outputs planar
// [C][H][W] from the given pointers).
template <bool COUNT, bool PACK>
__device__ inline void gbuffer_block(const float4* __restrict__ nodes, const float4* __restrict__ tris, int n_nodes,
                                     const float* __restrict__ albedo, const float2* __restrict__ spec,
                                     float* __restrict__ spec_out, const CamK& k, const LensK& l, const LightK& li,
                                     int lb, float* __restrict__ depth, float* __restrict__ normal,
                                     float* __restrict__ alb_out, float* __restrict__ color, int* __restrict__ tri_id,
                                     int* __restrict__ flags, unsigned long long* __restrict__ counters,
                                     float4* __restrict__ pack, float* __restrict__ tile_r) {
  __shared__ float wmax[4];
  const int bx_n = (k.W + 15) >> 4;
  const int bx = lb % bx_n, by = lb / bx_n;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int x = bx * 16 + (wave & 1) * 8 + (lane & 7), y = by * 16 + (wave >> 1) * 8 + (lane >> 3);
  const bool live = x < k.W && y < k.H;
  V3 v = pixel_dir(k, live ? x : 0, live ? y : 0);
  Ray r = make_ray(k.e, V3{l.S1 * v.x, l.S1 * v.y, l.S1 * v.z});
  Work wk{0, 0};
  Best b = traverse_wave_any<COUNT>(nodes, tris, n_nodes, r, live, flags, wk);
  float rr = 0.0f;
  if (live) {
    if (COUNT) {
      atomicAdd(&counters[0], 1ull);
      atomicAdd(&counters[1], (unsigned long long)wk.visits);
      atomicAdd(&counters[2], (unsigned long long)wk.tests);
    }
    const size_t N = (size_t)k.W * k.H, p = (size_t)y * k.W + x;
    float z = HDOF_ZMAX, ys = 0.0f;
    V3 L = V3{0.0f, 0.0f, 0.0f};
    if (b.tri >= 0) {
      V3 n, a;
      shade(tris, albedo, spec, li, r, b, L, n, a, ys);
      z = b.t * l.S1;
      normal[p] = n.x;
      normal[N + p] = n.y;
      normal[2 * N + p] = n.z;
      alb_out[p] = a.x;
      alb_out[N + p] = a.y;
      alb_out[2 * N + p] = a.z;
      tri_id[p] = b.id;
    } else {
      for (int c = 0; c < 3; ++c) {
        normal[c * N + p] = 0.0f;
        alb_out[c * N + p] = 0.0f;
      }
      tri_id[p] = -1;
    }
    depth[p] = z;
    if (spec_out) spec_out[p] = ys;
    color[p] = L.x;
    color[N + p] = L.y;
    color[2 * N + p] = L.z;
    if (PACK) {
      const float c = coc_px(l, z);
      pack[p] = make_float4(L.x, L.y, L.z, c);
      rr = 0.5f * fabsf(c);
    }
  }
  if (PACK) {
    for (int o = 32; o > 0; o >>= 1) rr = fmaxf(rr, __shfl_xor(rr, o));
    if (lane == 0) wmax[wave] = rr;
    __syncthreads();
    if (t == 0) tile_r[lb] = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
  }
}

template <bool COUNT, bool PACK>
__global__ __launch_bounds__(256) void k_gbuffer(const float4* __restrict__ nodes,
                                                 const float4* __restrict__ tris, int n_nodes,
                                                 const float* __restrict__ albedo,
                                                 const float2* __restrict__ spec, float* __restrict__ spec_out,
                                                 CamK k, LensK l,
                                                 LightK li, float* __restrict__ depth,
                                                 float* __restrict__ normal, float* __restrict__ alb_out,
                                                 float* __restrict__ color, int* __restrict__ tri_id,
                                                 int* __restrict__ flags,
                                                 unsigned long long* __restrict__ counters,
                                                 float4* __restrict__ pack, float* __restrict__ tile_r) {
  const int nb = ((k.W + 15) >> 4) * ((k.H + 15) >> 4);
  gbuffer_block<COUNT, PACK>(nodes, tris, n_nodes, albedo, spec, spec_out, k, l, li, xcd_block(blockIdx.x, nb),
                             depth, normal, alb_out, color, tri_id, flags, counters, pack, tile_r);
}

// queue entries: pixel index repeated spp times at its offset; also resets
// the persistent trace's work counters (same stream, runs before the trace).
// Batched: offsets are view-local, *ebase is the view's first queue entry
// and the stored index is the pixel's position in the batch (pxbase + p).
// Entries outside [0, cap) are dropped: inconsistent offsets never write out
// of bounds.
__global__ void k_queue_fill(const uint8_t* __restrict__ spp, const int* __restrict__ offsets, int N,
                             const int* __restrict__ ebase, int pxbase, long cap, int* __restrict__ queue,
                             int* __restrict__ counter) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < 8 * HDOF_SEG_STRIDE) counter[p] = 0;
  if (p >= N) return;
  int s = spp[p];
  long o = (long)offsets[p] + (ebase ? *ebase : 0);
  for (int j = 0; j < s; ++j)
    if (o + j >= 0 && o + j < cap) queue[o + j] = pxbase + p;
}

// Persistent trace.  Every lane runs its own ray one node step at a time;
// when at least `refill` lanes of a wave are idle the wave takes that many
// entries from the queue with one atomic and hands them to the idle lanes
// (refill = 64: batches of 64 rays).  The queue is cut into `segments`
// contiguous segments (bands of image rows; whole views in a batch), one
// per group of XCDs (blocks are dispatched round-robin over the 8 XCDs): a
// wave takes work from its own segment first, so each XCD's L2 holds the
// part of the BVH its rays touch, then moves on to the other segments.
// Every wave exits once all segments are drained and its lanes are idle.
using ViewK = BatchView;  // the device copy of a batch's view table

struct TraceArgs {
  const float4* nodes;
  const float4* tris;
  int n_nodes;
  const float* albedo;
  const float2* spec;  // nullable: Lambertian
  LightK li;
  const int* queue;
  const int* offsets;
  const int* total_p;
  int* counter;
  float* ray_col;
  float* ray_z;
  int* ray_id;
  size_t cap;
  int* flags;
  unsigned long long* counters;
  int refill, segments;
  int ray_quantum, n_cu, bpc;  // ray_quantum > 0: blocks kept per CU = ceil(rays / ray_quantum) in [1, bpc]
  ViewK v0;                // the view of a plain frame
  const ViewK* views;      // batch: device table of views
  const int* entry_base;   // batch: first queue entry of each view
  int n_views;
};

// The ray of queue entry ee of a segment ending at hi: its pixel from the
// queue, its sample index from the pixel's first entry, the lens sample
// from the view's counters.  False for an entry past hi or a corrupt pixel
// index.  pxb (batch): the first batch pixel of each view.
template <bool BATCH>
__device__ inline bool entry_ray(const TraceArgs& A, const int* pxb, int ee, int hi, Ray& r, float& S1) {
  const int g = ee < hi ? A.queue[ee] : -1;
  bool ok;
  int p, j;
  const ViewK* vk = &A.v0;
  if (BATCH) {
    // view of batch pixel g: last view whose first pixel is <= g
    int v = 0;
    for (int step = HDOF_MAX_VIEWS / 2; step >= 1; step >>= 1)
      if (v + step < A.n_views && pxb[v + step] <= g) v += step;
    vk = &A.views[v];
    p = g - pxb[v];
    ok = g >= 0 && p < vk->k.W * vk->k.H;
    j = ok ? ee - A.entry_base[v] - A.offsets[g] : 0;
  } else {
    p = g;
    ok = g >= 0 && g < A.v0.k.W * A.v0.k.H;
    j = ok ? ee - A.offsets[g] : 0;
  }
  if (!ok) return false;
  const CamK k = vk->k;
  const LensK l = vk->l;
  V3 O, D;
  lens_ray(k, l, p % k.W, p / k.W, (uint32_t)j, vk->view, vk->seed, vk->frame, O, D);
  r = make_ray(O, D);
  S1 = l.S1;
  return true;
}

// Shade the closest hit of a finished ray and store entry e's result.
template <bool COUNT>
__device__ inline void store_ray(const TraceArgs& A, const Ray& r, const Best& b, float S1, int e, const Work& wk) {
  float z = HDOF_ZMAX;
  V3 L = V3{0.0f, 0.0f, 0.0f};
  if (b.tri >= 0) {
    V3 n, a;
    float ys;
    shade(A.tris, A.albedo, A.spec, A.li, r, b, L, n, a, ys);
    z = b.t * S1;
  }
  A.ray_col[e] = L.x;
  A.ray_col[A.cap + e] = L.y;
  A.ray_col[2 * A.cap + e] = L.z;
  A.ray_z[e] = z;
  if (A.ray_id) A.ray_id[e] = b.tri >= 0 ? b.id : -1;
  if (COUNT) {
    atomicAdd(&A.counters[3], 1ull);
    atomicAdd(&A.counters[4], (unsigned long long)wk.visits);
    atomicAdd(&A.counters[5], (unsigned long long)wk.tests);
  }
}

// The G-buffers of a batch in one launch (packed texels and tile radii
// too): the launch's blocks, in XCD-contiguous order over the whole batch,
// are the views' 16x16-pixel blocks one view after another; blk_base[v] is
// view v's first block (blk_base[n] the total), which is also its first
// post-filter tile.  A view's planes start at its first batch pixel.
struct GbBatch {
  int n;
  int blk_base[HDOF_MAX_VIEWS + 1];
};

__global__ __launch_bounds__(256) void k_gbuffer_batch(const float4* __restrict__ nodes,
                                                       const float4* __restrict__ tris, int n_nodes,
                                                       const float* __restrict__ albedo, LightK li,
                                                       const ViewK* __restrict__ views, GbBatch gbb,
                                                       float* __restrict__ depth, float* __restrict__ normal,
                                                       float* __restrict__ alb_out, float* __restrict__ color,
                                                       int* __restrict__ tri_id, int* __restrict__ flags,
                                                       float4* __restrict__ pack, float* __restrict__ tile_r) {
  const int g = xcd_block(blockIdx.x, gbb.blk_base[gbb.n]);
  const int v = batch_view_of(gbb.blk_base, gbb.n, g);
  const ViewK& vk = views[v];
  const size_t pb = (size_t)vk.px_base;
  gbuffer_block<false, true>(nodes, tris, n_nodes, albedo, nullptr, nullptr, vk.k, vk.l, li, g - gbb.blk_base[v],
                             depth + pb, normal + 3 * pb, alb_out + 3 * pb, color + 3 * pb, tri_id + pb, flags,
                             nullptr, pack + pb, tile_r + gbb.blk_base[v]);
}

// Whether this block of the persistent trace takes part: with a ray
// quantum (a frame overlapping the trace with the post-filter gather) only
// the first ceil(total * n_cu / ray_quantum) blocks, one block per CU for
// every ray_quantum rays on average (at least one per CU, at most the
// grid), so a light trace leaves the CUs to the gather; the first blocks
// are kept, so every queue segment keeps its blocks.
__device__ inline bool keep_block(const TraceArgs& A, int total) {
  if (A.ray_quantum <= 0) return true;
  const long kept = ((long)total * A.n_cu + A.ray_quantum - 1) / A.ray_quantum;
  return (long)blockIdx.x < min((long)A.bpc * A.n_cu, max((long)A.n_cu, kept));
}

// Entries handed out: per queue segment (one per XCD, the block's
// blockIdx.x mod segments) an atomic counter of entries taken; a wave whose
// segment runs dry moves on to the next and stops once it has found every
// segment dry.
template <bool COUNT, bool BATCH>
__global__ __launch_bounds__(HDOF_TRACE_BLOCK, HDOF_TRACE_WAVES_PER_EU) void k_trace(TraceArgs A) {
  __shared__ int stk_all[HDOF_LDS_STACK * HDOF_TRACE_BLOCK];
  __shared__ int pxb[HDOF_MAX_VIEWS + 1];
  int spill[HDOF_SPILL_STACK];
  const int t = threadIdx.x, lane = t & 63;
  int* stk = stk_all + t;
  if (BATCH) {
    for (int v = t; v < A.n_views; v += HDOF_TRACE_BLOCK) pxb[v] = A.views[v].px_base;
    __syncthreads();
  }
  int total = *A.total_p;
  if (total < 0) total = 0;
  if ((size_t)total > A.cap) {
    if (blockIdx.x == 0 && t == 0) atomicOr(A.flags, HDOF_FLAG_CAPACITY);
    total = (int)A.cap;
  }
  if (!keep_block(A, total)) return;
  const int nseg = A.segments;
  const unsigned long long lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  bool active = false, drained = false;
  int e = 0, steps = 0;
  int seg = blockIdx.x % nseg, tried = 0;
  float S1 = A.v0.l.S1;
  Ray r;
  Trav s;
  Work wk{0, 0};
  for (;;) {
    const unsigned long long idle = __ballot(!active);
    const int nidle = __popcll(idle);
    if (!drained && nidle >= A.refill) {
      const int lo = (int)((long)total * seg / nseg), hi = (int)((long)total * (seg + 1) / nseg);
      int base = 0;
      if (lane == 0) base = atomicAdd(&A.counter[seg * HDOF_SEG_STRIDE], nidle);
      base = __shfl(base, 0) + lo;
      if (base + nidle >= hi) {  // this segment is used up: go on to the next one
        seg = seg + 1 == nseg ? 0 : seg + 1;
        drained = ++tried == nseg;
      }
      if (!active) {
        const int ee = base + __popcll(idle & lt_mask);
        if (entry_ray<BATCH>(A, pxb, ee, hi, r, S1)) {
          trav_init(s);
          e = ee;
          steps = 0;
          active = true;
          if (COUNT) wk = Work{0, 0};
        }
      }
    }
    if (!active) {
      if (drained) break;  // nothing left to hand out: an idle lane is done
      continue;
    }
    // box steps until the entry is a leaf (each internal node is entered at
    // most once per ray, so more than n_nodes of them means a malformed tree:
    // the ray stops and raises the device flag), then the leaf step
    bool done = false;
    while (!(s.cur & HDOF_LEAF_BIT)) {
      if (++steps > A.n_nodes) {
        atomicOr(A.flags, HDOF_FLAG_STACK_OVERFLOW);
        done = true;
        break;
      }
      if (box_step<HDOF_TRACE_BLOCK, COUNT>(A.nodes, r, stk, spill, s, A.flags, wk)) {
        done = true;
        break;
      }
    }
    if (!done) done = leaf_step<HDOF_TRACE_BLOCK, COUNT>(A.tris, r, stk, spill, s, wk);
    if (done) {
      store_ray<COUNT>(A, r, s.b, S1, e, wk);
      active = false;
    }
  }
}

// Wave-coherent form: a wave takes 64 consecutive entries of its segment at
// a time (the samples of a few neighbouring pixels, whose rays differ by
// their lens offsets) and walks the union of their paths with wave-uniform
// node loads (traverse_wave_any), then shades and stores them; no per-lane
// refill and no LDS stack.  Same hand-out of entries as k_trace, so the
// same results.
template <bool COUNT, bool BATCH>
__global__ __launch_bounds__(HDOF_TRACE_BLOCK, HDOF_TRACE_WAVES_PER_EU) void k_trace_wave(TraceArgs A) {
  __shared__ int pxb[HDOF_MAX_VIEWS + 1];
  const int t = threadIdx.x, lane = t & 63;
  if (BATCH) {
    for (int v = t; v < A.n_views; v += HDOF_TRACE_BLOCK) pxb[v] = A.views[v].px_base;
    __syncthreads();
  }
  int total = *A.total_p;
  if (total < 0) total = 0;
  if ((size_t)total > A.cap) {
    if (blockIdx.x == 0 && t == 0) atomicOr(A.flags, HDOF_FLAG_CAPACITY);
    total = (int)A.cap;
  }
  if (!keep_block(A, total)) return;
  const int nseg = A.segments;
  int seg = blockIdx.x % nseg, tried = 0;
  while (tried < nseg) {
    const int lo = (int)((long)total * seg / nseg), hi = (int)((long)total * (seg + 1) / nseg);
    int base = 0;
    if (lane == 0) base = atomicAdd(&A.counter[seg * HDOF_SEG_STRIDE], 64);
    base = __shfl(base, 0) + lo;
    if (base >= hi) {  // this segment is used up: go on to the next one
      seg = seg + 1 == nseg ? 0 : seg + 1;
      ++tried;
      continue;
    }
    const int e = base + lane;
    Ray r;
    float S1 = A.v0.l.S1;
    const bool live = entry_ray<BATCH>(A, pxb, e, hi, r, S1);
    if (!live) r = make_ray(V3{0.0f, 0.0f, 0.0f}, V3{0.0f, 0.0f, 1.0f});
    Work wk{0, 0};
    const Best b = traverse_wave_any<COUNT>(A.nodes, A.tris, A.n_nodes, r, live, A.flags, wk);
    if (live) store_ray<COUNT>(A, r, b, S1, e, wk);
  }
}

// per-pixel near/far split, hit ratio and luminance moments, fixed order;
// batched: *ebase is the view's first queue entry
// FARPOS: also the far-weighted mean hit point of the pixel's rays that hit
// (their rays regenerated from the same counters; t = z / S1 since the
// direction's forward component is S1) and its weight, 4 planes.
// VAR (whole frames): the variance history update of the pixel as well,
// from the moments just formed.
// coc_nf (nullable, 2 planes): the average CoC size of the near rays and of
// the far rays, sum w |c| / sum w and sum (1 - w) |c| / sum (1 - w).
template <bool FARPOS, bool VAR>
__device__ __forceinline__ void rt_reduce_px(int p, const uint8_t* __restrict__ spp, const int* __restrict__ offsets,
                                             int N, const int* __restrict__ ebase, const float* __restrict__ ray_col,
                                             const float* __restrict__ ray_z, size_t cap, const LensK& l,
                                             float* __restrict__ cn, float* __restrict__ cf, float* __restrict__ h,
                                             float* __restrict__ m1, float* __restrict__ m2, const CamK& k,
                                             uint32_t seed, uint32_t frame, uint32_t view,
                                             float* __restrict__ far_pos, const VarFuse& vf,
                                             float* __restrict__ coc_nf) {
  int s = spp[p];
  float Nw = 0.f, Fw = 0.f, snr = 0.f, sng = 0.f, snb = 0.f, sfr = 0.f, sfg = 0.f, sfb = 0.f, sy = 0.f, sy2 = 0.f;
  float Pw = 0.f, spx_ = 0.f, spy_ = 0.f, spz_ = 0.f, scn = 0.f, scf = 0.f;
  // untraced pixels (most of them) do not read their offset
  const long o = s > 0 ? (long)offsets[p] + (ebase ? *ebase : 0) : 0;
  if (o < 0 || o + s > (long)cap) s = 0;  // inconsistent offsets: nothing was traced here
  // spherical aberration: every ray weighs its lens sample's weight (the
  // sample regenerated from its counters); 1 for sa = 0
  const bool weighted = l.sa != 0.0f;
  float Sw = 0.f;
  if (s > 0) {
    for (int j = 0; j < s; ++j) {
      long e = o + j;
      float R = ray_col[e], G = ray_col[cap + e], B = ray_col[2 * cap + e];
      const float zj = ray_z[e];
      float c = coc_px(l, zj);
      float om = 1.0f;
      V3 O, D;
      if (FARPOS || weighted) lens_ray(k, l, p % k.W, p / k.W, (uint32_t)j, view, seed, frame, O, D, &om);
      float w = om * clamp01(fmaf(-c, 0.35355339059327376f, 0.5f));
      float wf = om - w;
      if (FARPOS && zj < HDOF_ZMAX) {
        const float t = zj * l.invS1;
        Pw += wf;
        spx_ = fmaf(wf, fmaf(t, D.x, O.x), spx_);
        spy_ = fmaf(wf, fmaf(t, D.y, O.y), spy_);
        spz_ = fmaf(wf, fmaf(t, D.z, O.z), spz_);
      }
      Sw += om;
      Nw += w;
      Fw += wf;
      scn = fmaf(w, fabsf(c), scn);
      scf = fmaf(wf, fabsf(c), scf);
      snr = fmaf(w, R, snr);
      sng = fmaf(w, G, sng);
      snb = fmaf(w, B, snb);
      sfr = fmaf(wf, R, sfr);
      sfg = fmaf(wf, G, sfg);
      sfb = fmaf(wf, B, sfb);
      float Y = fmaf(0.2126f, R, fmaf(0.7152f, G, 0.0722f * B));
      sy = fmaf(om, Y, sy);
      sy2 = fmaf(om * Y, Y, sy2);
    }
  }
  const float in_ = Nw > 0.f ? 1.0f / Nw : 0.f, if_ = Fw > 0.f ? 1.0f / Fw : 0.f;
  const float is = Sw > 0.f ? 1.0f / Sw : 0.f;
  const float ybar = sy * is, y2bar = sy2 * is;
  if (!vf.sparse_rt || spp[p] > 0) {
    cn[p] = snr * in_;
    cn[N + p] = sng * in_;
    cn[2 * (size_t)N + p] = snb * in_;
    cf[p] = sfr * if_;
    cf[N + p] = sfg * if_;
    cf[2 * (size_t)N + p] = sfb * if_;
    h[p] = Nw * is;
    m1[p] = ybar;
    m2[p] = y2bar;
  }
  if (VAR && !(vf.in_place && spp[p] == 0)) {  // in place: an untraced pixel's history is already there
    float a1 = vf.rm1[p], a2 = vf.rm2[p];
    uint8_t f = vf.rfl[p];
    if (spp[p] > 0) {
      if (f & HDOF_HIST_VALID) {
        a1 = fmaf(vf.alpha, ybar, (1.0f - vf.alpha) * a1);
        a2 = fmaf(vf.alpha, y2bar, (1.0f - vf.alpha) * a2);
        f = HDOF_HIST_VALID;
      } else {
        a1 = ybar;
        a2 = y2bar;
        f = HDOF_HIST_VALID | HDOF_HIST_NEW;
      }
    }
    vf.m1[p] = a1;
    vf.m2[p] = a2;
    vf.fl[p] = f;
    if (!vf.in_place) vf.hz[p] = vf.depth[p];
  }
  if (FARPOS) {
    const float ip = Pw > 0.f ? 1.0f / Pw : 0.f;
    far_pos[p] = spx_ * ip;
    far_pos[N + p] = spy_ * ip;
    far_pos[2 * (size_t)N + p] = spz_ * ip;
    far_pos[3 * (size_t)N + p] = Pw;
  }
  if (coc_nf) {
    coc_nf[p] = scn * in_;
    coc_nf[N + p] = scf * if_;
  }
}

template <bool FARPOS, bool VAR>
__global__ void k_rt_reduce(const uint8_t* __restrict__ spp, const int* __restrict__ offsets, int N,
                            const int* __restrict__ ebase, const float* __restrict__ ray_col,
                            const float* __restrict__ ray_z, size_t cap, LensK l, float* __restrict__ cn,
                            float* __restrict__ cf, float* __restrict__ h, float* __restrict__ m1,
                            float* __restrict__ m2, CamK k, uint32_t seed, uint32_t frame, uint32_t view,
                            float* __restrict__ far_pos, VarFuse vf, float* __restrict__ coc_nf) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  rt_reduce_px<FARPOS, VAR>(p, spp, offsets, N, ebase, ray_col, ray_z, cap, l, cn, cf, h, m1, m2, k, seed, frame,
                            view, far_pos, vf, coc_nf);
}

// The batched form's queue fill and reduction, one launch each over every
// view: blocks of HDOF_BATCH_PX_BLOCK pixels (256 threads, a pixel every
// 256), view v's from blk_base[v] (blk_base[n] the total), its pixels from
// its px_base and its queue entries from ebase[v].
struct PxBatch {
  int n;
  int blk_base[HDOF_MAX_VIEWS + 1];
};

__global__ void k_queue_fill_batch(const uint8_t* __restrict__ spp, const int* __restrict__ offsets,
                                   const ViewK* __restrict__ views, PxBatch b, const int* __restrict__ ebase,
                                   long cap, int* __restrict__ queue, int* __restrict__ counter) {
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < 8 * HDOF_SEG_STRIDE; i += blockDim.x) counter[i] = 0;
  const int v = batch_view_of(b.blk_base, b.n, blockIdx.x);
  const int N = views[v].k.W * views[v].k.H, pb = views[v].px_base;
  const int e0 = ebase[v];
  const int p0 = (blockIdx.x - b.blk_base[v]) * HDOF_BATCH_PX_BLOCK;
  for (int i = threadIdx.x; i < HDOF_BATCH_PX_BLOCK; i += blockDim.x) {
    const int p = p0 + i;
    if (p >= N) break;
    const int s = spp[pb + p];
    if (s == 0) continue;
    const long o = (long)offsets[pb + p] + e0;
    for (int j = 0; j < s; ++j)
      if (o + j >= 0 && o + j < cap) queue[o + j] = pb + p;
  }
}

// the trace planes are written at traced pixels only (the composite reads
// them nowhere else)
__global__ void k_rt_reduce_batch(const uint8_t* __restrict__ spp, const int* __restrict__ offsets,
                                  const ViewK* __restrict__ views, PxBatch b, const int* __restrict__ ebase,
                                  const float* __restrict__ ray_col, const float* __restrict__ ray_z, size_t cap,
                                  float* __restrict__ cn, float* __restrict__ cf, float* __restrict__ h,
                                  float* __restrict__ m1, float* __restrict__ m2) {
  const int v = batch_view_of(b.blk_base, b.n, blockIdx.x);
  const int N = views[v].k.W * views[v].k.H;
  const size_t pb = (size_t)views[v].px_base;
  const LensK l = views[v].l;
  const CamK k = views[v].k;
  VarFuse vf{};
  vf.sparse_rt = 1;
  const int p0 = (blockIdx.x - b.blk_base[v]) * HDOF_BATCH_PX_BLOCK;
  for (int i = threadIdx.x; i < HDOF_BATCH_PX_BLOCK; i += blockDim.x) {
    const int p = p0 + i;
    if (p >= N) break;
    if (spp[pb + p] == 0) continue;  // the planes are written at traced pixels only
    rt_reduce_px<false, false>(p, spp + pb, offsets + pb, N, ebase + v, ray_col, ray_z, cap, l, cn + 3 * pb,
                               cf + 3 * pb, h + pb, m1 + pb, m2 + pb, k, 0u, 0u, 0u, nullptr, vf, nullptr);
  }
}

// batch: first queue entry of each view and the batch total
__global__ void k_view_scan(const int* __restrict__ totals, int n, int* __restrict__ ebase,
                            int* __restrict__ grand) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  long run = 0;
  for (int v = 0; v < n; ++v) {
    ebase[v] = (int)run;
    run += totals[v];
  }
  *grand = (int)min(run, (long)0x7fffffff);
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

template <bool BATCH>
void launch_trace_kernel(hdof_ctx* ctx, const TraceArgs& A, hipStream_t st) {
  const int grid = ctx->n_cu * ctx->tune.blocks_per_cu;
  void (*kern)(TraceArgs);
  // automatic form: by the scene's triangle count (n_nodes + 1 for the binary tree)
  const bool wave = ctx->tune.wave == 1 || (ctx->tune.wave == 2 && A.n_nodes + 1 >= HDOF_WAVE_AUTO_TRIS);
  if (wave)
    kern = ctx->count_on ? k_trace_wave<true, BATCH> : k_trace_wave<false, BATCH>;
  else
    kern = ctx->count_on ? k_trace<true, BATCH> : k_trace<false, BATCH>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(HDOF_TRACE_BLOCK), 0, st, A);
}

__global__ void k_zero_f(float* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

TraceArgs base_args(hdof_ctx* ctx, const hdof_scene* sc, const LightK& li, size_t cap) {
  TraceArgs A{};
  A.nodes = sc->nodes;
  A.tris = sc->tris;
  A.n_nodes = sc->n_nodes;
  A.albedo = sc->albedo;
  A.spec = (const float2*)sc->spec;
  A.li = li;
  A.queue = (const int*)ctx->queue.p;
  A.counter = (int*)ctx->work_counter.p;
  A.ray_col = (float*)ctx->ray_col.p;
  A.cap = cap;
  A.flags = ctx->d_flags;
  A.counters = ctx->d_counters;
  A.refill = ctx->tune.refill;
  A.segments = ctx->tune.segments;
  A.ray_quantum = ctx->trace_ray_quantum;
  A.n_cu = ctx->n_cu;
  A.bpc = ctx->tune.blocks_per_cu;
  return A;
}

}  // namespace

// done (nullable): an event the G-buffer's own dispatch completes (its
// completion signal, with no marker packet between it and the next kernel
// on st)
hdof_status launch_gbuffer(hdof_ctx* ctx, const hdof_scene* sc, const CamK& k, const LensK& l,
                           const LightK& li, hdof_gbuffer_bufs out, hipStream_t st, float4* pack, float* tile_r,
                           hipEvent_t done) {
  int nb = cdiv(k.W, 16) * cdiv(k.H, 16);
  auto kern = ctx->count_on ? (pack ? k_gbuffer<true, true> : k_gbuffer<true, false>)
                            : (pack ? k_gbuffer<false, true> : k_gbuffer<false, false>);
  if (done)
    hipExtLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, st, nullptr, done, 0, sc->nodes, sc->tris, sc->n_nodes,
                          sc->albedo, (const float2*)sc->spec, sc->spec ? out.spec : nullptr, k, l, li, out.depth,
                          out.normal, out.albedo, out.color, out.tri_id, ctx->d_flags, ctx->d_counters, pack,
                          tile_r);
  else
    hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, st, sc->nodes, sc->tris, sc->n_nodes, sc->albedo,
                       (const float2*)sc->spec, sc->spec ? out.spec : nullptr, k, l, li, out.depth, out.normal,
                       out.albedo, out.color, out.tri_id, ctx->d_flags, ctx->d_counters, pack, tile_r);
  // a Lambertian scene has no specular part: its plane is 0
  if (!sc->spec && out.spec) hipLaunchKernelGGL(k_zero_f, dim3(cdiv(k.W * k.H, 256)), dim3(256), 0, st, out.spec,
                                                k.W * k.H);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

hdof_status launch_gbuffer_batched(hdof_ctx* ctx, const hdof_scene* sc, const LightK& li, int n_views,
                                   const BatchView* hviews, const void* views_dev, hdof_gbuffer_bufs out,
                                   float4* pack, float* tile_r, hipStream_t st) {
  GbBatch gbb;
  gbb.n = n_views;
  gbb.blk_base[0] = 0;
  for (int v = 0; v < n_views; ++v)
    gbb.blk_base[v + 1] = gbb.blk_base[v] + cdiv(hviews[v].k.W, 16) * cdiv(hviews[v].k.H, 16);
  for (int v = n_views + 1; v <= HDOF_MAX_VIEWS; ++v) gbb.blk_base[v] = gbb.blk_base[n_views];
  hipLaunchKernelGGL(k_gbuffer_batch, dim3(gbb.blk_base[n_views]), dim3(256), 0, st, sc->nodes, sc->tris,
                     sc->n_nodes, sc->albedo, li, (const ViewK*)views_dev, gbb, out.depth, out.normal, out.albedo,
                     out.color, out.tri_id, ctx->d_flags, pack, tile_r);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

hdof_status reserve_trace(hdof_ctx* ctx, size_t cap, bool own_depth) {
  hdof_status s;
  if ((s = hdof_ensure(ctx->queue, sizeof(int) * cap)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->ray_col, sizeof(float) * 3 * cap)) != HDOF_OK) return s;
  if (own_depth && (s = hdof_ensure(ctx->ray_z, sizeof(float) * cap)) != HDOF_OK) return s;
  if ((s = hdof_ensure(ctx->work_counter, sizeof(int) * 8 * HDOF_SEG_STRIDE)) != HDOF_OK) return s;
  return HDOF_OK;
}

hdof_status launch_trace(hdof_ctx* ctx, const hdof_scene* sc, const CamK& k, const LensK& l,
                         const LightK& li, int spp_max, const uint8_t* spp, const int32_t* offsets,
                         const int32_t* total, uint32_t seed, uint32_t frame, uint32_t view,
                         hdof_rt_bufs out, int32_t* ray_id, float* ray_depth, float* far_pos, hipStream_t st,
                         const VarFuse* vf, bool queue_ready, float* coc_nf) {
  const int N = k.W * k.H;
  const size_t cap = (size_t)N * (size_t)spp_max;
  hdof_status s;
  if ((s = reserve_trace(ctx, cap, !ray_depth)) != HDOF_OK) return s;
  float* rz = ray_depth ? ray_depth : (float*)ctx->ray_z.p;
  if (!queue_ready)
    hipLaunchKernelGGL(k_queue_fill, dim3(cdiv(N, 256)), dim3(256), 0, st, spp, offsets, N, (const int*)nullptr,
                       0, (long)cap, (int*)ctx->queue.p, (int*)ctx->work_counter.p);
  hdof_prof_mark(ctx, 3, st);
  TraceArgs A = base_args(ctx, sc, li, cap);
  A.offsets = offsets;
  A.total_p = total;
  A.ray_z = rz;
  A.ray_id = ray_id;
  A.v0 = ViewK{k, l, seed, frame, view, 0};
  launch_trace_kernel<false>(ctx, A, st);
  hdof_prof_mark(ctx, 4, st);
  const VarFuse vz = vf ? *vf : VarFuse{};
  auto kern = far_pos ? (vf ? k_rt_reduce<true, true> : k_rt_reduce<true, false>)
                      : (vf ? k_rt_reduce<false, true> : k_rt_reduce<false, false>);
  hipLaunchKernelGGL(kern, dim3(cdiv(N, 256)), dim3(256), 0, st, spp, offsets, N, (const int*)nullptr,
                     (const float*)ctx->ray_col.p, (const float*)rz, cap, l, out.c_near, out.c_far, out.hit_ratio,
                     out.lum_m1, out.lum_m2, k, seed, frame, view, far_pos, vz, coc_nf);
  if (!vf) hdof_prof_mark(ctx, 5, st);  // fused: the variance update stage is part of this one
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

// Batched trace: the views' masks have written per-view counts, view-local
// offsets and totals[v]; one scan gives each view's first queue entry, each
// view fills its part of the queue, ONE persistent launch traces all views,
// then each view reduces its own pixels.  `views` is the device copy of
// `hviews` (same order).
hdof_status launch_trace_batched(hdof_ctx* ctx, const hdof_scene* sc, const LightK& li, int spp_max,
                                 int n_views, const BatchView* hviews, const void* views_dev,
                                 const uint8_t* spp, const int32_t* offsets, const int32_t* totals,
                                 int32_t* ebase, int32_t* grand, hdof_rt_bufs* rt, hipStream_t st) {
  long npx = 0;
  for (int v = 0; v < n_views; ++v) npx += (long)hviews[v].k.W * hviews[v].k.H;
  const size_t cap = (size_t)npx * (size_t)spp_max;
  hdof_status s;
  if ((s = reserve_trace(ctx, cap, true)) != HDOF_OK) return s;
  PxBatch pxb{};
  pxb.n = n_views;
  for (int v = 0; v < n_views; ++v)
    pxb.blk_base[v + 1] = pxb.blk_base[v] + cdiv(hviews[v].k.W * hviews[v].k.H, HDOF_BATCH_PX_BLOCK);
  hipLaunchKernelGGL(k_view_scan, dim3(1), dim3(64), 0, st, totals, n_views, ebase, grand);
  hipLaunchKernelGGL(k_queue_fill_batch, dim3(pxb.blk_base[n_views]), dim3(256), 0, st, spp, offsets,
                     (const ViewK*)views_dev, pxb, (const int*)ebase, (long)cap, (int*)ctx->queue.p,
                     (int*)ctx->work_counter.p);
  TraceArgs A = base_args(ctx, sc, li, cap);
  A.offsets = offsets;
  A.total_p = grand;
  A.ray_z = (float*)ctx->ray_z.p;
  A.ray_id = nullptr;
  A.views = (const ViewK*)views_dev;
  A.entry_base = ebase;
  A.n_views = n_views;
  A.v0 = ViewK{hviews[0].k, hviews[0].l, 0, 0, 0, 0};
  launch_trace_kernel<true>(ctx, A, st);
  hipLaunchKernelGGL(k_rt_reduce_batch, dim3(pxb.blk_base[n_views]), dim3(256), 0, st, spp, offsets,
                     (const ViewK*)views_dev, pxb, (const int*)ebase, (const float*)ctx->ray_col.p,
                     (const float*)ctx->ray_z.p, cap, rt->c_near, rt->c_far, rt->hit_ratio, rt->lum_m1,
                     rt->lum_m2);
  HDOF_HIP(hipGetLastError());
  return HDOF_OK;
}

size_t batch_view_bytes() { return sizeof(ViewK); }

void batch_view_pack(const BatchView* hv, int n, void* out) {
  ViewK* o = (ViewK*)out;
  for (int v = 0; v < n; ++v) o[v] = ViewK{hv[v].k, hv[v].l, hv[v].seed, hv[v].frame, hv[v].view, hv[v].px_base};
}
