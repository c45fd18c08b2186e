/*
 * hdof_oracle.c -- plain FP64 CPU oracle of the hybrid depth-of-field hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers.  The GPU library never
 * links, loads or calls this file and shares no code with it: the two sides
 * are written independently from the same reading of the paper
 * (Tan, Chua, Biette, Bhojan: "Hybrid DoF: Ray-Traced and Post-Processed
 * Hybrid Depth of Field Effect for Real-Time Rendering", SIGGRAPH 2020 posters).
 *
 * Everything is double precision; inputs arrive as float32 values widened
 * exactly by the caller.  Loops are the plainest form of each step; OpenMP
 * only splits independent pixels or rays over host threads.
 *
 * Map of the paper to the functions here (section names of the paper):
 *   Design (thin lens of Potmesil & Chakravarty, near/far by the focus plane)
 *       or_coc, or_lens_ray
 *   Design (G-buffer with a sharp rasterised image, deferred shading)
 *       or_gbuffer, shade()
 *   Ray Trace (adaptive ray mask: Gaussian, Sobel on normal and depth,
 *   temporally accumulated luminance variance)
 *       or_mask, or_var_reproject, or_var_update
 *   Ray Trace (lens samples in a circle, near/far split by Z, hit ratio)
 *       or_trace
 *   Reconstruction (temporal: EMA, near/far reprojection, hit-ratio
 *   normalisation)
 *       or_recon
 *   Design (post-process filter) + Reconstruction (CoC-radius rejection)
 *       or_postfilter
 *   Composite (focus zone below sqrt(2), near rule, far hit-ratio blend)
 *       or_composite
 * Closest hits come from a median-split BVH over the triangles and carry an
 * ambiguity flag: a ray is ambiguous when another correct implementation in
 * a different precision could legitimately pick a different triangle.
 *
 * Parity unpinned: none of these functions is left without a pin; the only
 * unpinned claim is whole-frame visual fidelity against the paper's images,
 * which are not available.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_ZMAX 1.0e4
#define OR_SQRT2 1.4142135623730951
#define OR_PI 3.14159265358979323846
#define OR_EPS 1.0e-5      /* ambiguity band: edges, ties, thresholds */
#define OR_BOX_MARGIN 1.0e-3 /* absolute box growth so near misses are visited */
#define OR_LEAF 4
#define OR_MAX_CAND 96

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */
static inline void v_sub(const double* a, const double* b, double* o) { o[0]=a[0]-b[0]; o[1]=a[1]-b[1]; o[2]=a[2]-b[2]; }
static inline double v_dot(const double* a, const double* b) { return a[0]*b[0]+a[1]*b[1]+a[2]*b[2]; }
static inline void v_cross(const double* a, const double* b, double* o) {
  o[0] = a[1]*b[2] - a[2]*b[1];
  o[1] = a[2]*b[0] - a[0]*b[2];
  o[2] = a[0]*b[1] - a[1]*b[0];
}
static inline double v_len(const double* a) { return sqrt(v_dot(a, a)); }
static inline double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }
static inline double maxd(double a, double b) { return a > b ? a : b; }
static inline double mind(double a, double b) { return a < b ? a : b; }

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* Camera and thin lens                                                       */
/* cam[13] = eye(3), right(3), up(3), fwd(3), tan_half_fov_x                  */
/* lens[6] = focal length f, aperture diameter A, focus distance S1, blades   */
/* B (0: a disk, else a regular B-gon, B >= 3, of circumradius A/2),        */
/* rotation theta of its first vertex (rad), spherical aberration s_a        */
/* (relative weight 1 + s_a (2 rho^2 - 1) of a lens sample at normalised    */
/* radius rho, clamped at 0).  The CoC stays the circumscribed circle's.    */
/* ------------------------------------------------------------------------- */
typedef struct {
  double e[3], r[3], u[3], w[3];
  double tx, ty, spx;
  int W, H;
} cam_t;

static cam_t mk_cam(const double* c, int W, int H) {
  cam_t k;
  for (int i = 0; i < 3; ++i) { k.e[i]=c[i]; k.r[i]=c[3+i]; k.u[i]=c[6+i]; k.w[i]=c[9+i]; }
  k.tx = c[12];
  k.ty = c[12] * (double)H / (double)W;     /* square pixels */
  k.spx = (double)W / (2.0 * c[12]);         /* pixels per unit of tan-space */
  k.W = W; k.H = H;
  return k;
}

/* Direction through the centre of pixel (x, y) with unit forward component:
 * v = w + sx r + sy u, image y pointing down, centres at +0.5. */
static void pixel_dir(const cam_t* k, int x, int y, double* v) {
  double sx = (2.0 * (x + 0.5) / k->W - 1.0) * k->tx;
  double sy = (1.0 - 2.0 * (y + 0.5) / k->H) * k->ty;
  for (int i = 0; i < 3; ++i) v[i] = k->w[i] + sx * k->r[i] + sy * k->u[i];
}

/* Signed circle-of-confusion diameter in pixels for axial depth z under the
 * thin-lens model: A (1/S1 - 1/z) s_px.  Negative in front of the focus plane
 * (near field), positive behind it (far field). */
static double coc_px(const cam_t* k, const double* lens, double z) {
  return lens[1] * (1.0 / lens[2] - 1.0 / z) * k->spx;
}

double or_coc(const double* cam, int W, int H, const double* lens, double z) {
  cam_t k = mk_cam(cam, W, H);
  return coc_px(&k, lens, z);
}

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11). */
/* Ten rounds of two 64x64->128 multiplies; the key is bumped by the two      */
/* Weyl constants between rounds.                                             */
/* ------------------------------------------------------------------------- */
static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PH_M1 = 0xCA5A826395121157ULL;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PH_W1 = 0xBB67AE8584CAA73BULL;

void or_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += PH_W0; k1 += PH_W1; }
    unsigned __int128 p0 = (unsigned __int128)PH_M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)PH_M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Lens-sample uniforms: the top 24 bits of the first two outputs, scaled by
 * 2^-24 (exact in both float and double).  Counter = (pixel, sample, view, 0),
 * key = (seed, frame). */
static void lens_uniforms(uint64_t pix, uint64_t j, uint64_t view, uint64_t seed, uint64_t frame,
                          double* u0, double* u1) {
  uint64_t c[4] = {pix, j, view, 0}, kk[2] = {seed, frame}, o[4];
  or_philox4x64_10(c, kk, o);
  *u0 = (double)(o[0] >> 40) * (1.0 / 16777216.0);
  *u1 = (double)(o[1] >> 40) * (1.0 / 16777216.0);
}

/* Relative weight of a lens sample (or post-filter tap) at normalised     */
/* radius rho under spherical aberration s_a (our reading of the paper's    */
/* future work on the relative weight of samples): 1 + s_a (2 rho^2 - 1),  */
/* clamped at 0; 1 for s_a = 0.                                             */
static double sa_weight(double sa, double rho) { return maxd(0.0, 1.0 + sa * (2.0 * rho * rho - 1.0)); }

/* The boundary radius of the regular B-gon of circumradius 1 whose first  */
/* vertex is at angle theta, in direction phi.                              */
static double poly_radius(int B, double theta, double phi) {
  double sector = 2.0 * OR_PI / B;
  double a = fmod(phi - theta, sector);
  if (a < 0.0) a += sector;
  return cos(OR_PI / B) / cos(a - OR_PI / B);
}

/* Thin-lens ray for sample j of pixel p: a uniform point on the aperture,
 * aimed through the point where the pixel's pinhole ray meets the focus
 * plane.  Disk (B = 0): radius A/2, polar mapping sqrt(u0), 2 pi u1.
 * Regular B-gon of circumradius a = A/2 (our reading of the paper's future
 * work on aperture silhouettes): the fan triangle k = floor(B u0) from the
 * centre to vertices k, k + 1, and in it the point sqrt(f) ((1 - u1) V_k +
 * u1 V_k+1), f = B u0 - k (uniform over the triangle, so over the polygon).
 * Origin O = e + l, direction D = S1 v - l (not normalised; D . w = S1, so
 * axial depth = t S1).  *w_out = the spherical-aberration weight of the
 * sample (1 for s_a = 0). */
static void lens_ray(const cam_t* k, const double* lens, int x, int y, uint64_t j,
                     uint64_t seed, uint64_t frame, uint64_t view, int pinhole,
                     double* O, double* D, double* w_out) {
  double v[3];
  pixel_dir(k, x, y, v);
  double l[3] = {0, 0, 0}, rho_n = 0.0;
  if (!pinhole) {
    double u0, u1, lx, ly;
    lens_uniforms((uint64_t)y * k->W + x, j, view, seed, frame, &u0, &u1);
    double a = 0.5 * lens[1];
    int B = (int)lens[3];
    if (B >= 3) {
      int kk = (int)floor(u0 * B);
      if (kk > B - 1) kk = B - 1;
      double f = u0 * B - kk, sq = sqrt(f);
      double t0 = lens[4] + 2.0 * OR_PI * kk / B, t1 = lens[4] + 2.0 * OR_PI * (kk + 1) / B;
      lx = a * sq * ((1.0 - u1) * cos(t0) + u1 * cos(t1));
      ly = a * sq * ((1.0 - u1) * sin(t0) + u1 * sin(t1));
    } else {
      double rho = a * sqrt(u0);
      double th = 2.0 * OR_PI * u1;
      lx = rho * cos(th);
      ly = rho * sin(th);
    }
    rho_n = a > 0.0 ? sqrt(lx * lx + ly * ly) / a : 0.0;
    for (int i = 0; i < 3; ++i) l[i] = lx * k->r[i] + ly * k->u[i];
  }
  for (int i = 0; i < 3; ++i) { O[i] = k->e[i] + l[i]; D[i] = lens[2] * v[i] - l[i]; }
  if (w_out) *w_out = sa_weight(lens[5], rho_n);
}

void or_lens_ray(const double* cam, int W, int H, const double* lens, int x, int y, uint64_t j,
                 uint64_t seed, uint64_t frame, uint64_t view, int pinhole, double* O, double* D, double* w) {
  cam_t k = mk_cam(cam, W, H);
  lens_ray(&k, lens, x, y, j, seed, frame, view, pinhole, O, D, w);
}

/* ------------------------------------------------------------------------- */
/* Scene + median-split BVH                                                   */
/* ------------------------------------------------------------------------- */
typedef struct { double lo[3], hi[3]; int left, right, first, count; } onode_t;

typedef struct {
  int n;
  double* v;    /* n * 9 */
  double* alb;  /* n * 3 */
  double* spec; /* n * 2 (k_s, shininess) or NULL: Lambertian */
  int* idx;     /* permutation of triangles, leaves own contiguous ranges */
  onode_t* nodes;
  int nnodes;
  double* cen;  /* centroids, n * 3 (build only) */
} or_scene;

static void tri_bounds(const or_scene* s, int t, double* lo, double* hi) {
  const double* v = s->v + 9 * (size_t)t;
  for (int a = 0; a < 3; ++a) {
    lo[a] = mind(v[a], mind(v[3 + a], v[6 + a]));
    hi[a] = maxd(v[a], maxd(v[3 + a], v[6 + a]));
  }
}

/* quickselect on idx[lo, hi) by centroid coordinate `axis` so that position
 * `k` holds the element of rank k (nth_element). */
static void select_kth(const or_scene* s, int* idx, int lo, int hi, int k, int axis) {
  while (hi - lo > 1) {
    int mid = lo + (hi - lo) / 2;
    double pv = s->cen[3 * (size_t)idx[mid] + axis];
    int i = lo, j = hi - 1;
    while (i <= j) {
      while (s->cen[3 * (size_t)idx[i] + axis] < pv) ++i;
      while (s->cen[3 * (size_t)idx[j] + axis] > pv) --j;
      if (i <= j) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; ++i; --j; }
    }
    if (k <= j) hi = j + 1;
    else if (k >= i) lo = i;
    else return;
  }
}

static int build_rec(or_scene* s, int first, int count) {
  int id = s->nnodes++;
  onode_t* nd = &s->nodes[id];
  for (int a = 0; a < 3; ++a) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = first; i < first + count; ++i) {
    double lo[3], hi[3];
    tri_bounds(s, s->idx[i], lo, hi);
    for (int a = 0; a < 3; ++a) {
      nd->lo[a] = mind(nd->lo[a], lo[a]); nd->hi[a] = maxd(nd->hi[a], hi[a]);
      double c = s->cen[3 * (size_t)s->idx[i] + a];
      clo[a] = mind(clo[a], c); chi[a] = maxd(chi[a], c);
    }
  }
  if (count <= OR_LEAF) {
    nd->left = nd->right = -1; nd->first = first; nd->count = count;
    return id;
  }
  int axis = 0;
  for (int a = 1; a < 3; ++a) if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
  int half = count / 2;
  select_kth(s, s->idx, first, first + count, first + half, axis);
  nd->count = 0; nd->first = -1;
  int l = build_rec(s, first, half);
  int r = build_rec(s, first + half, count - half);
  s->nodes[id].left = l; s->nodes[id].right = r;
  return id;
}

or_scene* or_scene_create(const double* verts, const double* albedo, int n) {
  or_scene* s = (or_scene*)calloc(1, sizeof(or_scene));
  s->n = n;
  s->v = (double*)malloc(sizeof(double) * 9 * (size_t)n);
  s->alb = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  memcpy(s->v, verts, sizeof(double) * 9 * (size_t)n);
  memcpy(s->alb, albedo, sizeof(double) * 3 * (size_t)n);
  s->idx = (int*)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  s->cen = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) {
    s->idx[i] = i;
    for (int a = 0; a < 3; ++a)
      s->cen[3 * (size_t)i + a] = (s->v[9 * (size_t)i + a] + s->v[9 * (size_t)i + 3 + a] + s->v[9 * (size_t)i + 6 + a]) / 3.0;
  }
  s->nodes = (onode_t*)malloc(sizeof(onode_t) * (size_t)(2 * (n > 0 ? n : 1)));
  s->nnodes = 0;
  if (n > 0) build_rec(s, 0, n);
  free(s->cen); s->cen = NULL;
  return s;
}

void or_scene_destroy(or_scene* s) {
  if (!s) return;
  free(s->v); free(s->alb); free(s->spec); free(s->idx); free(s->nodes); free(s);
}

/* specular materials per triangle (input order): k_s >= 0, shininess >= 1; */
/* NULL makes every triangle Lambertian again                               */
void or_scene_set_spec(or_scene* s, const double* spec) {
  free(s->spec);
  s->spec = NULL;
  if (!spec) return;
  s->spec = (double*)malloc(sizeof(double) * 2 * (size_t)(s->n > 0 ? s->n : 1));
  memcpy(s->spec, spec, sizeof(double) * 2 * (size_t)s->n);
}

int or_scene_nodes(const or_scene* s) { return s->nnodes; }

/* ------------------------------------------------------------------------- */
/* Closest hit with ambiguity                                                 */
/* ------------------------------------------------------------------------- */
typedef struct { double t, mu; int id; } cand_t;

/* Angular margin of the ray (O, D) against triangle t.  For each edge (i, j)
 * the quantity  Dn . (a_i x a_j) / |a_i x a_j|  (a = vertex - O, Dn = unit D)
 * is the sine of the angle between the ray and the plane through O and that
 * edge.  The ray passes through the triangle iff the three have one sign;
 * mu = the smallest of them after orienting by that sign is positive inside
 * (the angular distance to the nearest edge) and negative outside.
 * t is the parameter of the hit with the triangle's plane.  Returns 0 for
 * degenerate triangles and rays parallel to the plane. */
static int tri_eval(const or_scene* s, int tri, const double* O, const double* D, const double* Dn,
                    double* t_out, double* mu_out) {
  const double* v = s->v + 9 * (size_t)tri;
  double a0[3], a1[3], a2[3];
  v_sub(v, O, a0); v_sub(v + 3, O, a1); v_sub(v + 6, O, a2);
  double c01[3], c12[3], c20[3];
  v_cross(a0, a1, c01); v_cross(a1, a2, c12); v_cross(a2, a0, c20);
  double l01 = v_len(c01), l12 = v_len(c12), l20 = v_len(c20);
  double e01 = v_dot(Dn, c01), e12 = v_dot(Dn, c12), e20 = v_dot(Dn, c20);
  double sum = e01 + e12 + e20;
  double e1[3], e2[3], n[3];
  v_sub(v + 3, v, e1); v_sub(v + 6, v, e2); v_cross(e1, e2, n);
  double den = v_dot(n, D);
  if (den == 0.0 || sum == 0.0) return 0;
  if (l01 == 0.0 || l12 == 0.0 || l20 == 0.0) return 0;
  double sg = sum > 0 ? 1.0 : -1.0;
  double m0 = sg * e01 / l01, m1 = sg * e12 / l12, m2 = sg * e20 / l20;
  *mu_out = mind(m0, mind(m1, m2));
  *t_out = v_dot(n, a0) / den;
  return 1;
}

static int box_hit(const onode_t* nd, const double* O, const double* invD, double tlim) {
  double t0 = 0.0, t1 = tlim;
  for (int a = 0; a < 3; ++a) {
    double lo = nd->lo[a] - OR_BOX_MARGIN, hi = nd->hi[a] + OR_BOX_MARGIN;
    if (isinf(invD[a])) {
      if (O[a] < lo || O[a] > hi) return 0;
      continue;
    }
    double ta = (lo - O[a]) * invD[a], tb = (hi - O[a]) * invD[a];
    if (ta > tb) { double x = ta; ta = tb; tb = x; }
    t0 = maxd(t0, ta); t1 = mind(t1, tb);
    if (t0 > t1) return 0;
  }
  return 1;
}

typedef struct { double t; int id; int amb; } ohit_t;

/* Closest hit: smallest t > 0 among triangles the ray passes through
 * (boundary counts as inside), ties to the lowest triangle index.  The ray is
 * ambiguous when the chosen triangle is within OR_EPS (angular) of an edge,
 * when another triangle within OR_EPS of being hit lies closer, or when a
 * second hit lies within relative OR_EPS in t. */
static ohit_t cast_ray(const or_scene* s, const double* O, const double* D, int brute) {
  double dl = v_len(D);
  double Dn[3] = {D[0] / dl, D[1] / dl, D[2] / dl};
  double invD[3];
  for (int a = 0; a < 3; ++a) invD[a] = D[a] != 0.0 ? 1.0 / D[a] : INFINITY;
  cand_t cand[OR_MAX_CAND];
  int nc = 0, overflow = 0;
  double tbest = INFINITY;
  int best = -1;
  double best_mu = 0.0;

#define OR_CONSIDER(tri)                                                         \
  do {                                                                           \
    double tt, mu;                                                               \
    if (tri_eval(s, (tri), O, D, Dn, &tt, &mu) && tt > 0.0 && mu > -OR_EPS) {    \
      if (nc < OR_MAX_CAND) { cand[nc].t = tt; cand[nc].mu = mu; cand[nc].id = (tri); ++nc; } \
      else overflow = 1;                                                         \
      if (mu >= 0.0 && (tt < tbest || (tt == tbest && (tri) < best))) {          \
        tbest = tt; best = (tri); best_mu = mu;                                  \
      }                                                                          \
    }                                                                            \
  } while (0)

  if (brute || s->nnodes == 0) {
    for (int tri = 0; tri < s->n; ++tri) OR_CONSIDER(tri);
  } else {
    int stack[256], sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
      const onode_t* nd = &s->nodes[stack[--sp]];
      double tlim = isinf(tbest) ? INFINITY : tbest * (1.0 + 4.0 * OR_EPS) + OR_BOX_MARGIN;
      if (!box_hit(nd, O, invD, tlim)) continue;
      if (nd->count > 0) {
        for (int i = nd->first; i < nd->first + nd->count; ++i) OR_CONSIDER(s->idx[i]);
      } else {
        if (sp + 2 > 256) { overflow = 1; break; }
        stack[sp++] = nd->right;
        stack[sp++] = nd->left;
      }
    }
  }
#undef OR_CONSIDER
  ohit_t h;
  h.t = tbest; h.id = best; h.amb = overflow;
  if (best >= 0 && best_mu < OR_EPS) h.amb = 1;
  for (int i = 0; i < nc; ++i) {
    if (cand[i].id == best) continue;
    if (best < 0) { h.amb = 1; break; }          /* a near miss on a missing ray */
    if (cand[i].t <= tbest * (1.0 + OR_EPS)) { h.amb = 1; break; }
  }
  return h;
}

/* Batch of rays: O, D are n*3; outputs t (inf on miss), id (-1 on miss), amb. */
void or_cast_rays(const or_scene* s, int n, const double* O, const double* D, int brute,
                  double* t, int* id, int* amb) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < n; ++i) {
    ohit_t h = cast_ray(s, O + 3 * (size_t)i, D + 3 * (size_t)i, brute);
    t[i] = h.t; id[i] = h.id; amb[i] = h.amb;
  }
}

/* ------------------------------------------------------------------------- */
/* Shading (our reading of the paper's deferred shading): two-sided Lambertian */
/* normal, one point light with inverse-square falloff, ambient term, no      */
/* shadow rays.  light[9] = position, rgb intensity, rgb ambient.             */
/* Specular materials (the bright highlights whose bokeh the paper's         */
/* composite treats apart): a Blinn-Phong lobe added to the colour,          */
/* k_s I max(0, n.h)^shininess / max(d^2, 1e-4) while the light is on the    */
/* viewer's side (n.l > 0), h the unit half vector of the light direction   */
/* and the direction back along the ray; *ys_out = its luminance.           */
/* ------------------------------------------------------------------------- */
static inline double luminance(const double* L);
static void shade(const or_scene* s, const double* light, int tri, const double* O, const double* D,
                  double t, double* L, double* n_out, double* ys_out) {
  const double* v = s->v + 9 * (size_t)tri;
  double e1[3], e2[3], n[3];
  v_sub(v + 3, v, e1); v_sub(v + 6, v, e2); v_cross(e1, e2, n);
  double nl = v_len(n);
  for (int a = 0; a < 3; ++a) n[a] /= nl;
  if (v_dot(n, D) > 0.0) for (int a = 0; a < 3; ++a) n[a] = -n[a];
  double P[3], l[3];
  for (int a = 0; a < 3; ++a) P[a] = O[a] + t * D[a];
  v_sub(light, P, l);
  double d2 = v_dot(l, l);
  double d = sqrt(d2);
  double cosv = d > 0.0 ? v_dot(n, l) / d : 0.0;
  double irr = maxd(0.0, cosv) / maxd(d2, 1e-4);
  const double* al = s->alb + 3 * (size_t)tri;
  for (int c = 0; c < 3; ++c) L[c] = al[c] * (light[6 + c] + light[3 + c] * irr);
  double ys = 0.0;
  if (s->spec && s->spec[2 * (size_t)tri] > 0.0 && cosv > 0.0) {
    double hv[3], dl = v_len(D);
    for (int a = 0; a < 3; ++a) hv[a] = l[a] / d - D[a] / dl;
    double hl = v_len(hv);
    double nh = hl > 0.0 ? maxd(0.0, v_dot(n, hv) / hl) : 0.0;
    double f = s->spec[2 * (size_t)tri] * pow(nh, s->spec[2 * (size_t)tri + 1]) / maxd(d2, 1e-4);
    double Ls[3];
    for (int c = 0; c < 3; ++c) { Ls[c] = f * light[3 + c]; L[c] += Ls[c]; }
    ys = luminance(Ls);
  }
  if (ys_out) *ys_out = ys;
  if (n_out) for (int a = 0; a < 3; ++a) n_out[a] = n[a];
}

static inline double luminance(const double* L) { return 0.2126 * L[0] + 0.7152 * L[1] + 0.0722 * L[2]; }

/* ------------------------------------------------------------------------- */
/* G-buffer: one pinhole ray through each pixel centre (lens offset 0).       */
/* Planar outputs [C][H][W]: depth z (axial, OR_ZMAX on miss), face normal,   */
/* albedo, shaded colour C_r, triangle id (-1 on miss), ambiguity flag.       */
/* `pix` lists linear pixel indices (NULL = all pixels, then n = W*H); the    */
/* outputs are indexed by list position.                                      */
/* ------------------------------------------------------------------------- */
void or_gbuffer(const or_scene* s, const double* cam, int W, int H, const double* lens,
                const double* light, const int64_t* pix, int64_t n,
                double* z, double* nrm, double* alb, double* col, int* id, int* amb, double* spec) {
  cam_t k = mk_cam(cam, W, H);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = pix ? pix[i] : i;
    int x = (int)(p % W), y = (int)(p / W);
    double O[3], D[3];
    lens_ray(&k, lens, x, y, 0, 0, 0, 0, 1, O, D, NULL);
    ohit_t h = cast_ray(s, O, D, 0);
    double L[3] = {0, 0, 0}, nn[3] = {0, 0, 0}, al[3] = {0, 0, 0};
    double zz = OR_ZMAX, ys = 0.0;
    if (h.id >= 0) {
      shade(s, light, h.id, O, D, h.t, L, nn, &ys);
      for (int c = 0; c < 3; ++c) al[c] = s->alb[3 * (size_t)h.id + c];
      zz = h.t * lens[2];
    }
    z[i] = zz;
    for (int c = 0; c < 3; ++c) {
      nrm[(size_t)c * n + i] = nn[c];
      alb[(size_t)c * n + i] = al[c];
      col[(size_t)c * n + i] = L[c];
    }
    id[i] = h.id;
    amb[i] = h.amb;
    if (spec) spec[i] = ys;
  }
}

/* ------------------------------------------------------------------------- */
/* Adaptive ray mask                                                          */
/*  1. Gaussian (sigma; taps exp(-i^2 / 2 sigma^2), radius floor(3 sigma+0.5),*/
/*     normalised; separable x then y; clamp to edge) on min(z, zmax), n.     */
/*  2. 3x3 Sobel (clamp to edge) on the blurred channels:                     */
/*     g_z = |grad z~| / (8 max(z~, 1e-3)),  g_n = sqrt(sum_c |grad n~_c|^2)/8.*/
/*  3. m = max(g_z / tau_z, g_n / tau_n, V / tau_v).                         */
/*  4. s_raw = 0 if m < 1, else min(spp_max, ceil(m)).                       */
/*  5. tile max over tile x tile pixels, then max over tiles within          */
/*     Chebyshev tile distance `dilate`; s(p) = value of p's tile.           */
/*  6. offsets = exclusive prefix sum of s in row-major pixel order.         */
/* s_lo / s_hi bound s when m moves by a relative OR_EPS (threshold ambiguity)*/
/* ------------------------------------------------------------------------- */
static int s_of_m(double m, int spp_max) {
  if (!(m >= 1.0)) return 0;
  if (isinf(m)) return spp_max;
  double c = ceil(m);
  return c >= (double)spp_max ? spp_max : (int)c;
}

void or_gauss_taps(double sigma, int* radius, double* taps /* >= 13 */) {
  int R = (int)floor(3.0 * sigma + 0.5);
  double sum = 0.0;
  for (int i = -R; i <= R; ++i) { taps[i + R] = exp(-(double)(i * i) / (2.0 * sigma * sigma)); sum += taps[i + R]; }
  for (int i = -R; i <= R; ++i) taps[i + R] /= sum;
  *radius = R;
}

static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Mask resolution scaled by the frame's maximum CoC (our reading of the    */
/* paper's Discussion, which plans to scale the ray mask's resolution with  */
/* the maximum CoC against tiling artifacts): R = max over the pixels of    */
/* |c(z)| / 2, tile edge 4 for R < 16 px, 8 for R < 32 px, else 16 (about   */
/* R / 2, within the tile sizes the mask supports).  *r_max receives R.     */
int or_mask_scaled_tile(const double* cam, int W, int H, const double* lens, const double* z, double* r_max) {
  cam_t k = mk_cam(cam, W, H);
  double R = 0.0;
  for (size_t p = 0; p < (size_t)W * H; ++p) R = maxd(R, 0.5 * fabs(coc_px(&k, lens, z[p])));
  if (r_max) *r_max = R;
  return R < 16.0 ? 4 : (R < 32.0 ? 8 : 16);
}

int or_mask(int W, int H, const double* z, const double* nrm, const double* V,
            double sigma, double tau_z, double tau_n, double tau_v,
            int spp_max, int tile, int dilate,
            double* blur /* 4*W*H, may be NULL */, double* gz_out, double* gn_out, double* m_out,
            int* s, int* s_lo, int* s_hi, int64_t* offsets, int64_t* total) {
  size_t N = (size_t)W * H;
  int R;
  double taps[32];
  if (sigma <= 0.0 || sigma > 4.0) return 1;
  or_gauss_taps(sigma, &R, taps);
  double* ch = (double*)malloc(sizeof(double) * 4 * N);
  double* tmp = (double*)malloc(sizeof(double) * 4 * N);
  for (size_t i = 0; i < N; ++i) {
    ch[i] = mind(z[i], OR_ZMAX);
    for (int c = 0; c < 3; ++c) ch[(size_t)(c + 1) * N + i] = nrm[(size_t)c * N + i];
  }
  /* separable Gaussian: x pass then y pass */
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int c = 0; c < 4; ++c)
      for (int x = 0; x < W; ++x) {
        double acc = 0.0;
        for (int i = -R; i <= R; ++i) acc += taps[i + R] * ch[(size_t)c * N + (size_t)y * W + clampi(x + i, 0, W - 1)];
        tmp[(size_t)c * N + (size_t)y * W + x] = acc;
      }
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int c = 0; c < 4; ++c)
      for (int x = 0; x < W; ++x) {
        double acc = 0.0;
        for (int i = -R; i <= R; ++i) acc += taps[i + R] * tmp[(size_t)c * N + (size_t)clampi(y + i, 0, H - 1) * W + x];
        ch[(size_t)c * N + (size_t)y * W + x] = acc;
      }
  if (blur) memcpy(blur, ch, sizeof(double) * 4 * N);
  int* sr = (int*)malloc(sizeof(int) * N);
  int* srl = (int*)malloc(sizeof(int) * N);
  int* srh = (int*)malloc(sizeof(int) * N);
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      double gsq[4];
      for (int c = 0; c < 4; ++c) {
        const double* b = ch + (size_t)c * N;
#define B(xx, yy) b[(size_t)clampi((yy), 0, H - 1) * W + clampi((xx), 0, W - 1)]
        double gx = (B(x + 1, y - 1) - B(x - 1, y - 1)) + 2.0 * (B(x + 1, y) - B(x - 1, y)) + (B(x + 1, y + 1) - B(x - 1, y + 1));
        double gy = (B(x - 1, y + 1) - B(x - 1, y - 1)) + 2.0 * (B(x, y + 1) - B(x, y - 1)) + (B(x + 1, y + 1) - B(x + 1, y - 1));
#undef B
        gsq[c] = gx * gx + gy * gy;
      }
      size_t p = (size_t)y * W + x;
      double gz = sqrt(gsq[0]) / (8.0 * maxd(ch[p], 1e-3));
      double gn = sqrt(gsq[1] + gsq[2] + gsq[3]) / 8.0;
      double vv = V ? V[p] : 0.0;
      double m = maxd(gz / tau_z, maxd(gn / tau_n, vv / tau_v));
      if (gz_out) gz_out[p] = gz;
      if (gn_out) gn_out[p] = gn;
      if (m_out) m_out[p] = m;
      sr[p] = s_of_m(m, spp_max);
      srl[p] = isinf(m) ? spp_max : s_of_m(m * (1.0 - OR_EPS), spp_max);
      srh[p] = isinf(m) ? spp_max : s_of_m(m * (1.0 + OR_EPS), spp_max);
    }
  /* tile max then dilation over tiles */
  int TW = (W + tile - 1) / tile, TH = (H + tile - 1) / tile;
  int* tm = (int*)calloc((size_t)TW * TH * 3, sizeof(int));
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t p = (size_t)y * W + x, t = (size_t)(y / tile) * TW + x / tile;
      if (sr[p] > tm[3 * t]) tm[3 * t] = sr[p];
      if (srl[p] > tm[3 * t + 1]) tm[3 * t + 1] = srl[p];
      if (srh[p] > tm[3 * t + 2]) tm[3 * t + 2] = srh[p];
    }
  int* td = (int*)calloc((size_t)TW * TH * 3, sizeof(int));
  for (int ty = 0; ty < TH; ++ty)
    for (int tx = 0; tx < TW; ++tx)
      for (int dy = -dilate; dy <= dilate; ++dy)
        for (int dx = -dilate; dx <= dilate; ++dx) {
          int yy = ty + dy, xx = tx + dx;
          if (yy < 0 || yy >= TH || xx < 0 || xx >= TW) continue;
          for (int q = 0; q < 3; ++q) {
            int v = tm[3 * ((size_t)yy * TW + xx) + q];
            if (v > td[3 * ((size_t)ty * TW + tx) + q]) td[3 * ((size_t)ty * TW + tx) + q] = v;
          }
        }
  int64_t run = 0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t p = (size_t)y * W + x, t = (size_t)(y / tile) * TW + x / tile;
      s[p] = td[3 * t];
      if (s_lo) s_lo[p] = td[3 * t + 1];
      if (s_hi) s_hi[p] = td[3 * t + 2];
      if (offsets) offsets[p] = run;
      run += s[p];
    }
  if (total) *total = run;
  free(ch); free(tmp); free(sr); free(srl); free(srh); free(tm); free(td);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Thin-lens distributed ray trace + per-pixel reduction                      */
/* For listed pixel i (linear index pix[i]) with s = spp[i] samples:          */
/*   per ray j: lens ray, closest hit, shade -> L_j, axial depth z_j          */
/*   (OR_ZMAX on miss), luminance Y_j (Rec. 709).                              */
/*   near weight w_j = clamp(0.5 - c(z_j) / (2 sqrt 2), 0, 1): 1 in front of */
/*   the focus zone, 0 behind it, linear across |c| <= sqrt 2 (our reading of */
/*   "split ... based on its Z-distance from the separating focus plane").    */
/*   C_tn = sum w L / sum w, C_tf = sum (1-w) L / sum (1-w) (0 if empty),      */
/*   h = sum w / s (hit ratio), lum_m1 = mean Y, lum_m2 = mean Y^2.           */
/*   Under spherical aberration every sum (and s) weights ray j by its lens  */
/*   sample's aberration weight (1 when s_a = 0).                             */
/* Per-ray outputs (nullable) go to ray_base[i] + j; ray_base = exclusive      */
/* prefix sum of spp over the list.  px_amb = any ray of the pixel ambiguous. */
/* far_pos (nullable, 4 planes of n): over the rays that hit, the far-weighted */
/* mean hit point sum (1-w) P / sum (1-w) (planes 0-2) and sum (1-w) (plane */
/* 3); 0 when no ray hits with a far weight.                                  */
/* coc_nf (nullable, 2 planes of n): the average CoC size of the pixel's near */
/* and far rays, sum w |c| / sum w and sum (1-w) |c| / sum (1-w) (0 when the */
/* weight sum is 0; a miss counts at depth OR_ZMAX), the per-frame CoC that  */
/* the spatial reconstruction blends.                                        */
/* ------------------------------------------------------------------------- */
void or_trace(const or_scene* s, const double* cam, int W, int H, const double* lens, const double* light,
              const int64_t* pix, const int* spp, int64_t n, const int64_t* ray_base,
              uint64_t seed, uint64_t frame, uint64_t view,
              int* ray_id, double* ray_z, double* ray_L, int* ray_amb, int64_t n_rays,
              double* c_near, double* c_far, double* hit, double* m1, double* m2, int* px_amb,
              double* far_pos, double* coc_nf) {
  cam_t k = mk_cam(cam, W, H);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = pix ? pix[i] : i;
    int x = (int)(p % W), y = (int)(p / W);
    int ns = spp[i];
    double Nw = 0.0, Fw = 0.0, sn[3] = {0, 0, 0}, sf[3] = {0, 0, 0}, sy = 0.0, sy2 = 0.0;
    double Pw = 0.0, sP[3] = {0, 0, 0}, scn = 0.0, scf = 0.0;
    int pa = 0;
    double Sw = 0.0;  /* sum of the samples' aberration weights (ns for s_a = 0) */
    for (int j = 0; j < ns; ++j) {
      double O[3], D[3], om;
      lens_ray(&k, lens, x, y, (uint64_t)j, seed, frame, view, 0, O, D, &om);
      ohit_t h = cast_ray(s, O, D, 0);
      double L[3] = {0, 0, 0}, zz = OR_ZMAX;
      if (h.id >= 0) { shade(s, light, h.id, O, D, h.t, L, NULL, NULL); zz = h.t * lens[2]; }
      double Y = luminance(L);
      double c = coc_px(&k, lens, zz);
      double w = clampd(0.5 - c / (2.0 * OR_SQRT2), 0.0, 1.0);
      double wn = om * w, wf = om * (1.0 - w);
      Sw += om;
      Nw += wn; Fw += wf;
      scn += wn * fabs(c); scf += wf * fabs(c);
      for (int q = 0; q < 3; ++q) { sn[q] += wn * L[q]; sf[q] += wf * L[q]; }
      if (h.id >= 0) {
        Pw += wf;
        for (int q = 0; q < 3; ++q) sP[q] += wf * (O[q] + h.t * D[q]);
      }
      sy += om * Y; sy2 += om * Y * Y;
      pa |= h.amb;
      if (ray_base) {
        int64_t r = ray_base[i] + j;
        if (r >= 0 && r < n_rays) {
          if (ray_id) ray_id[r] = h.id;
          if (ray_z) ray_z[r] = zz;
          if (ray_L) for (int q = 0; q < 3; ++q) ray_L[(size_t)q * n_rays + r] = L[q];
          if (ray_amb) ray_amb[r] = h.amb;
        }
      }
    }
    for (int q = 0; q < 3; ++q) {
      c_near[(size_t)q * n + i] = Nw > 0.0 ? sn[q] / Nw : 0.0;
      c_far[(size_t)q * n + i] = Fw > 0.0 ? sf[q] / Fw : 0.0;
    }
    hit[i] = Sw > 0.0 ? Nw / Sw : 0.0;
    m1[i] = Sw > 0.0 ? sy / Sw : 0.0;
    m2[i] = Sw > 0.0 ? sy2 / Sw : 0.0;
    if (px_amb) px_amb[i] = pa;
    if (far_pos) {
      for (int q = 0; q < 3; ++q) far_pos[(size_t)q * n + i] = Pw > 0.0 ? sP[q] / Pw : 0.0;
      far_pos[(size_t)3 * n + i] = Pw;
    }
    if (coc_nf) {
      coc_nf[i] = Nw > 0.0 ? scn / Nw : 0.0;
      coc_nf[(size_t)n + i] = Fw > 0.0 ? scf / Fw : 0.0;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Temporally accumulated luminance variance (our reading of the paper's      */
/* SVGF-style estimate, reprojected with depth like Lehtinen et al.)          */
/* History per pixel: lum_m1, lum_m2, flags (bit0 valid, bit1 new), depth.    */
/* Reprojection: X = e + z v; project with the previous camera, round to the  */
/* nearest pixel; valid if in bounds, previous entry valid and               */
/* |z_prev - z_expected| / z_expected <= 0.01.                                */
/* V = +inf if the reprojected entry is new, max(0, m2 - m1^2) if valid,      */
/* 0 if invalid.  amb marks rounding within OR_EPS of a pixel boundary or a   */
/* depth ratio within OR_EPS of the bound.                                    */
/* ------------------------------------------------------------------------- */
#define OR_VALID 1
#define OR_NEW 2

void or_var_reproject(const double* cam, int W, int H, const double* z,
                      const double* pcam, int PW, int PH,
                      const double* pm1, const double* pm2, const int* pflags, const double* pz,
                      double* rm1, double* rm2, int* rflags, double* V, int* amb) {
  cam_t k = mk_cam(cam, W, H), kp = mk_cam(pcam, PW, PH);
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t p = (size_t)y * W + x;
      double v[3], X[3], d[3];
      pixel_dir(&k, x, y, v);
      for (int a = 0; a < 3; ++a) X[a] = k.e[a] + z[p] * v[a];
      v_sub(X, kp.e, d);
      double zc = v_dot(d, kp.w);
      int ok = 0, am = 0;
      double a1 = 0, a2 = 0;
      int fl = 0;
      if (zc > 0.0) {
        double sxp = v_dot(d, kp.r) / zc, syp = v_dot(d, kp.u) / zc;
        double fx = (sxp / kp.tx + 1.0) * 0.5 * PW;
        double fy = (1.0 - syp / kp.ty) * 0.5 * PH;
        double px = floor(fx), py = floor(fy);
        if (fx - px < OR_EPS * maxd(1.0, fabs(fx)) || px + 1.0 - fx < OR_EPS * maxd(1.0, fabs(fx))) am = 1;
        if (fy - py < OR_EPS * maxd(1.0, fabs(fy)) || py + 1.0 - fy < OR_EPS * maxd(1.0, fabs(fy))) am = 1;
        if (px >= 0 && px < PW && py >= 0 && py < PH) {
          size_t q = (size_t)py * PW + (size_t)px;
          if (pflags[q] & OR_VALID) {
            double rel = fabs(pz[q] - zc) / zc;
            if (fabs(rel - 0.01) < OR_EPS) am = 1;
            if (rel <= 0.01) { ok = 1; a1 = pm1[q]; a2 = pm2[q]; fl = pflags[q]; }
          }
        }
      }
      rm1[p] = ok ? a1 : 0.0;
      rm2[p] = ok ? a2 : 0.0;
      rflags[p] = ok ? fl : 0;
      V[p] = ok ? ((fl & OR_NEW) ? INFINITY : maxd(0.0, a2 - a1 * a1)) : 0.0;
      if (amb) amb[p] = am;
    }
}

/* After the trace: EMA with weight alpha where traced with valid history,
 * restart (and mark new) where traced without history, carry where untraced. */
void or_var_update(int W, int H, const int* spp, const double* rm1, const double* rm2, const int* rflags,
                   const double* ybar, const double* y2bar, double alpha, const double* z,
                   double* m1, double* m2, int* flags, double* zh) {
  size_t N = (size_t)W * H;
  for (size_t p = 0; p < N; ++p) {
    if (spp[p] > 0) {
      if (rflags[p] & OR_VALID) {
        m1[p] = (1.0 - alpha) * rm1[p] + alpha * ybar[p];
        m2[p] = (1.0 - alpha) * rm2[p] + alpha * y2bar[p];
        flags[p] = OR_VALID;
      } else {
        m1[p] = ybar[p]; m2[p] = y2bar[p]; flags[p] = OR_VALID | OR_NEW;
      }
    } else {
      m1[p] = rm1[p]; m2[p] = rm2[p]; flags[p] = rflags[p];
    }
    zh[p] = z[p];
  }
}

/* ------------------------------------------------------------------------- */
/* Temporal reconstruction of the near and far ray-traced colours (our        */
/* reading of the paper's Reconstruction section: an exponential moving       */
/* average like TAA, near pixels reprojected by their screen-space motion,    */
/* far pixels through the average world position of their far hits with a    */
/* neighbour fallback, colours composed with the latest hit ratio but         */
/* normalised by the accumulated one).                                        */
/* History per pixel: 8 planes N_r N_g N_b Hn F_r F_g F_b Hf (premultiplied   */
/* near colour h C_tn and its accumulated hit ratio; premultiplied far colour */
/* (1-h) C_tf and the hit ratio accumulated along the far path), a valid     */
/* flag and the depth of the frame that wrote it.                            */
/* For a traced pixel p with hit ratio h:                                     */
/*   near: X = e + z v (the G-buffer surface), nearest previous pixel q_n;    */
/*     usable if the previous camera exists, q_n is inside and valid and      */
/*     |z_prev - z_expected| / z_expected <= 0.01.                            */
/*   far: X_f = p's far-hit mean if its far weight > 0, else the plain mean   */
/*     of the far-hit means of its 8 neighbours that have one; nearest        */
/*     previous pixel q_f; usable if X_f exists, q_f is inside and valid.     */
/*   N' = (1-a) N(q_n) + a h C_tn, Hn' = (1-a) Hn(q_n) + a h   (else h C_tn, h)*/
/*   F' = (1-a) F(q_f) + a (1-h) C_tf, Hf' = (1-a) Hf(q_f) + a h              */
/*                                              (else (1-h) C_tf, h)          */
/*   out near = N'/Hn' (C_tn if Hn' = 0), out far = F'/(1-Hf') (C_tf if       */
/*   Hf' = 1); the composite then mixes them with the latest h.               */
/* Untraced pixels: colours unchanged, history invalid.  amb marks a rounded  */
/* coordinate within OR_EPS of a pixel boundary, a depth ratio within OR_EPS  */
/* of the bound, or an ambiguous ray (trace px_amb) in p or in the           */
/* neighbours its far position comes from.                                    */
/* ------------------------------------------------------------------------- */
static int reproj_px(const cam_t* kp, int PW, int PH, const double* X, size_t* q, double* zc, int* am) {
  double d[3];
  v_sub(X, kp->e, d);
  *zc = v_dot(d, kp->w);
  if (!(*zc > 0.0)) return 0;
  double sxp = v_dot(d, kp->r) / *zc, syp = v_dot(d, kp->u) / *zc;
  double fx = (sxp / kp->tx + 1.0) * 0.5 * PW;
  double fy = (1.0 - syp / kp->ty) * 0.5 * PH;
  double px = floor(fx), py = floor(fy);
  if (fx - px < OR_EPS * maxd(1.0, fabs(fx)) || px + 1.0 - fx < OR_EPS * maxd(1.0, fabs(fx))) *am = 1;
  if (fy - py < OR_EPS * maxd(1.0, fabs(fy)) || py + 1.0 - fy < OR_EPS * maxd(1.0, fabs(fy))) *am = 1;
  if (!(px >= 0 && px < PW && py >= 0 && py < PH)) return 0;
  *q = (size_t)py * PW + (size_t)px;
  return 1;
}

void or_recon(const double* cam, int W, int H, const double* z, const int* spp,
              const double* pcam /* NULL: no history */, const double* hist, const int* hvalid, const double* hz,
              const double* hit, const double* cn, const double* cf, const double* far_pos, const int* px_amb,
              double alpha, double* cn_out, double* cf_out, double* hist_out, int* hvalid_out, double* hz_out,
              int* amb) {
  cam_t k = mk_cam(cam, W, H), kp;
  if (pcam) kp = mk_cam(pcam, W, H);
  size_t N = (size_t)W * H;
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t p = (size_t)y * W + x;
      int am = 0;
      hz_out[p] = z[p];
      if (spp[p] <= 0) {
        for (int c = 0; c < 3; ++c) { cn_out[c * N + p] = cn[c * N + p]; cf_out[c * N + p] = cf[c * N + p]; }
        for (int c = 0; c < 8; ++c) hist_out[c * N + p] = 0.0;
        hvalid_out[p] = 0;
        if (amb) amb[p] = 0;
        continue;
      }
      double h = hit[p];
      if (px_amb && px_amb[p]) am = 1;
      /* near path */
      int okn = 0;
      size_t qn = 0;
      if (pcam) {
        double v[3], X[3], zc;
        pixel_dir(&k, x, y, v);
        for (int a = 0; a < 3; ++a) X[a] = k.e[a] + z[p] * v[a];
        if (reproj_px(&kp, W, H, X, &qn, &zc, &am) && hvalid[qn]) {
          double rel = fabs(hz[qn] - zc) / zc;
          if (fabs(rel - 0.01) < OR_EPS) am = 1;
          okn = rel <= 0.01;
        }
      }
      /* far path */
      int okf = 0;
      size_t qf = 0;
      if (pcam) {
        double Xf[3] = {0, 0, 0};
        int have = 0;
        if (far_pos[3 * N + p] > 0.0) {
          for (int a = 0; a < 3; ++a) Xf[a] = far_pos[a * N + p];
          have = 1;
        } else {
          int cnt = 0;
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              int xx = x + dx, yy = y + dy;
              if ((dx == 0 && dy == 0) || xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
              size_t o = (size_t)yy * W + xx;
              if (spp[o] > 0 && far_pos[3 * N + o] > 0.0) {
                for (int a = 0; a < 3; ++a) Xf[a] += far_pos[a * N + o];
                if (px_amb && px_amb[o]) am = 1;
                ++cnt;
              }
            }
          if (cnt > 0) { for (int a = 0; a < 3; ++a) Xf[a] /= cnt; have = 1; }
        }
        double zc;
        if (have && reproj_px(&kp, W, H, Xf, &qf, &zc, &am) && hvalid[qf]) okf = 1;
      }
      double Np[3], Fp[3], Hn, Hf;
      for (int c = 0; c < 3; ++c) {
        Np[c] = okn ? (1.0 - alpha) * hist[c * N + qn] + alpha * h * cn[c * N + p] : h * cn[c * N + p];
        Fp[c] = okf ? (1.0 - alpha) * hist[(4 + c) * N + qf] + alpha * (1.0 - h) * cf[c * N + p]
                    : (1.0 - h) * cf[c * N + p];
      }
      Hn = okn ? (1.0 - alpha) * hist[3 * N + qn] + alpha * h : h;
      Hf = okf ? (1.0 - alpha) * hist[7 * N + qf] + alpha * h : h;
      for (int c = 0; c < 3; ++c) {
        cn_out[c * N + p] = Hn > 0.0 ? Np[c] / Hn : cn[c * N + p];
        cf_out[c * N + p] = 1.0 - Hf > 0.0 ? Fp[c] / (1.0 - Hf) : cf[c * N + p];
        hist_out[c * N + p] = Np[c];
        hist_out[(4 + c) * N + p] = Fp[c];
      }
      hist_out[3 * N + p] = Hn;
      hist_out[7 * N + p] = Hf;
      hvalid_out[p] = 1;
      if (amb) amb[p] = am;
    }
}

/* ------------------------------------------------------------------------- */
/* Spatial reconstruction of the near and far ray-traced colours (our reading */
/* of the last paragraph of the paper's Reconstruction section: the near and */
/* far CoC sizes blended by the accumulated hit ratio set the radius and the */
/* sampling level of detail of a circular gather; neighbours whose CoC      */
/* radius is smaller than their distance are rejected as in the post-filter; */
/* a clamped variance estimate weights the gathered colour).                 */
/* Per traced pixel q (s_q = spp > 0), with H_q its accumulated hit ratio    */
/* (the latest one, h_q, without temporal history) and cbar the mean |CoC|  */
/* of its near / far rays:                                                   */
/*   r_q = min(r_cap, (H_q cbar_n(q) + (1 - H_q) cbar_f(q)) / 2).            */
/* Level L texel (i, j) = the traced pixels q of the block                  */
/*   [i 2^L, (i+1) 2^L) x [j 2^L, (j+1) 2^L), summed:                        */
/*   An = sum s h C_tn, Bn = sum s h, Af = sum s (1-h) C_tf, Bf = sum s (1-h),*/
/*   rho = sum r, kappa = count   (s h: the pixel's near-ray weight).       */
/* Traced pixel p at (x, y), N taps:                                         */
/*   L = floor(log2(r_p sqrt(pi / N))) clamped to [0, OR_SP_LMAX] (texels no */
/*   wider than the taps' mean spacing; L = 0 when r_p sqrt(pi/N) < 1);      */
/*   tap k: u_k = sqrt((k - 0.5)/N) (cos k g, sin k g), g = pi (3 - sqrt 5); */
/*   the pixel containing (x + 0.5, y + 0.5) + r_p u_k, clamped to the      */
/*   image, shifted right by L gives the texel; d_k = r_p |u_k|;             */
/*   a_k = clamp(rho / kappa - d_k + 0.5, 0, 1) (0 when kappa = 0).          */
/*   G_n = (s_p h_p C_tn(p) + sum_k a_k An_k) / (s_p h_p + sum_k a_k Bn_k),   */
/*   C_tn(p) when the denominator is 0; G_f alike with the far sums.         */
/*   lambda = clamp(V_p / v_clamp, 0, 1), 1 where V_p = +inf or no variance  */
/*   is given; C_tn' = C_tn + lambda (G_n - C_tn), C_tf' alike.             */
/* Untraced pixels are copied.                                               */
/* Ambiguity (amb, nullable, per pixel; 0 where untraced): the level and the */
/* tap pixels are integers decided by floating point.  Bit 1: the spacing   */
/* r_p sqrt(pi/N) lies within relative OR_EPS of a level boundary 2^m       */
/* (m = 1..OR_SP_LMAX).  Bit 2: a tap coordinate v = x + 0.5 + r_p u lies   */
/* within OR_EPS + 2^-20 (|x + 0.5| + |r_p u|) of an integer.  The band     */
/* grows with the operands because a single-precision evaluation of v      */
/* rounds at up to 2^-24 |v| (6e-5 px at v = 1000) on top of the roundings  */
/* of r_p and u; 2^-20 is sixteen such units.                              */
/* cond (nullable, 2 planes: near, far): the sensitivity of each output to  */
/* errors in the acceptances.  A tap whose argument rho/kappa - d + 0.5     */
/* lies within OR_SP_DA of the ramp [0, 1] (inside it, or near an end) can  */
/* move; one clear of it cannot.  cond = lambda (sum of the weights Bn_k of */
/* such taps) / (the accepted near weight s_p h_p + sum a_k Bn_k), far      */
/* alike; an error e in every such acceptance moves the output by at most   */
/* e cond max_k |An_k / Bn_k - G_n| (0 where untraced).                     */
/* ------------------------------------------------------------------------- */
#define OR_SP_LMAX 5
#define OR_SP_DA 1.0e-3

typedef struct {
  int W, H;
  const int* spp;
  const double *cn, *cf, *h, *hacc, *coc;
  double r_cap;
} sp_in_t;

static double sp_radius(const sp_in_t* I, size_t q) {
  double Hq = I->hacc ? I->hacc[q] : I->h[q];
  size_t N = (size_t)I->W * I->H;
  return mind(I->r_cap, 0.5 * (Hq * I->coc[q] + (1.0 - Hq) * I->coc[N + q]));
}

/* the sums of level-L texel (i, j): o[0..2] An, o[3] Bn, o[4..6] Af, o[7] Bf,
 * o[8] rho, o[9] kappa */
static void sp_texel(const sp_in_t* I, int L, int i, int j, double* o) {
  size_t N = (size_t)I->W * I->H;
  for (int a = 0; a < 10; ++a) o[a] = 0.0;
  int b = 1 << L;
  for (int y = j * b; y < (j + 1) * b && y < I->H; ++y)
    for (int x = i * b; x < (i + 1) * b && x < I->W; ++x) {
      size_t q = (size_t)y * I->W + x;
      if (I->spp[q] <= 0) continue;
      double s = I->spp[q], hq = I->h[q];
      for (int c = 0; c < 3; ++c) {
        o[c] += s * hq * I->cn[c * N + q];
        o[4 + c] += s * (1.0 - hq) * I->cf[c * N + q];
      }
      o[3] += s * hq;
      o[7] += s * (1.0 - hq);
      o[8] += sp_radius(I, q);
      o[9] += 1.0;
    }
}

void or_sp_level(int W, int H, const int* spp, const double* cn, const double* cf, const double* h,
                 const double* hacc, const double* coc, double r_cap, int L, double* out) {
  sp_in_t I = {W, H, spp, cn, cf, h, hacc, coc, r_cap};
  int WL = (W + (1 << L) - 1) >> L, HL = (H + (1 << L) - 1) >> L;
  size_t NL = (size_t)WL * HL;
#pragma omp parallel for
  for (int j = 0; j < HL; ++j)
    for (int i = 0; i < WL; ++i) {
      double o[10];
      sp_texel(&I, L, i, j, o);
      for (int a = 0; a < 10; ++a) out[a * NL + (size_t)j * WL + i] = o[a];
    }
}

/* v within band of an integer */
static int sp_near_int(double v, double band) {
  double f = floor(v);
  return v - f < band || f + 1.0 - v < band;
}

void or_spatial(int W, int H, const int* spp, const double* cn, const double* cf, const double* h,
                const double* hacc, const double* coc, const double* V, int n_taps, double r_cap,
                double v_clamp, double* cn_out, double* cf_out, int* amb, double* cond) {
  sp_in_t I = {W, H, spp, cn, cf, h, hacc, coc, r_cap};
  size_t N = (size_t)W * H;
  const double g = OR_PI * (3.0 - sqrt(5.0));
#pragma omp parallel for schedule(dynamic, 4)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t p = (size_t)y * W + x;
      int am = 0;
      for (int c = 0; c < 3; ++c) { cn_out[c * N + p] = cn[c * N + p]; cf_out[c * N + p] = cf[c * N + p]; }
      if (cond) cond[p] = cond[N + p] = 0.0;
      if (spp[p] <= 0) { if (amb) amb[p] = 0; continue; }
      double rp = sp_radius(&I, p);
      double spacing = rp * sqrt(OR_PI / n_taps);
      int L = 0;
      if (spacing >= 1.0) L = (int)floor(log2(spacing));
      if (L > OR_SP_LMAX) L = OR_SP_LMAX;
      for (int m = 1; m <= OR_SP_LMAX; ++m)
        if (fabs(spacing - (double)(1 << m)) < OR_EPS * (double)(1 << m)) am |= 1;
      double sn = spp[p] * h[p], sf = spp[p] * (1.0 - h[p]);
      double An[3], Af[3], Bn = sn, Bf = sf, Sn = 0.0, Sf = 0.0;
      for (int c = 0; c < 3; ++c) { An[c] = sn * cn[c * N + p]; Af[c] = sf * cf[c * N + p]; }
      for (int k = 1; k <= n_taps; ++k) {
        double rr = sqrt((k - 0.5) / n_taps);
        double ux = rr * cos(k * g), uy = rr * sin(k * g);
        double fx = x + 0.5 + rp * ux, fy = y + 0.5 + rp * uy;
        if (sp_near_int(fx, OR_EPS + ldexp(fabs(x + 0.5) + fabs(rp * ux), -20)) ||
            sp_near_int(fy, OR_EPS + ldexp(fabs(y + 0.5) + fabs(rp * uy), -20)))
          am |= 2;
        int px = clampi((int)floor(fx), 0, W - 1), py = clampi((int)floor(fy), 0, H - 1);
        double o[10];
        sp_texel(&I, L, px >> L, py >> L, o);
        if (o[9] <= 0.0) continue;
        double arg = o[8] / o[9] - rp * rr + 0.5;
        double a = clampd(arg, 0.0, 1.0);
        for (int c = 0; c < 3; ++c) { An[c] += a * o[c]; Af[c] += a * o[4 + c]; }
        Bn += a * o[3];
        Bf += a * o[7];
        if (arg > -OR_SP_DA && arg < 1.0 + OR_SP_DA) { Sn += o[3]; Sf += o[7]; }
      }
      double lam = 1.0;
      if (V && !isinf(V[p])) lam = clampd(V[p] / v_clamp, 0.0, 1.0);
      for (int c = 0; c < 3; ++c) {
        double Gn = Bn > 0.0 ? An[c] / Bn : cn[c * N + p];
        double Gf = Bf > 0.0 ? Af[c] / Bf : cf[c * N + p];
        cn_out[c * N + p] = cn[c * N + p] + lam * (Gn - cn[c * N + p]);
        cf_out[c * N + p] = cf[c * N + p] + lam * (Gf - cf[c * N + p]);
      }
      if (cond) {
        cond[p] = Bn > 0.0 ? lam * Sn / Bn : 0.0;
        cond[N + p] = Bf > 0.0 ? lam * Sf / Bf : 0.0;
      }
      if (amb) amb[p] = am;
    }
}

/* ------------------------------------------------------------------------- */
/* Post-process gather DoF filter (our reading of the paper's adapted         */
/* post-process plus its CoC-radius rejection rule).                         */
/*  c_p = signed CoC (px), r_p = |c_p| / 2.                                   */
/*  R(p) = min(R_cap, max of r over the tiles within ceil(R_cap / tile)      */
/*         tiles (Chebyshev) of p's tile).                                    */
/*  taps k = 1..N: u_k = sqrt((k - 0.5)/N) (cos k g, sin k g), g = pi(3-sqrt5)*/
/*  q_k = pixel centre + R u_k, d_k = R |u_k|; bilinear fetch of colour and  */
/*  signed CoC (texel centres at +0.5, clamp to edge).                        */
/*  background clamp t = clamp((c_q - c_p) / bg_ramp, 0, 1),                 */
/*  r_eff = r_q - t max(0, r_q - r_p), a = clamp(r_eff - d_k + 0.5, 0, 1),   */
/*  w_k = a (R^2 / N) / max(r_q, 0.5)^2, centre w_0 = 1 / max(r_p, 0.5)^2.   */
/*  C_pp = (w_0 C_p + sum w_k C_q) / (w_0 + sum w_k).                        */
/*  Aperture B-gon (B >= 3): u_k is moved radially onto the polygon,        */
/*  u_k' = u_k P(angle of u_k), P the polygon's boundary radius, so the tap */
/*  keeps the gauge distance |u_k| of the polygonal CoC (d_k unchanged);   */
/*  spherical aberration multiplies w_k by the weight of radius |u_k'|.     */
/*  The sampling kernel so takes the aperture's silhouette and weighting    */
/*  (our reading of the paper's future work).                               */
/* pp[4] = n_taps, tile, r_cap, bg_ramp_px.  Out for listed pixels.           */
/* ------------------------------------------------------------------------- */
static void bilerp(const double* img, int W, int H, double fx, double fy, double* o, int nch, size_t plane) {
  double gx = fx - 0.5, gy = fy - 0.5;
  double x0f = floor(gx), y0f = floor(gy);
  double ax = gx - x0f, ay = gy - y0f;
  int x0 = (int)x0f, y0 = (int)y0f;
  int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
  int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
  for (int c = 0; c < nch; ++c) {
    const double* b = img + (size_t)c * plane;
    double v00 = b[(size_t)ya * W + xa], v10 = b[(size_t)ya * W + xb];
    double v01 = b[(size_t)yb * W + xa], v11 = b[(size_t)yb * W + xb];
    o[c] = (1 - ay) * ((1 - ax) * v00 + ax * v10) + ay * ((1 - ax) * v01 + ax * v11);
  }
}

void or_pp_radius(int W, int H, const double* cimg, double r_cap, int tile, double* Rout) {
  int TW = (W + tile - 1) / tile, TH = (H + tile - 1) / tile;
  double* rt = (double*)calloc((size_t)TW * TH, sizeof(double));
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      double r = 0.5 * fabs(cimg[(size_t)y * W + x]);
      size_t t = (size_t)(y / tile) * TW + x / tile;
      if (r > rt[t]) rt[t] = r;
    }
  int K = (int)ceil(r_cap / tile);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int tx = x / tile, ty = y / tile;
      double m = 0.0;
      for (int dy = -K; dy <= K; ++dy)
        for (int dx = -K; dx <= K; ++dx) {
          int yy = ty + dy, xx = tx + dx;
          if (yy < 0 || yy >= TH || xx < 0 || xx >= TW) continue;
          m = maxd(m, rt[(size_t)yy * TW + xx]);
        }
      Rout[(size_t)y * W + x] = mind(r_cap, m);
    }
  free(rt);
}

void or_postfilter(const double* cam, int W, int H, const double* lens, const double* color, const double* z,
                   const double* pp, const int64_t* pix, int64_t n, double* out) {
  cam_t k = mk_cam(cam, W, H);
  size_t N = (size_t)W * H;
  int NT = (int)pp[0], tile = (int)pp[1];
  double r_cap = pp[2], ramp = pp[3];
  double* img = (double*)malloc(sizeof(double) * 4 * N); /* rgb + signed CoC */
  double* R = (double*)malloc(sizeof(double) * N);
  for (size_t p = 0; p < N; ++p) {
    for (int c = 0; c < 3; ++c) img[(size_t)c * N + p] = color[(size_t)c * N + p];
    img[3 * N + p] = coc_px(&k, lens, z[p]);
  }
  or_pp_radius(W, H, img + 3 * N, r_cap, tile, R);
  double g = OR_PI * (3.0 - sqrt(5.0));
  int B = (int)lens[3];
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = pix ? pix[i] : i;
    int x = (int)(p % W), y = (int)(p / W);
    double cp = img[3 * N + p], rp = 0.5 * fabs(cp);
    double Rp = R[p];
    double w0 = 1.0 / (maxd(rp, 0.5) * maxd(rp, 0.5));
    double acc[3], wsum = w0;
    for (int c = 0; c < 3; ++c) acc[c] = w0 * img[(size_t)c * N + p];
    for (int kk = 1; kk <= NT; ++kk) {
      double rad = sqrt((kk - 0.5) / NT);
      /* aperture B-gon: the tap moved radially onto the polygon (its gauge */
      /* distance stays rad); aberration weight of its radius               */
      double sc = B >= 3 ? poly_radius(B, lens[4], kk * g) : 1.0;
      double ux = rad * sc * cos(kk * g), uy = rad * sc * sin(kk * g);
      double om = sa_weight(lens[5], rad * sc);
      double qx = x + 0.5 + Rp * ux, qy = y + 0.5 + Rp * uy;
      double smp[4];
      bilerp(img, W, H, qx, qy, smp, 4, N);
      double dk = Rp * rad;
      double cq = smp[3], rq = 0.5 * fabs(cq);
      double t = clampd((cq - cp) / ramp, 0.0, 1.0);
      double reff = rq - t * maxd(0.0, rq - rp);
      double a = clampd(reff - dk + 0.5, 0.0, 1.0);
      double w = om * a * (Rp * Rp / NT) / (maxd(rq, 0.5) * maxd(rq, 0.5));
      for (int c = 0; c < 3; ++c) acc[c] += w * smp[c];
      wsum += w;
    }
    for (int c = 0; c < 3; ++c) out[(size_t)c * n + i] = acc[c] / wsum;
  }
  free(img); free(R);
}

/* ------------------------------------------------------------------------- */
/* Composite (paper's Composite section; our readings of its thresholds).     */
/*  phi = clamp(|c_p| - sqrt 2, 0, 1): out-of-focus weight (focus zone is    */
/*        |c| < sqrt 2 with a 1-px ramp above it);                            */
/*  nu  = clamp(0.5 - c_p / (2 sqrt 2), 0, 1): near (1) / far (0);            */
/*  C_rt = h C_tn + (1 - h) C_tf;                                             */
/*  rho = [s > 0] (1 - spec), spec = 0 for Lambertian scenes;                 */
/*  beta = [s > 0] clamp(1 - h / h_t, 0, 1);                                  */
/*  C_oof = nu (rho C_rt + (1 - rho) C_pp) + (1 - nu)(beta C_rt + (1-beta)C_pp)*/
/*  out = (1 - phi) C_r + phi C_oof;  rt_override: out = C_rt where s > 0.   */
/* ------------------------------------------------------------------------- */
void or_composite(const double* cam, int W, int H, const double* lens,
                  const double* color, const double* cpp, const double* z, const int* spp,
                  const double* c_near, const double* c_far, const double* hit,
                  double h_t, int rt_override, const double* pp_spec, double spec_y, double* out) {
  cam_t k = mk_cam(cam, W, H);
  size_t N = (size_t)W * H;
  for (size_t p = 0; p < N; ++p) {
    double c = coc_px(&k, lens, z[p]);
    double phi = clampd(fabs(c) - OR_SQRT2, 0.0, 1.0);
    double nu = clampd(0.5 - c / (2.0 * OR_SQRT2), 0.0, 1.0);
    double h = hit[p];
    int traced = spp[p] > 0;
    double rho = traced ? 1.0 : 0.0;
    double beta = traced ? clampd(1.0 - h / h_t, 0.0, 1.0) : 0.0;
    /* specular bokeh: near and traced, the post-process colour is favoured */
    /* by sigma = clamp(Y_s,pp / spec_y, 0, 1), Y_s,pp the post-filtered   */
    /* specular luminance                                                  */
    double sig = (pp_spec && spec_y > 0.0) ? clampd(pp_spec[p] / spec_y, 0.0, 1.0) : 0.0;
    for (int q = 0; q < 3; ++q) {
      double crt = h * c_near[(size_t)q * N + p] + (1.0 - h) * c_far[(size_t)q * N + p];
      double cp = cpp[(size_t)q * N + p];
      double cnear = crt + sig * (cp - crt);
      double oof = nu * (rho * cnear + (1.0 - rho) * cp) + (1.0 - nu) * (beta * crt + (1.0 - beta) * cp);
      double o = (1.0 - phi) * color[(size_t)q * N + p] + phi * oof;
      if (rt_override && traced) o = crt;
      out[(size_t)q * N + p] = o;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Adjoint of post-filter + composite (the differentiable form).              */
/* out(C_r, S1, A) with depth, counts and ray-trace colours held fixed.       */
/* Given g = dL/dout, returns dL/dC_r (reverse mode: the gather's transpose,  */
/* a scatter through the bilinear weights) and dL/dS1, dL/dA (forward mode    */
/* through the recomputed gather: dc/dS1 = -A s_px / S1^2,                    */
/* dc/dA = (1/S1 - 1/z) s_px).  The gather radius follows the CoC of its      */
/* tile-max pixel (lowest index on ties) unless capped; clamp ramps take      */
/* subgradient 0 at their kinks.                                              */
/* ------------------------------------------------------------------------- */
typedef struct { double v, ds, da; } dual;  /* value and its S1 / A derivatives */

static inline dual dmk(double v, double ds, double da) { dual r = {v, ds, da}; return r; }
static inline dual dadd(dual a, dual b) { return dmk(a.v + b.v, a.ds + b.ds, a.da + b.da); }
static inline dual dsub(dual a, dual b) { return dmk(a.v - b.v, a.ds - b.ds, a.da - b.da); }
static inline dual dmul(dual a, dual b) { return dmk(a.v * b.v, a.ds * b.v + a.v * b.ds, a.da * b.v + a.v * b.da); }
static inline dual dscale(dual a, double s) { return dmk(a.v * s, a.ds * s, a.da * s); }
static inline dual ddiv(dual a, dual b) {
  double q = a.v / b.v;
  return dmk(q, (a.ds - q * b.ds) / b.v, (a.da - q * b.da) / b.v);
}
static inline dual dconst(double v) { return dmk(v, 0.0, 0.0); }
/* clamp with subgradient 0 outside (lo, hi) */
static inline dual dclamp(dual x, double lo, double hi) {
  if (x.v <= lo) return dconst(lo);
  if (x.v >= hi) return dconst(hi);
  return x;
}
static inline dual dmax0(dual x) { return x.v > 0.0 ? x : dconst(0.0); }
static inline dual dmaxc(dual x, double c) { return x.v > c ? x : dconst(c); }
static inline dual dabs(dual x) { return x.v >= 0.0 ? x : dscale(x, -1.0); }

/* bilinear sample of (rgb, c) and its x/y derivatives at continuous q */
static void bilerp_grad(const double* img, int W, int H, size_t N, double qx, double qy,
                        double* s, double* sx, double* sy, int* tx, int* ty, double* tw) {
  double gx = qx - 0.5, gy = qy - 0.5;
  double x0f = floor(gx), y0f = floor(gy);
  double ax = gx - x0f, ay = gy - y0f;
  int x0 = (int)x0f, y0 = (int)y0f;
  int xa = clampi(x0, 0, W - 1), xb = clampi(x0 + 1, 0, W - 1);
  int ya = clampi(y0, 0, H - 1), yb = clampi(y0 + 1, 0, H - 1);
  for (int c = 0; c < 4; ++c) {
    const double* b = img + (size_t)c * N;
    double v00 = b[(size_t)ya * W + xa], v10 = b[(size_t)ya * W + xb];
    double v01 = b[(size_t)yb * W + xa], v11 = b[(size_t)yb * W + xb];
    s[c] = (1 - ay) * ((1 - ax) * v00 + ax * v10) + ay * ((1 - ax) * v01 + ax * v11);
    sx[c] = (1 - ay) * (v10 - v00) + ay * (v11 - v01);
    sy[c] = (1 - ax) * (v01 - v00) + ax * (v11 - v10);
  }
  tx[0] = xa; ty[0] = ya; tw[0] = (1 - ax) * (1 - ay);
  tx[1] = xb; ty[1] = ya; tw[1] = ax * (1 - ay);
  tx[2] = xa; ty[2] = yb; tw[2] = (1 - ax) * ay;
  tx[3] = xb; ty[3] = yb; tw[3] = ax * ay;
}

/* gather radius per pixel and the pixel whose CoC sets it (-1 when capped
 * or zero): tile max of r (lowest index on ties), then max over the tiles
 * within ceil(r_cap / tile) (largest value, lowest pixel index on ties). */
void or_pp_radius_arg(int W, int H, const double* cimg, double r_cap, int tile, double* Rout, int64_t* arg) {
  int TW = (W + tile - 1) / tile, TH = (H + tile - 1) / tile;
  double* rt = (double*)calloc((size_t)TW * TH, sizeof(double));
  int64_t* ra = (int64_t*)malloc(sizeof(int64_t) * (size_t)TW * TH);
  for (size_t t = 0; t < (size_t)TW * TH; ++t) ra[t] = -1;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t p = (size_t)y * W + x, t = (size_t)(y / tile) * TW + x / tile;
      double r = 0.5 * fabs(cimg[p]);
      if (ra[t] < 0 || r > rt[t] || (r == rt[t] && (int64_t)p < ra[t])) { rt[t] = r; ra[t] = (int64_t)p; }
    }
  int K = (int)ceil(r_cap / tile);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int tx = x / tile, ty = y / tile;
      double m = -1.0;
      int64_t am = -1;
      for (int dy = -K; dy <= K; ++dy)
        for (int dx = -K; dx <= K; ++dx) {
          int yy = ty + dy, xx = tx + dx;
          if (yy < 0 || yy >= TH || xx < 0 || xx >= TW) continue;
          size_t t = (size_t)yy * TW + xx;
          if (rt[t] > m || (rt[t] == m && ra[t] < am)) { m = rt[t]; am = ra[t]; }
        }
      size_t p = (size_t)y * W + x;
      Rout[p] = mind(r_cap, m);
      arg[p] = (m < r_cap && m > 0.0) ? am : -1;
    }
  free(rt); free(ra);
}

void or_pp_composite_backward(const double* cam, int W, int H, const double* lens, const double* color,
                              const double* z, const int* spp, const double* c_near, const double* c_far,
                              const double* hit, const double* pp, double h_t, int rt_override,
                              const double* g, double* gcolor, double* glens /* dS1, dA */) {
  cam_t k = mk_cam(cam, W, H);
  size_t N = (size_t)W * H;
  int NT = (int)pp[0], tile = (int)pp[1];
  double r_cap = pp[2], ramp = pp[3];
  double A = lens[1], S1 = lens[2];
  double* img = (double*)malloc(sizeof(double) * 4 * N);
  double* R = (double*)malloc(sizeof(double) * N);
  int64_t* arg = (int64_t*)malloc(sizeof(int64_t) * N);
  /* dc/dS1 (same for every pixel) and dc/dA per pixel */
  double dcs = -A * k.spx / (S1 * S1);
  double* dca = (double*)malloc(sizeof(double) * N);
  for (size_t p = 0; p < N; ++p) {
    for (int c = 0; c < 3; ++c) img[(size_t)c * N + p] = color[(size_t)c * N + p];
    img[3 * N + p] = coc_px(&k, lens, z[p]);
    dca[p] = (1.0 / S1 - 1.0 / z[p]) * k.spx;
  }
  or_pp_radius_arg(W, H, img + 3 * N, r_cap, tile, R, arg);
  memset(gcolor, 0, sizeof(double) * 3 * N);
  double gs = 0.0, ga = 0.0;
  double gam = OR_PI * (3.0 - sqrt(5.0));
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t p = (size_t)y * W + x;
      dual cp = dmk(img[3 * N + p], dcs, dca[p]);
      /* composite weights */
      dual phi = dclamp(dsub(dabs(cp), dconst(OR_SQRT2)), 0.0, 1.0);
      dual nu = dclamp(dsub(dconst(0.5), dscale(cp, 1.0 / (2.0 * OR_SQRT2))), 0.0, 1.0);
      double h = hit[p];
      int traced = spp[p] > 0;
      double rho = traced ? 1.0 : 0.0;
      double beta = traced ? clampd(1.0 - h / h_t, 0.0, 1.0) : 0.0;
      /* coefficients of C_rt and C_pp in the out-of-focus colour */
      dual acoef = dadd(dscale(nu, rho), dscale(dsub(dconst(1.0), nu), beta));
      dual bcoef = dadd(dscale(nu, 1.0 - rho), dscale(dsub(dconst(1.0), nu), 1.0 - beta));
      double gq[3];
      for (int c = 0; c < 3; ++c) gq[c] = g[(size_t)c * N + p];
      if (rt_override && traced) continue;  /* out = C_rt: independent of C_r, S1, A */
      /* forward-mode post-filter at p */
      dual rp = dscale(dabs(cp), 0.5);
      dual rp5 = dmaxc(rp, 0.5);
      dual w0 = ddiv(dconst(1.0), dmul(rp5, rp5));
      dual Rd = dconst(R[p]);
      if (arg[p] >= 0) {
        double cm = img[3 * N + arg[p]];
        double sg = cm >= 0.0 ? 0.5 : -0.5;
        Rd = dmk(R[p], sg * dcs, sg * dca[arg[p]]);
      }
      dual num[3], den = w0;
      for (int c = 0; c < 3; ++c) num[c] = dscale(w0, img[(size_t)c * N + p]);
      /* per-tap weights kept for the colour scatter */
      double wk_v[256];
      int tx[256][4], ty[256][4];
      double tw[256][4];
      for (int kk = 1; kk <= NT && Rd.v > 0.0; ++kk) {
        double rad = sqrt((kk - 0.5) / NT);
        double ux = rad * cos(kk * gam), uy = rad * sin(kk * gam);
        double qx = x + 0.5 + Rd.v * ux, qy = y + 0.5 + Rd.v * uy;
        double s[4], sx[4], sy[4];
        bilerp_grad(img, W, H, N, qx, qy, s, sx, sy, tx[kk - 1], ty[kk - 1], tw[kk - 1]);
        /* d(sample)/dtheta: position moves with R, c also changes in place */
        double dsp_s = ux * Rd.ds, dsp_a = ux * Rd.da, dsq_s = uy * Rd.ds, dsq_a = uy * Rd.da;
        dual smp[3];
        for (int c = 0; c < 3; ++c) smp[c] = dmk(s[c], sx[c] * dsp_s + sy[c] * dsq_s, sx[c] * dsp_a + sy[c] * dsq_a);
        /* bilinear of dc/dA: interpolate dca with the same weights */
        double dca_q = 0.0;
        for (int i = 0; i < 4; ++i) dca_q += tw[kk - 1][i] * dca[(size_t)ty[kk - 1][i] * W + tx[kk - 1][i]];
        dual cq = dmk(s[3], dcs + sx[3] * dsp_s + sy[3] * dsq_s, dca_q + sx[3] * dsp_a + sy[3] * dsq_a);
        dual rq = dscale(dabs(cq), 0.5);
        dual tk = dclamp(dscale(dsub(cq, cp), 1.0 / ramp), 0.0, 1.0);
        dual reff = dsub(rq, dmul(tk, dmax0(dsub(rq, rp))));
        dual dk = dscale(Rd, rad);
        dual a = dclamp(dadd(dsub(reff, dk), dconst(0.5)), 0.0, 1.0);
        dual rq5 = dmaxc(rq, 0.5);
        dual w = ddiv(dmul(a, dscale(dmul(Rd, Rd), 1.0 / NT)), dmul(rq5, rq5));
        for (int c = 0; c < 3; ++c) num[c] = dadd(num[c], dmul(w, smp[c]));
        den = dadd(den, w);
        wk_v[kk - 1] = w.v;
      }
      int ntaps = Rd.v > 0.0 ? NT : 0;
      double crt[3];
      for (int c = 0; c < 3; ++c) crt[c] = h * c_near[(size_t)c * N + p] + (1.0 - h) * c_far[(size_t)c * N + p];
      for (int c = 0; c < 3; ++c) {
        dual cpp = ddiv(num[c], den);
        double cr = img[(size_t)c * N + p];
        /* out = (1 - phi) C_r + phi (a C_rt + b C_pp) */
        dual oof = dadd(dscale(acoef, crt[c]), dmul(bcoef, cpp));
        dual out = dadd(dscale(dsub(dconst(1.0), phi), cr), dmul(phi, oof));
        gs += gq[c] * out.ds;
        ga += gq[c] * out.da;
        /* colour: direct term, then the post-filter's transpose */
        gcolor[(size_t)c * N + p] += gq[c] * (1.0 - phi.v);
        double gpp = gq[c] * phi.v * bcoef.v / den.v;
        gcolor[(size_t)c * N + p] += gpp * w0.v;
        for (int kk = 0; kk < ntaps; ++kk)
          for (int i = 0; i < 4; ++i)
            gcolor[(size_t)c * N + (size_t)ty[kk][i] * W + tx[kk][i]] += gpp * wk_v[kk] * tw[kk][i];
      }
    }
  glens[0] = gs;
  glens[1] = ga;
  free(img); free(R); free(arg); free(dca);
}
