// geom.hpp -- exact lattice geometry of the voxelizer: grid snap, candidate ranges, the
// closed-box touch tests and the clipped measures.  Pure functions usable on device and host
// (the host side serves unit checks of the predicates).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vx.h"

#define VX_HD __host__ __device__

namespace vx {

struct Lat {
  double bmin[3];
  double inv;        // lattice units per world unit, 2^23 / extent
  int64_t s;         // lattice units per voxel, 2^(23 - log2R)
  int32_t Sb;        // log2(s)
  int32_t R;
  int64_t rho;       // capsule radius in lattice units (fibers)
};

// The lattice figures the touch tests and weights need, selected by value: choosing between
// a kernel argument and a table entry by address would put the argument in scratch memory.
struct LatQ {
  int64_t s;
  int64_t rho;
  int32_t Sb;
};
VX_HD inline LatQ lat_q(const Lat* lats, int32_t patch, const Lat& L) {
  if (lats) {
    const Lat& P = lats[patch];
    return LatQ{P.s, P.rho, P.Sb};
  }
  return LatQ{L.s, L.rho, L.Sb};
}

// per-primitive record, 16 x int32: [0..8] snapped vertices (fibers: A, B, unused),
// [9..11] first candidate voxel, [12..14] candidate extent per axis
constexpr int kRec = 16;

VX_HD inline int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
VX_HD inline int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }
VX_HD inline int64_t floor_shift(int64_t a, int Sb) { return a >> Sb; }
// 1 / x to a few ulp: the hardware estimate refined by two Newton steps on the device
VX_HD inline double rcp_fast(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
#else
  return 1.0 / x;
#endif
}
VX_HD inline int64_t ceil_shift(int64_t a, int Sb) { return -((-a) >> Sb); }

// Sec. 3.1: P_volume = (P - bmin) / extent * R, on the lattice; false for non-finite or
// out-of-range input.  The subtract and multiply are not fused, as in the definition.
VX_HD inline bool snap_point(const float* p, const Lat& L, int32_t q[3]) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double g;
    {
#pragma clang fp contract(off)
      g = (double(p[a]) - L.bmin[a]) * L.inv;
    }
    const double r = rint(g);
    const bool good = (r >= -8388608.0) && (r <= 16777216.0);   // NaN compares false
    ok = ok && good;
    q[a] = good ? int32_t(r) : 0;
  }
  return ok;
}

VX_HD inline int64_t candidate_range(int64_t mn, int64_t mx, const Lat& L, int32_t& vlo) {
  int64_t lo = ceil_shift(mn, L.Sb) - 1;
  int64_t hi = floor_shift(mx, L.Sb);
  lo = lo < 0 ? 0 : lo;
  hi = hi > L.R - 1 ? L.R - 1 : hi;
  vlo = int32_t(lo);
  return hi >= lo ? hi - lo + 1 : 0;
}


// ---------------------------------------------------------------------------------------------
// candidate -> (primitive, voxel)
// ---------------------------------------------------------------------------------------------
// Primitive records: 16 x int32, [0..8] snapped vertices (fibers: A, B, zeros), [9..11] first
// candidate voxel, [12..14] candidate extent per axis.  Returns the number of candidates (0
// when the input is invalid, with ok = false).  dir: unit normal and twice the area (voxel^2)
// for triangles, unit tangent and length (voxel) for segments.
VX_HD inline int64_t prep_triangle(const float* t9, const Lat& L, int32_t* r, float4* dir, bool& ok) {
  int32_t q[9];
  ok = true;
  for (int v = 0; v < 3; ++v) ok = snap_point(t9 + v * 3, L, q + 3 * v) && ok;
  int64_t cnt = 1;
  for (int a = 0; a < 3; ++a) {
    const int64_t mn = imin(q[a], imin(q[3 + a], q[6 + a]));
    const int64_t mx = imax(q[a], imax(q[3 + a], q[6 + a]));
    int32_t vlo;
    const int64_t na = candidate_range(mn, mx, L, vlo);
    r[9 + a] = vlo;
    r[12 + a] = int32_t(na);
    cnt *= na;
  }
  for (int k = 0; k < 9; ++k) r[k] = q[k];
  r[15] = 0;
  int64_t e0[3], e1[3];
  for (int a = 0; a < 3; ++a) { e0[a] = int64_t(q[3 + a]) - q[a]; e1[a] = int64_t(q[6 + a]) - q[a]; }
  const double nx = double(e0[1] * e1[2] - e0[2] * e1[1]);
  const double ny = double(e0[2] * e1[0] - e0[0] * e1[2]);
  const double nz = double(e0[0] * e1[1] - e0[1] * e1[0]);
  const double len = sqrt(nx * nx + ny * ny + nz * nz);
  const double inv = len > 0 ? 1.0 / len : 0.0;
  const double s2 = double(L.s) * double(L.s);
  *dir = make_float4(float(nx * inv), float(ny * inv), float(nz * inv), float(len / s2));
  return ok ? cnt : 0;
}

// b == nullptr: point a ends its fiber and starts no segment (it is still validated)
VX_HD inline int64_t prep_segment(const float* a, const float* b, const Lat& L, int32_t* r, float4* dir, bool& ok) {
  int32_t A[3], B[3] = {0, 0, 0};
  ok = snap_point(a, L, A);
  if (b) ok = snap_point(b, L, B) && ok;
  int64_t cnt = b ? 1 : 0;
  for (int k = 0; k < 3; ++k) {
    const int64_t mn = imin(A[k], B[k]) - L.rho;
    const int64_t mx = imax(A[k], B[k]) + L.rho;
    int32_t vlo;
    const int64_t na = candidate_range(mn, mx, L, vlo);
    r[k] = A[k];
    r[3 + k] = B[k];
    r[6 + k] = 0;
    r[9 + k] = vlo;
    r[12 + k] = int32_t(na);
    cnt *= na;
  }
  r[15] = 0;
  const double d0 = double(B[0] - A[0]), d1 = double(B[1] - A[1]), d2 = double(B[2] - A[2]);
  const double len = b ? sqrt(d0 * d0 + d1 * d1 + d2 * d2) : 0.0;
  const double inv = len > 0 ? 1.0 / len : 0.0;
  *dir = make_float4(float(d0 * inv), float(d1 * inv), float(d2 * inv), float(len / double(L.s)));
  return ok ? cnt : 0;
}

// last p in [lo, n_prims) with cand_off[p] <= c, given cand_off[lo] <= c: galloping search from
// lo (a run of 64 candidates spans few primitives), then bisection
VX_HD inline int64_t find_prim(const int64_t* __restrict__ cand_off, int64_t lo, int64_t n_prims, int64_t c) {
  int64_t step = 1, hi = lo + 1;
  while (hi < n_prims && cand_off[hi] <= c) {
    lo = hi;
    step <<= 1;
    hi = lo + step;
  }
  if (hi > n_prims) hi = n_prims;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (cand_off[mid] <= c) lo = mid; else hi = mid;
  }
  return lo;
}

// last p in [0, n_prims) with cand_off[p] <= c, by bisection (cand_off[0] = 0 <= c)
VX_HD inline int64_t find_prim_bisect(const int64_t* __restrict__ cand_off, int64_t n_prims, int64_t c) {
  int64_t lo = 0, hi = n_prims;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (cand_off[mid] <= c) lo = mid; else hi = mid;
  }
  return lo;
}

VX_HD inline void candidate_voxel(const int32_t* r, int64_t li, int64_t v[3]) {
  const int64_t nx = r[12], ny = r[13];
  int64_t ix, iy, iz;
  if (li < 0x7fffffff && nx * ny < 0x7fffffff) {
    uint32_t l = uint32_t(li), x = uint32_t(nx), y = uint32_t(ny);
    uint32_t t = l / x;
    ix = l - t * x;
    iz = t / y;
    iy = t - uint32_t(iz) * y;
  } else {
    int64_t t = li / nx;
    ix = li - t * nx;
    iz = t / ny;
    iy = t - iz * ny;
  }
  v[0] = r[9] + ix;
  v[1] = r[10] + iy;
  v[2] = r[11] + iz;
}

// ---------------------------------------------------------------------------------------------
// exact triangle / closed box test (the box-axis tests hold by construction of the candidate
// range): the triangle's plane and the nine edge x axis directions.
// ---------------------------------------------------------------------------------------------
// The rare exact paths are out of line and take their operands by value: an array argument
// would make every caller keep its copy in scratch memory, whether the path runs or not.
VX_HD inline __attribute__((noinline)) bool plane_exact(int64_t n0, int64_t n1, int64_t n2, int64_t r0, int64_t r1,
                                                        int64_t r2, int64_t s) {
  const int64_t n[3] = {n0, n1, n2}, rel[3] = {r0, r1, r2};
  __int128 base = 0, lo = 0, hi = 0;
  for (int a = 0; a < 3; ++a) {
    base += (__int128)n[a] * rel[a];
    if (n[a] > 0) hi += (__int128)n[a] * s; else lo += (__int128)n[a] * s;
  }
  return !(base + lo > 0 || base + hi < 0);
}

// Every quantity of the edge tests is an integer below 2^53 in magnitude, so FP64 evaluates them
// exactly (and with none of the 64-bit integer multiplies, which take several quarter-rate
// instructions each on gfx950): vertex offsets from the box corner c lie in (-2^24, 2^24], edges
// e in [-2^25, 2^25], the projections a . c on an edge-cross-axis direction (two products) in
// [-2^50, 2^50], the box's projection bounds in [-2^48, 2^48], and the plane normal's
// components (differences of two products of edges) in [-2^51, 2^51].
VX_HD inline bool tri_touch(const int32_t* q, const int64_t v[3], int64_t s, int Sb) {
  double c[3][3];   // vertices relative to the box corner
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) c[i][a] = double(q[3 * i + a] - (int32_t(v[a]) << Sb));
  double e[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    e[0][a] = c[1][a] - c[0][a];
    e[1][a] = c[2][a] - c[1][a];
    e[2][a] = c[0][a] - c[2][a];
  }
  const double ds = double(s);
  // nine edge x box-axis directions: projections of the triangle and of the box [0, s]^3.  On
  // the direction of edge j the edge's two ends project alike, so the triangle projects onto
  // the interval between vertex j and the opposite vertex.  (Most candidates pass all nine:
  // the separations are gathered and decided once, without a branch per direction.)
  bool sep = false;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int u = (k + 1) % 3, w = (k + 2) % 3;     // axis = e_k x e_j -> components on u and w
      const double au = -e[j][w], aw = e[j][u];
      const double p0 = fma(au, c[j][u], aw * c[j][w]);
      const double p2 = fma(au, c[(j + 2) % 3][u], aw * c[(j + 2) % 3][w]);
      const double pmin = fmin(p0, p2), pmax = fmax(p0, p2);
      const double blo = (fmin(au, 0.0) + fmin(aw, 0.0)) * ds;
      const double bhi = (fmax(au, 0.0) + fmax(aw, 0.0)) * ds;
      sep = sep | (pmax < blo) | (pmin > bhi);
    }
  }
  if (sep) return false;
  // plane: corner offsets n . (corner - c0) must not all share a strict sign
  double n[3];
  n[0] = fma(e[0][2], e[2][1], -(e[0][1] * e[2][2]));
  n[1] = fma(e[0][0], e[2][2], -(e[0][2] * e[2][0]));
  n[2] = fma(e[0][1], e[2][0], -(e[0][0] * e[2][1]));
  double base = -(n[0] * c[0][0] + n[1] * c[0][1] + n[2] * c[0][2]);
  double lo = base, hi = base, mag = fabs(n[0] * c[0][0]) + fabs(n[1] * c[0][1]) + fabs(n[2] * c[0][2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double t = n[a] * ds;
    if (n[a] > 0) hi += t; else lo += t;
    mag += fabs(t);
  }
  const double err = mag * 0x1p-48;
  if (lo > err || hi < -err) return false;           // strictly on one side
  if (lo < -err && hi > err) return true;            // strictly across
  return plane_exact(int64_t(n[0]), int64_t(n[1]), int64_t(n[2]), -int64_t(c[0][0]), -int64_t(c[0][1]),
                     -int64_t(c[0][2]), s);
}

// ---------------------------------------------------------------------------------------------
// capsules: is the centreline within rho of the closed box?
// ---------------------------------------------------------------------------------------------
VX_HD inline double fdist2(double t, const double c[3], const double d[3], double s) {
  double f = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double x = fma(t, d[a], c[a]);
    double g = x < 0 ? -x : (x > s ? x - s : 0.0);
    f = fma(g, g, f);
  }
  return f;
}

// exact: f is evaluated at 0, 1, every breakpoint, and at the stationary point of the quadratic
// of every (axis state) combination whose region contains it.
VX_HD inline __attribute__((noinline)) bool cap_exact(int64_t c0, int64_t c1, int64_t c2, int64_t d0, int64_t d1,
                                                      int64_t d2, int64_t s, int64_t rho) {
  const int64_t c[3] = {c0, c1, c2}, d[3] = {d0, d1, d2};
  typedef __int128 I;
  const I r2 = (I)rho * rho;
  // f(num / den) * den^2 <= rho^2 den^2 at den > 0
  auto eval = [&](I num, I den) -> bool {
    I sum = 0;
    for (int a = 0; a < 3; ++a) {
      I g = (I)c[a] * den + num * d[a];
      I sd = (I)s * den;
      I dist = g < 0 ? -g : (g > sd ? g - sd : (I)0);
      sum += dist * dist;
    }
    return sum <= r2 * den * den;
  };
  if (eval(0, 1) || eval(1, 1)) return true;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0) continue;
    for (int side = 0; side < 2; ++side) {
      I num = (I)((side ? s : 0) - c[a]), den = d[a];
      if (den < 0) { num = -num; den = -den; }
      if (num >= 0 && num <= den && eval(num, den)) return true;
    }
  }
  for (int combo = 1; combo < 27; ++combo) {
    int st[3] = {combo % 3, (combo / 3) % 3, combo / 9};   // 0 inside, 1 below 0, 2 above s
    I Q = 0, P = 0;
    int64_t e[3];
    for (int a = 0; a < 3; ++a) {
      e[a] = st[a] == 1 ? c[a] : (st[a] == 2 ? c[a] - s : 0);
      if (st[a]) { Q += (I)d[a] * d[a]; P -= (I)e[a] * d[a]; }
    }
    if (Q == 0) continue;
    if (P < 0 || P > Q) continue;                             // t* outside [0, 1]
    bool member = true;
    for (int a = 0; a < 3; ++a) {
      I g = (I)c[a] * Q + P * d[a];
      I sq = (I)s * Q;
      if (st[a] == 1) member = member && g <= 0;
      else if (st[a] == 2) member = member && g >= sq;
      else member = member && g >= 0 && g <= sq;
    }
    if (!member) continue;
    I num = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = a + 1; b < 3; ++b) {
        if (!st[a] || !st[b]) continue;
        I x = (I)e[a] * d[b] - (I)e[b] * d[a];
        num += x * x;
      }
    if (num <= r2 * Q) return true;
  }
  return false;
}

// exact capsule / closed box test: min over t in [0,1] of f(t) = dist^2(c + t d, [0, s]^3)
// against rho^2.  FP64 with an error bound (all inputs are exact integers below 2^26; every
// rounding of the bracketing, the interpolation and the evaluation stays far inside
// M^2 2^-44); exact 128-bit integers when too close to call.
struct CapIn {
  int64_t ci[3], di[3];
  double c[3], d[3];
  double err;
};

// Lattice coordinates lie within [-2^24, 2^24] and voxel corners within [0, 2^23), so the
// differences fit int32.
VX_HD inline void cap_setup(const int32_t* r, const int64_t v[3], int64_t s, int Sb, CapIn& q) {
  double M = double(s);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t ci = r[a] - (int32_t(v[a]) << Sb);
    const int32_t di = r[3 + a] - r[a];
    q.ci[a] = ci;
    q.di[a] = di;
    q.c[a] = double(ci);
    q.d[a] = double(di);
    M = fmax(M, fabs(q.c[a]) + fabs(q.d[a]) + double(s));
  }
  q.err = M * M * 0x1p-44;
}

// The box holds the ball of radius h = s/2 around its centre and lies in the ball of radius
// h sqrt(3): the distance from the centre to the segment decides most candidates.
// Returns 1 (touch), 0 (no touch) or -1 (undecided: cap_bracket decides).
// 1 / |B - A|^2 of a segment record in lattice units (0 for a point): the ball test's only
// quotient, the same for all of the segment's candidates
VX_HD inline double cap_inv_len2(const int32_t* r) {
  double dd = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double d = double(r[3 + a] - r[a]);
    dd = fma(d, d, dd);
  }
  return dd > 0.0 ? 1.0 / dd : 0.0;
}

// inv_dd: cap_inv_len2(r).  The parameter tc of the point nearest the centre is a product by it
// rather than a quotient: any tc in [0, 1] names a point of the segment, and its rounding moves
// the distance by far less than err.
VX_HD inline int cap_ball(const int32_t* r, const int64_t v[3], int64_t s, int Sb, int64_t rho, double inv_dd) {
  CapIn q;
  cap_setup(r, v, s, Sb, q);
  const double h = 0.5 * double(s);
  double wx = h - q.c[0], wy = h - q.c[1], wz = h - q.c[2];
  double tc = (wx * q.d[0] + wy * q.d[1] + wz * q.d[2]) * inv_dd;
  tc = fmin(fmax(tc, 0.0), 1.0);
  wx = fma(-tc, q.d[0], wx);
  wy = fma(-tc, q.d[1], wy);
  wz = fma(-tc, q.d[2], wz);
  const double dc2 = wx * wx + wy * wy + wz * wz;
  const double rin = h + double(rho);
  if (dc2 + q.err <= rin * rin) return 1;
  const double rout = h * 1.7320508075688772 + double(rho);
  if (dc2 - q.err > rout * rout * (1.0 + 0x1p-40)) return 0;
  // Second look at the same point: f(t), the squared distance from the segment's point at t to
  // the box, is convex and continuously differentiable, so f(tc) <= rho^2 is a touch and the
  // tangent at tc bounds f from below on [0, 1].  Every rounding here stays far inside err.
  const double ds = double(s);
  double f = 0.0, g = 0.0;                  // f(tc) and f'(tc) / 2
  for (int a = 0; a < 3; ++a) {
    const double x = fma(tc, q.d[a], q.c[a]);
    const double e = x < 0 ? x : (x > ds ? x - ds : 0.0);
    f = fma(e, e, f);
    g = fma(e, q.d[a], g);
  }
  const double r2 = double(rho) * double(rho);
  if (f + q.err <= r2) return 1;
  const double lb = g > 0.0 ? fma(-2.0 * g, tc, f) : fma(2.0 * g, 1.0 - tc, f);
  if (lb - q.err > r2) return 0;
  return -1;
}

// f is convex and piecewise quadratic, so f' is monotone and piecewise linear with its
// breakpoints where a coordinate crosses 0 or s.  Let t_lo be the largest of {0, 1,
// breakpoints} with f' <= 0 and t_hi the smallest with f' >= 0: no breakpoint lies strictly
// between them, f' is linear there and its zero is the minimiser.
VX_HD inline bool cap_bracket(const int32_t* r, const int64_t v[3], int64_t s, int Sb, int64_t rho) {
  CapIn q;
  cap_setup(r, v, s, Sb, q);
  const double ds = double(s);
  const double r2 = double(rho) * double(rho);
  double tb[8];
  tb[0] = 0.0;
  tb[1] = 1.0;
  for (int a = 0; a < 3; ++a) {
    double t0 = 0.0, t1 = 0.0;
    if (q.di[a] != 0) {
      const double inv = 1.0 / q.d[a];
      t0 = fmin(fmax(-q.c[a] * inv, 0.0), 1.0);
      t1 = fmin(fmax((ds - q.c[a]) * inv, 0.0), 1.0);
    }
    tb[2 + 2 * a] = t0;
    tb[3 + 2 * a] = t1;
  }
  double t_lo = -1.0, g_lo = 0.0, t_hi = 2.0, g_hi = 0.0;
  for (int k = 0; k < 8; ++k) {
    const double t = tb[k];
    double g = 0.0;                         // f'(t) / 2
    for (int a = 0; a < 3; ++a) {
      const double x = fma(t, q.d[a], q.c[a]);
      const double e = x < 0 ? x : (x > ds ? x - ds : 0.0);
      g = fma(e, q.d[a], g);
    }
    if (g <= 0.0 && t > t_lo) { t_lo = t; g_lo = g; }
    if (g >= 0.0 && t < t_hi) { t_hi = t; g_hi = g; }
  }
  double ts;
  if (t_lo < 0.0) ts = 0.0;                 // f' > 0 on [0, 1]
  else if (t_hi > 1.0) ts = 1.0;            // f' < 0 on [0, 1]
  else if (t_hi <= t_lo || g_hi - g_lo <= 0.0) ts = t_lo;
  else ts = fmin(fmax(t_lo - g_lo * (t_hi - t_lo) / (g_hi - g_lo), t_lo), t_hi);
  const double fmin_ = fdist2(ts, q.c, q.d, ds);
  if (fmin_ + q.err <= r2) return true;
  if (fmin_ - q.err > r2) return false;
  return cap_exact(q.ci[0], q.ci[1], q.ci[2], q.di[0], q.di[1], q.di[2], s, rho);
}

VX_HD inline bool cap_touch(const int32_t* r, const int64_t v[3], int64_t s, int Sb, int64_t rho) {
  const int b = cap_ball(r, v, s, Sb, rho, cap_inv_len2(r));
  return b >= 0 ? b == 1 : cap_bracket(r, v, s, Sb, rho);
}

// ---------------------------------------------------------------------------------------------
// weights
// ---------------------------------------------------------------------------------------------
// length of the segment inside [v, v+1)^3 in voxel units (half-open for axis-parallel segments)
VX_HD inline float seg_length(const int32_t* r, const int64_t v[3], int Sb, float len_vox) {
  double t0 = 0.0, t1 = 1.0;
  const double inv_s = 1.0 / double(int64_t(1) << Sb);
  bool empty = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t ci = int64_t(r[a]) - (v[a] << Sb);
    const int64_t di = int64_t(r[3 + a]) - int64_t(r[a]);
    if (di == 0) {
      empty = empty || !(ci >= 0 && ci < (int64_t(1) << Sb));
    } else {
      const double c = double(ci) * inv_s, d = double(di) * inv_s;
      const double ta = -c / d, tb = (1.0 - c) / d;
      t0 = fmax(t0, fmin(ta, tb));
      t1 = fmin(t1, fmax(ta, tb));
    }
  }
  if (empty || !(t1 > t0)) return 0.0f;
  return float((t1 - t0) * double(len_vox));
}

// Length (voxel units) of the segment A-B inside [lo, lo+1)^3 and its derivatives with respect
// to both ends, FP64 voxel coordinates.  A clipped end slides inside its clipping plane when an
// end point moves: its velocity is the end point's velocity projected along d onto that plane.
VX_HD inline double seg_length_grad(const double A[3], const double B[3], const double lo[3], double gA[3],
                                    double gB[3]) {
  double d[3];
  double t_in = 0.0, t_out = 1.0;
  int ax_in = -1, ax_out = -1;
  for (int a = 0; a < 3; ++a) {
    gA[a] = 0.0;
    gB[a] = 0.0;
    d[a] = B[a] - A[a];
  }
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (!(A[a] >= lo[a] && A[a] < lo[a] + 1.0)) return 0.0;
      continue;
    }
    const double t0 = (lo[a] - A[a]) / d[a], t1 = (lo[a] + 1.0 - A[a]) / d[a];
    const double lo_t = t0 < t1 ? t0 : t1, hi_t = t0 < t1 ? t1 : t0;
    if (lo_t > t_in) { t_in = lo_t; ax_in = a; }
    if (hi_t < t_out) { t_out = hi_t; ax_out = a; }
  }
  if (!(t_out > t_in)) return 0.0;
  const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  // length = u . (exit - entry), u = d / len; a free end moves with its point, a clipped end
  // with that motion minus its component that leaves the plane along d
  double ue[3], ui[3];
  for (int a = 0; a < 3; ++a) { ue[a] = d[a] / len; ui[a] = d[a] / len; }
  if (ax_out >= 0) ue[ax_out] -= len / d[ax_out];
  if (ax_in >= 0) ui[ax_in] -= len / d[ax_in];
  for (int a = 0; a < 3; ++a) {
    gA[a] = ue[a] * (1.0 - t_out) - ui[a] * (1.0 - t_in);
    gB[a] = ue[a] * t_out - ui[a] * t_in;
  }
  return (t_out - t_in) * len;
}

VX_HD inline Lat make_lat(const vx_grid* g, int kind, float radius) {
  Lat L;
  for (int a = 0; a < 3; ++a) L.bmin[a] = g->bmin[a];
  L.inv = ldexp(1.0, 23) / g->extent;
  L.Sb = 23 - g->log2_res;
  L.s = int64_t(1) << L.Sb;
  L.R = 1 << g->log2_res;
  L.rho = kind == 1 ? int64_t(rint(double(radius) * L.inv)) : 0;
  return L;
}

// Area of the triangle inside [v, v+1)^3 (voxel^2), in registers.
//
// In the triangle's barycentric plane (l1, l2) -- the point q0 + l1 (q1 - q0) + l2 (q2 - q0) --
// the piece is the convex polygon cut out by half-planes h(l) = a + b l1 + g l2 >= 0: the
// triangle's three (l1 >= 0, l2 >= 0, 1 - l1 - l2 >= 0) and the box's, x >= 0 and s - x >= 0 for
// every axis (x in lattice units from the voxel corner).  A box half-plane that holds on the
// whole (closed) triangle clips nothing and is left out; one that no point passes strictly
// empties the piece.  By Green's theorem the area is half the sum over the polygon's edges of
// the cross products of their end points, and each line carries at most one edge: walked in
// direction (g, -b), inside on the left, from the foot P = -a (b, g) / n of the origin
// (n = b^2 + g^2), its edge runs from the last constraint turning inside (D > 0) to the first
// turning outside (D < 0), D = g_j . (g, -b), and contributes cross(P_e, P_x) = a (t_x - t_e).
// The two lines through the origin (l1 = 0, l2 = 0) contribute nothing; they only bound.
//
// Line intersections come from Cramer's rule with exact numerators and denominators (lattice
// integers below 2^25: products below 2^52).  Each pair of lines is visited once and bounds both
// of its lines; the best bounds are chosen by comparing cross products of numerators and
// denominators (no division), and the chosen ones are then divided exactly (one rounding, the
// same for every pair of lines through one point), so a piece that degenerates to a point or a
// segment closes exactly and has area 0.
// A line is parametrised by the coordinate (l1 or l2) that changes more along it.  Parallel
// lines are decided exactly: an outside one removes the line, a coincident one with the same
// inside keeps the edge on one line only, one with the opposite inside flattens the piece (area
// 0).  A triangle flat on an axis has no lines on it: it lies in one layer [k, k+1) or in none.
//
// The fast form holds each axis's active lines as one primary line and, for one axis only, a
// second: when the triangle crosses both box planes of two axes, the exact routine below takes
// the piece.
struct AreaLine {
  double a, b, g;      // h(l) = a + b l1 + g l2
  bool on;
};

// the bounds of one line K: walked with the inside on its left, parametrised by the coordinate
// (l1 or l2) that changes more along it, sig = +-1 so that sig * coordinate grows along the walk
struct AreaEdge {
  bool use_x, dead;
  double sig;
  double ne, de;       // entry: exact numerator and denominator of the coordinate (de = 0: none yet)
  double nx, dx;       // exit
};

VX_HD inline void area_edge_init(AreaEdge& E, const AreaLine& K) {
  E.use_x = fabs(K.g) >= fabs(K.b);
  E.sig = E.use_x ? (K.g > 0.0 ? 1.0 : -1.0) : (K.b > 0.0 ? -1.0 : 1.0);
  E.dead = false;
  E.ne = 0.0;
  E.de = 0.0;
  E.nx = 0.0;
  E.dx = 0.0;
}

// K bounded where it meets another line at (N1 / D, N2 / D); the other line turns inside along
// K where D > 0 (an entry) and outside where D < 0 (an exit).  The latest entry and the earliest
// exit along the walk are kept: sig n / D against sig ne / de with both sides multiplied by the
// positive D de (D dx for exits); the first of equal bounds stays.
VX_HD inline void area_bound(AreaEdge& E, double D, double N1, double N2, bool valid = true) {
  const double n = E.use_x ? N1 : N2;
  // one comparison for either side (no branch per side): an entry is later when sig n / D is
  // larger, an exit earlier when it is smaller
  const bool ent = D > 0.0;
  const double dc = ent ? E.de : E.dx, nc = ent ? E.ne : E.nx;
  const double l = n * dc, r = nc * D;
  const bool take = valid && (dc == 0.0 || (((E.sig > 0.0) == ent) ? l > r : l < r));
  const bool te = take && ent, tx = take && !ent;
  E.ne = te ? n : E.ne;
  E.de = te ? D : E.de;
  E.nx = tx ? n : E.nx;
  E.dx = tx ? D : E.dx;
}

// the sign along K of a parallel line's half-plane, from the exact intersection numerators
VX_HD inline double parallel_side(const AreaLine& K, double N1, double N2) {
  return K.b != 0.0 ? (K.b > 0.0 ? N2 : -N2) : (K.g > 0.0 ? -N1 : N1);
}

// K (index ik) against the triangle's line T: 0 (l1 = 0), 1 (l2 = 0), 2 (l1 + l2 = 1), whose
// constant coefficients fold.  A box line never coincides with a triangle line here (one through
// a triangle edge holds on the whole triangle or empties the piece).
template <int T>
VX_HD inline void area_tri_bound(AreaEdge& E, const AreaLine& K) {
  double D, N1, N2;
  if (T == 0) { D = K.g; N1 = 0.0; N2 = -K.a; }
  else if (T == 1) { D = -K.b; N1 = K.a; N2 = 0.0; }
  else { D = K.b - K.g; N1 = -(K.a + K.g); N2 = K.a + K.b; }
  const bool par = D == 0.0;
  if (par && parallel_side(K, N1, N2) < 0.0) E.dead = true;
  area_bound(E, D, N1, N2, !par);
}

// K (index ik) against another box line J (index ij)
VX_HD inline void area_box_bound(AreaEdge& E, const AreaLine& K, int ik, const AreaLine& J, int ij, bool& flat) {
  if (!J.on) return;
  const double D = fma(J.b, K.g, -(J.g * K.b));           // exact
  const double N1 = fma(K.a, J.g, -(J.a * K.g));          // intersection (N1 / D, N2 / D), exact
  const double N2 = fma(J.a, K.b, -(K.a * J.b));
  if (D == 0.0) {
    const double side = parallel_side(K, N1, N2);
    if (side < 0.0) E.dead = true;
    if (side == 0.0) {                                    // coincident
      if (fma(J.b, K.b, J.g * K.g) < 0.0) flat = true;    // opposite insides: a segment
      if (ij < ik) E.dead = true;                         // the edge stays on the lower line
    }
    return;
  }
  area_bound(E, D, N1, N2);
}

// the edge's cross-product term a (t_x - t_e).  t_x - t_e = nx / dx - ne / de =
// (nx de - ne dx) / (dx de); the numerator is formed exactly up to its final rounding (each
// product split into its rounded value and exact error by an FMA), so it is exactly 0 when the
// two bounds meet in one point: a piece that closes to a point or a segment adds nothing.
VX_HD inline double area_edge_term(const AreaEdge& E, const AreaLine& K) {
  const double p1 = E.nx * E.de, p2 = E.ne * E.dx;
  const double num = (p1 - p2) + (fma(E.nx, E.de, -p1) - fma(E.ne, E.dx, -p2));
  // sig (t_x - t_e) > 0 with dx de < 0 (de > 0 > dx): sig num < 0.  Without both bounds (or on a
  // dead line) there is no edge; the term is computed regardless and dropped.
  const double sn = E.sig * num;
  const bool edge = !E.dead && E.de != 0.0 && E.dx != 0.0 && sn < 0.0;
  const double t = K.a * sn * rcp_fast(E.dx * E.de * (E.use_x ? fabs(K.g) : fabs(K.b)));
  return edge ? t : 0.0;
}

// line ik's edge bounded by the triangle's lines and every other box line
template <int IK>
VX_HD inline double area_line_term(const AreaLine* L, bool& flat) {
  const AreaLine& K = L[IK];
  if (!K.on) return 0.0;
  AreaEdge E;
  area_edge_init(E, K);
  area_tri_bound<0>(E, K);
  area_tri_bound<1>(E, K);
#pragma unroll
  for (int j = 2; j < 7; ++j)
    if (j != IK) {
      if (j == 2) area_tri_bound<2>(E, K);
      else area_box_bound(E, K, IK, L[j], j, flat);
    }
  return area_edge_term(E, K);
}

// the piece's area in barycentric units (the whole triangle has 1/2), or -1 when the exact
// routine must take it
VX_HD inline double tri_area_bary(const int32_t* q, const int64_t v[3], int Sb) {
  const int32_t s = int32_t(1) << Sb;
  const double ds = double(s);
  // lines 2..6: the triangle's l1 + l2 = 1 (always there), the primary box line of x, y, z and
  // one second box line (l1 >= 0 and l2 >= 0 only bound; their coefficients are folded in)
  AreaLine L[7];
  L[2] = {1.0, -1.0, -1.0, true};
  L[6] = {0.0, 0.0, 0.0, false};
  bool second = false;
  // the first deciding case over the axes, in axis order: 1 an empty piece (area 0), 2 two axes
  // crossed through (the exact routine); the axes are set up without a branch each
  int ev = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t c0 = q[a] - (int32_t(v[a]) << Sb);
    const int32_t e0 = q[3 + a] - q[a];
    const int32_t e1 = q[6 + a] - q[a];
    const double c = double(c0), d0 = double(e0), d1 = double(e1);
    const bool flat = e0 == 0 && e1 == 0;
    const bool flat_out = flat && !(c0 >= 0 && c0 < s);   // flat on axis a, owned by another layer
    // the two box half-planes of this axis at the vertices (0, 0), (1, 0), (0, 1), exact
    const double l0 = c, l1 = c + d0, l2 = c + d1;
    const double u0 = ds - c, u1 = u0 - d0, u2 = u0 - d1;
    const bool empty = !flat && (fmax(l0, fmax(l1, l2)) <= 0.0 || fmax(u0, fmax(u1, u2)) <= 0.0);
    const bool lo = !flat && fmin(l0, fmin(l1, l2)) < 0.0, hi = !flat && fmin(u0, fmin(u1, u2)) < 0.0;
    const bool both = lo && hi;
    ev = ev != 0 ? ev : (flat_out || empty ? 1 : (both && second ? 2 : 0));
    if (both && !second) L[6] = {u0, -d0, -d1, true};
    second = second || both;
    L[3 + a] = lo ? AreaLine{c, d0, d1, true} : (hi ? AreaLine{u0, -d0, -d1, true} : AreaLine{0.0, 0.0, 0.0, false});
  }
  if (ev == 1) return 0.0;
  if (ev == 2) return -1.0;
  bool flat = false;
  const double sum = area_line_term<2>(L, flat) + area_line_term<3>(L, flat) + area_line_term<4>(L, flat) +
                     area_line_term<5>(L, flat) + area_line_term<6>(L, flat);
  if (flat) return 0.0;
  return 0.5 * fabs(sum);
}

// The same area with exactly computed line intersections (Cramer's rule with exact numerators and
// denominators, one rounding each; both lines of a vertex compute it alike, so a degenerate
// piece closes exactly and has area 0): one line at a time against all the others.
VX_HD inline __attribute__((noinline)) double tri_area_exact(const int32_t* q, int64_t v0, int64_t v1, int64_t v2,
                                                             int Sb) {
  const int64_t v[3] = {v0, v1, v2};
  const int32_t s = int32_t(1) << Sb;
  const double ds = double(s);
  double al[9], be[9], ga[9];
  al[0] = 0.0; be[0] = 1.0; ga[0] = 0.0;
  al[1] = 0.0; be[1] = 0.0; ga[1] = 1.0;
  al[2] = 1.0; be[2] = -1.0; ga[2] = -1.0;
  unsigned act = 7u;
  for (int a = 0; a < 3; ++a) {
    const int32_t c0 = q[a] - (int32_t(v[a]) << Sb);
    const int32_t e0 = q[3 + a] - q[a];
    const int32_t e1 = q[6 + a] - q[a];
    al[3 + 2 * a] = double(c0);
    be[3 + 2 * a] = double(e0);
    ga[3 + 2 * a] = double(e1);
    al[4 + 2 * a] = ds - double(c0);
    be[4 + 2 * a] = -double(e0);
    ga[4 + 2 * a] = -double(e1);
    if (e0 == 0 && e1 == 0) {
      if (!(c0 >= 0 && c0 < s)) return 0.0;
      continue;
    }
    for (int side = 0; side < 2; ++side) {
      const int k = 3 + 2 * a + side;
      const double h0 = al[k], h1 = al[k] + be[k], h2 = al[k] + ga[k];
      if (fmax(h0, fmax(h1, h2)) <= 0.0) return 0.0;
      if (fmin(h0, fmin(h1, h2)) <= 0.0) act |= 1u << k;
    }
  }
  double sum = 0.0;
  for (int k = 2; k < 9; ++k) {
    if (!((act >> k) & 1u)) continue;
    const double ak = al[k], bk = be[k], gk = ga[k];
    const double nk = fma(bk, bk, gk * gk);
    double Te = -1.0, De = 0.0, N1e = 0.0, N2e = 0.0;    // De = 0: no entry bound yet
    double Tx = 1.0, Dx = 0.0, N1x = 0.0, N2x = 0.0;
    bool dead = false;
    for (int j = 0; j < 9; ++j) {
      if (j == k || !((act >> j) & 1u)) continue;
      const double D = fma(be[j], gk, -(ga[j] * bk));
      const double N1 = fma(ak, ga[j], -(al[j] * gk));
      const double N2 = fma(al[j], bk, -(ak * be[j]));
      const double dot = fma(be[j], bk, ga[j] * gk);
      if (D == 0.0) {
        const double hs = bk != 0.0 ? (bk > 0.0 ? N2 : -N2) : (gk > 0.0 ? -N1 : N1);
        if (hs < 0.0) dead = true;
        else if (hs == 0.0) {
          if (dot < 0.0) return 0.0;
          if (j < k) dead = true;
        }
        continue;
      }
      const double T = fma(ak, dot, -(al[j] * nk));
      if (D > 0.0) {
        if (De == 0.0 || T * De > Te * D) { Te = T; De = D; N1e = N1; N2e = N2; }
      } else {
        if (Dx == 0.0 || T * Dx < Tx * D) { Tx = T; Dx = D; N1x = N1; N2x = N2; }
      }
    }
    if (dead || De == 0.0 || Dx == 0.0) continue;
    const double xe = N1e / De, ye = N2e / De, xx = N1x / Dx, yx = N2x / Dx;
    const double te = fma(gk, xe, -(bk * ye)), tx = fma(gk, xx, -(bk * yx));
    if (!(tx > te)) continue;
    sum += fma(xe, yx, -(ye * xx));
  }
  return 0.5 * fabs(sum);
}

// area of the triangle inside [v, v+1)^3 in voxel^2 (area2: twice the triangle's area)
VX_HD inline float tri_area(const int32_t* q, const int64_t v[3], int Sb, float area2) {
  if (!(area2 > 0.0f)) return 0.0f;
  double a = tri_area_bary(q, v, Sb);
  if (a < 0.0) a = tri_area_exact(q, v[0], v[1], v[2], Sb);
  return float(a * double(area2));
}

}  // namespace vx
