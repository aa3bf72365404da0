// vxo.cpp -- FP64 CPU oracle for sparse SGGX voxelization (TEST INFRASTRUCTURE ONLY).
//
// Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load this
// library.  It shares no code with the HIP path: it is a plain, slow, direct statement of
// what the voxelizer computes, in double precision with exact integer predicates.
//
// What it computes (paper Sec. 3.1 grid transform; Sec. 3.3 gathering of everything a
// primitive contributes to a leaf voxel; Sec. 3.4 / Sec. 4.1 one SGGX matrix per voxel;
// Sec. 4.3 2x2x2 aggregation; Sec. 4.4 merging of similar lobes), under these readings:
//   * Sec. 3.1 transform: P_volume = (P - bmin) / extent * R with cubic bounds.  Both the
//     oracle and the GPU snap P_volume to the lattice of 2^-(23 - log2 R) voxel:
//     q = nearbyint((double(P) - bmin) * (2^23 / extent)), so one voxel is s = 2^(23-log2R)
//     lattice units and every predicate below is an exact integer computation.
//   * a primitive touches voxel v iff it meets the CLOSED box [v, v+1]^3 (triangles), or
//     its centreline lies within distance r of that closed box (fibers / capsules).
//   * weights use half-open ownership [v, v+1)^3: the clipped triangle area, or the
//     clipped centreline length, in voxel units.
//   * moments: M = n n^T for a triangle's unit normal, M = I - t t^T for a segment's unit
//     tangent (the SGGX surface and fiber forms); zero for degenerate primitives.
//   * per voxel: count = number of touching primitives, w = sum of weights,
//     S = sum of weight * M (unnormalised; the SGGX matrix is S / w).
//   * keys: Morton order, x at bit 3b, y at 3b+1, z at 3b+2, parent = key >> 3.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC -pthread vxo.cpp -o libvxo.so
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

typedef long long i64;
typedef __int128 i128;
typedef unsigned long long u64;

namespace {

constexpr int OK = 0, E_ARG = 1, E_INPUT = 4;

struct Lattice {
  double bmin[3];
  double inv;     // lattice units per world unit = 2^23 / extent
  int log2R;
  i64 R;
  i64 s;          // lattice units per voxel
};

bool make_lattice(const double* bmin, double extent, int log2R, Lattice* L) {
  if (!(extent > 0.0) || !std::isfinite(extent) || log2R < 1 || log2R > 20) return false;
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(bmin[a])) return false;
    L->bmin[a] = bmin[a];
  }
  L->inv = std::ldexp(1.0, 23) / extent;
  L->log2R = log2R;
  L->R = i64(1) << log2R;
  L->s = i64(1) << (23 - log2R);
  return true;
}

// Sec. 3.1 normalisation, snapped to the lattice.  Lattice coordinates must lie in
// [-2^23, 2^24] (one grid of margin on every side), else the input is rejected.
int snap(const Lattice& L, const float* p, i64 q[3]) {
  for (int a = 0; a < 3; ++a) {
    double x = double(p[a]);
    if (!std::isfinite(x)) return E_INPUT;
    double g = (x - L.bmin[a]) * L.inv;
    double r = std::nearbyint(g);
    if (!(r >= -8388608.0 && r <= 16777216.0)) return E_INPUT;
    q[a] = i64(r);
  }
  return OK;
}

u64 morton(i64 x, i64 y, i64 z, int bits) {
  u64 k = 0;
  for (int b = 0; b < bits; ++b) {
    k |= u64((x >> b) & 1) << (3 * b);
    k |= u64((y >> b) & 1) << (3 * b + 1);
    k |= u64((z >> b) & 1) << (3 * b + 2);
  }
  return k;
}

i64 floor_div(i64 a, i64 s) { return a >= 0 ? a / s : -((-a + s - 1) / s); }
i64 ceil_div(i64 a, i64 s) { return -floor_div(-a, s); }

// ---------------------------------------------------------------------------------------------
// Triangles: exact closed-box separating-axis test on lattice integers.
// ---------------------------------------------------------------------------------------------
bool tri_touch(const i64 q[3][3], const i64 lo[3], i64 s) {
  // the three box normals
  for (int a = 0; a < 3; ++a) {
    i64 mn = std::min({q[0][a], q[1][a], q[2][a]});
    i64 mx = std::max({q[0][a], q[1][a], q[2][a]});
    if (mx < lo[a] || mn > lo[a] + s) return false;
  }
  i64 e[3][3];
  for (int a = 0; a < 3; ++a) {
    e[0][a] = q[1][a] - q[0][a];
    e[1][a] = q[2][a] - q[1][a];
    e[2][a] = q[0][a] - q[2][a];
  }
  // the triangle's plane: corners' signed offsets n . (c - q0) must not all share a strict sign
  i64 n[3] = {e[0][1] * (-e[2][2]) - e[0][2] * (-e[2][1]),
              e[0][2] * (-e[2][0]) - e[0][0] * (-e[2][2]),
              e[0][0] * (-e[2][1]) - e[0][1] * (-e[2][0])};
  i128 base = 0, lo_off = 0, hi_off = 0;
  for (int a = 0; a < 3; ++a) {
    base += i128(n[a]) * i128(lo[a] - q[0][a]);
    if (n[a] > 0) hi_off += i128(n[a]) * s; else lo_off += i128(n[a]) * s;
  }
  if (base + lo_off > 0 || base + hi_off < 0) return false;
  // nine cross products of a triangle edge with a box axis
  for (int j = 0; j < 3; ++j) {
    for (int k = 0; k < 3; ++k) {
      i64 ax[3];
      if (k == 0) { ax[0] = 0; ax[1] = -e[j][2]; ax[2] = e[j][1]; }
      else if (k == 1) { ax[0] = e[j][2]; ax[1] = 0; ax[2] = -e[j][0]; }
      else { ax[0] = -e[j][1]; ax[1] = e[j][0]; ax[2] = 0; }
      i128 pmin = 0, pmax = 0;
      for (int i = 0; i < 3; ++i) {
        i128 p = 0;
        for (int a = 0; a < 3; ++a) p += i128(ax[a]) * q[i][a];
        if (i == 0 || p < pmin) pmin = p;
        if (i == 0 || p > pmax) pmax = p;
      }
      i128 blo = 0, bhi = 0;
      for (int a = 0; a < 3; ++a) {
        blo += i128(ax[a]) * lo[a];
        bhi += i128(ax[a]) * lo[a];
        if (ax[a] > 0) bhi += i128(ax[a]) * s; else blo += i128(ax[a]) * s;
      }
      if (pmax < blo || pmin > bhi) return false;
    }
  }
  return true;
}

// Area of the part of the triangle inside [v, v+1)^3, voxel units, by clipping against the
// six box planes.
// A triangle lying in an axis plane x_a = c belongs to the voxels with v_a <= c < v_a + 1.
double tri_area(const i64 q[3][3], const i64 lo[3], i64 s) {
  bool flat[3];
  for (int a = 0; a < 3; ++a) {
    flat[a] = (q[0][a] == q[1][a] && q[1][a] == q[2][a]);
    if (flat[a] && !(lo[a] <= q[0][a] && q[0][a] < lo[a] + s)) return 0.0;
  }
  std::vector<std::array<double, 3>> poly(3), next;
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) poly[i][a] = double(q[i][a] - lo[a]) / double(s);
  for (int a = 0; a < 3; ++a) {
    if (flat[a]) continue;
    for (int side = 0; side < 2; ++side) {
      next.clear();
      size_t m = poly.size();
      for (size_t i = 0; i < m; ++i) {
        const auto& P = poly[i];
        const auto& Q = poly[(i + 1) % m];
        double dp = side == 0 ? P[a] : 1.0 - P[a];
        double dq = side == 0 ? Q[a] : 1.0 - Q[a];
        bool ip = dp >= 0.0, iq = dq >= 0.0;
        if (ip) next.push_back(P);
        if (ip != iq) {
          double t = dp / (dp - dq);
          std::array<double, 3> X;
          for (int c = 0; c < 3; ++c) X[c] = P[c] + t * (Q[c] - P[c]);
          next.push_back(X);
        }
      }
      poly.swap(next);
      if (poly.size() < 3) return 0.0;
    }
  }
  double A[3] = {0, 0, 0};
  for (size_t i = 1; i + 1 < poly.size(); ++i) {
    double u[3], v[3];
    for (int c = 0; c < 3; ++c) {
      u[c] = poly[i][c] - poly[0][c];
      v[c] = poly[i + 1][c] - poly[0][c];
    }
    A[0] += u[1] * v[2] - u[2] * v[1];
    A[1] += u[2] * v[0] - u[0] * v[2];
    A[2] += u[0] * v[1] - u[1] * v[0];
  }
  return 0.5 * std::sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
}

// ---------------------------------------------------------------------------------------------
// Capsules: exact test dist(segment, closed box) <= rho on lattice integers.
// f(t) = dist^2(c + t d, [0, s]^3) is convex and piecewise quadratic in t; its minimum over
// [0, 1] is attained at 0, 1, a breakpoint (where some coordinate crosses 0 or s), or at the
// stationary point of the quadratic of one piece.  Every candidate is a rational num/den and
// is evaluated exactly.
// ---------------------------------------------------------------------------------------------
struct Rat { i128 num, den; };   // den > 0

bool rat_less(const Rat& a, const Rat& b) { return a.num * b.den < b.num * a.den; }

// f(num/den) * den^2 <= rho^2 * den^2 ?
bool eval_le(const i64 c[3], const i64 d[3], i64 s, i64 rho, const Rat& t) {
  i128 sum = 0;
  for (int a = 0; a < 3; ++a) {
    i128 g = i128(c[a]) * t.den + t.num * i128(d[a]);
    i128 sd = i128(s) * t.den;
    i128 dist = g < 0 ? -g : (g > sd ? g - sd : 0);
    sum += dist * dist;
  }
  return sum <= i128(rho) * rho * t.den * t.den;
}

bool cap_touch(const i64 c[3], const i64 d[3], i64 s, i64 rho) {
  std::vector<Rat> ts = {{0, 1}, {1, 1}};
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0) continue;
    for (i64 b : {i64(0), s}) {
      Rat t{i128(b - c[a]), i128(d[a])};
      if (t.den < 0) { t.num = -t.num; t.den = -t.den; }
      if (t.num > 0 && t.num < t.den) ts.push_back(t);
    }
  }
  std::sort(ts.begin(), ts.end(), rat_less);
  for (const Rat& t : ts)
    if (eval_le(c, d, s, rho, t)) return true;
  for (size_t i = 0; i + 1 < ts.size(); ++i) {
    const Rat& ta = ts[i];
    const Rat& tb = ts[i + 1];
    if (!rat_less(ta, tb)) continue;
    // side of every axis on the open piece, read at its midpoint
    Rat mid{ta.num * tb.den + tb.num * ta.den, 2 * ta.den * tb.den};
    i128 Q = 0, P = 0;
    i64 e[3];
    bool act[3];
    for (int a = 0; a < 3; ++a) {
      i128 g = i128(c[a]) * mid.den + mid.num * i128(d[a]);
      act[a] = true;
      if (g < 0) e[a] = c[a];
      else if (g > i128(s) * mid.den) e[a] = c[a] - s;
      else { act[a] = false; e[a] = 0; }
      if (act[a]) {
        Q += i128(d[a]) * d[a];
        P -= i128(e[a]) * d[a];
      }
    }
    if (!act[0] && !act[1] && !act[2]) return true;   // the piece runs inside the box
    if (Q == 0) continue;                              // constant on the piece
    // stationary point P/Q strictly inside (ta, tb)?
    if (!(P * ta.den > ta.num * Q && P * tb.den < tb.num * Q)) continue;
    // minimum value * Q = |e x d|^2 over the active axes (Lagrange identity)
    i128 num = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = a + 1; b < 3; ++b) {
        if (!act[a] || !act[b]) continue;
        i128 x = i128(e[a]) * d[b] - i128(e[b]) * d[a];
        num += x * x;
      }
    if (num <= i128(rho) * rho * Q) return true;
  }
  return false;
}

// Length of the centreline inside [v, v+1)^3, voxel units (Liang-Barsky parameter clip).
double seg_length(const i64 c[3], const i64 d[3], i64 s) {
  double t0 = 0.0, t1 = 1.0;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0) {
      if (!(c[a] >= 0 && c[a] < s)) return 0.0;
      continue;
    }
    double ta = double(-c[a]) / double(d[a]);
    double tb = double(s - c[a]) / double(d[a]);
    t0 = std::max(t0, std::min(ta, tb));
    t1 = std::min(t1, std::max(ta, tb));
  }
  if (t1 <= t0) return 0.0;
  double len = std::sqrt(double(d[0]) * d[0] + double(d[1]) * d[1] + double(d[2]) * d[2]) / double(s);
  return (t1 - t0) * len;
}

// ---------------------------------------------------------------------------------------------
// Gathering and aggregation.
// ---------------------------------------------------------------------------------------------
struct Pair { u64 key; i64 prim; double w; };

struct Result {
  std::vector<u64> keys;
  std::vector<uint32_t> count;
  std::vector<double> w;
  std::vector<double> S;   // [n][6]: xx yy zz xy xz yz
  i64 n_pairs = 0;
};

struct Region { i64 lo[3], hi[3]; };   // voxel indices, hi exclusive

void candidate_range(const i64 mn[3], const i64 mx[3], i64 s, const Region& rg, i64 vlo[3], i64 vhi[3]) {
  for (int a = 0; a < 3; ++a) {
    vlo[a] = std::max(ceil_div(mn[a], s) - 1, rg.lo[a]);
    vhi[a] = std::min(floor_div(mx[a], s), rg.hi[a] - 1);
  }
}

Result* reduce_pairs(std::vector<std::vector<Pair>>& parts, const std::vector<double>& M /*[prim][6]*/) {
  std::vector<Pair> all;
  size_t tot = 0;
  for (auto& p : parts) tot += p.size();
  all.reserve(tot);
  for (auto& p : parts) { all.insert(all.end(), p.begin(), p.end()); std::vector<Pair>().swap(p); }
  std::sort(all.begin(), all.end(), [](const Pair& a, const Pair& b) {
    return a.key != b.key ? a.key < b.key : a.prim < b.prim;
  });
  Result* r = new Result;
  r->n_pairs = i64(all.size());
  for (size_t i = 0; i < all.size();) {
    size_t j = i;
    double w = 0, S[6] = {0, 0, 0, 0, 0, 0};
    while (j < all.size() && all[j].key == all[i].key) {
      w += all[j].w;
      for (int c = 0; c < 6; ++c) S[c] += all[j].w * M[size_t(all[j].prim) * 6 + c];
      ++j;
    }
    r->keys.push_back(all[i].key);
    r->count.push_back(uint32_t(j - i));
    r->w.push_back(w);
    for (int c = 0; c < 6; ++c) r->S.push_back(S[c]);
    i = j;
  }
  return r;
}

template <class F>
void parallel_for(i64 n, int nthreads, F f) {
  nthreads = std::max(1, nthreads);
  if (nthreads == 1 || n < 1024) { f(0, 0, n); return; }
  std::vector<std::thread> th;
  i64 chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    i64 a = std::min(n, t * chunk), b = std::min(n, a + chunk);
    th.emplace_back(f, t, a, b);
  }
  for (auto& x : th) x.join();
}

Region make_region(const Lattice& L, const i64* region) {
  Region rg;
  for (int a = 0; a < 3; ++a) {
    rg.lo[a] = region ? std::max<i64>(0, region[a]) : 0;
    rg.hi[a] = region ? std::min<i64>(L.R, region[3 + a]) : L.R;
  }
  return rg;
}

}  // namespace

extern "C" {

// status: 0 ok, 1 bad argument, 4 non-finite or out-of-range coordinates
int vxo_snap(const double* bmin, double extent, int log2R, const float* p, i64 n, i64* q_out) {
  Lattice L;
  if (!make_lattice(bmin, extent, log2R, &L)) return E_ARG;
  for (i64 i = 0; i < n; ++i) {
    int st = snap(L, p + 3 * i, q_out + 3 * i);
    if (st) return st;
  }
  return OK;
}

u64 vxo_morton(i64 x, i64 y, i64 z, int bits) { return morton(x, y, z, bits); }

int vxo_tri_touch(const i64* q9, const i64* lo3, i64 s) {
  i64 q[3][3];
  std::memcpy(q, q9, sizeof q);
  return tri_touch(q, lo3, s) ? 1 : 0;
}
double vxo_tri_area(const i64* q9, const i64* lo3, i64 s) {
  i64 q[3][3];
  std::memcpy(q, q9, sizeof q);
  return tri_area(q, lo3, s);
}
int vxo_cap_touch(const i64* a3, const i64* b3, const i64* lo3, i64 s, i64 rho) {
  i64 c[3], d[3];
  for (int k = 0; k < 3; ++k) { c[k] = a3[k] - lo3[k]; d[k] = b3[k] - a3[k]; }
  return cap_touch(c, d, s, rho) ? 1 : 0;
}
double vxo_seg_length(const i64* a3, const i64* b3, const i64* lo3, i64 s) {
  i64 c[3], d[3];
  for (int k = 0; k < 3; ++k) { c[k] = a3[k] - lo3[k]; d[k] = b3[k] - a3[k]; }
  return seg_length(c, d, s);
}

// Voxelize a triangle soup tris[n][3][3].  region (optional, 6 values: lo xyz, hi xyz,
// hi exclusive) restricts the output to voxels inside it.  Returns an opaque result.
void* vxo_voxelize_triangles(const double* bmin, double extent, int log2R, const float* tris, i64 n,
                             const i64* region, int nthreads, int* status) {
  Lattice L;
  if (!make_lattice(bmin, extent, log2R, &L) || n < 0) { *status = E_ARG; return nullptr; }
  std::vector<i64> Q(size_t(n) * 9);
  for (i64 i = 0; i < n * 3; ++i) {
    int st = snap(L, tris + 3 * i, &Q[size_t(i) * 3]);
    if (st) { *status = st; return nullptr; }
  }
  Region rg = make_region(L, region);
  std::vector<double> M(size_t(n) * 6);
  for (i64 i = 0; i < n; ++i) {
    const i64* q = &Q[size_t(i) * 9];
    i64 e0[3], e1[3];
    for (int a = 0; a < 3; ++a) { e0[a] = q[3 + a] - q[a]; e1[a] = q[6 + a] - q[a]; }
    double nn[3] = {double(e0[1] * e1[2] - e0[2] * e1[1]), double(e0[2] * e1[0] - e0[0] * e1[2]),
                    double(e0[0] * e1[1] - e0[1] * e1[0])};
    double l2 = nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2];
    double* m = &M[size_t(i) * 6];
    if (l2 > 0) {
      m[0] = nn[0] * nn[0] / l2; m[1] = nn[1] * nn[1] / l2; m[2] = nn[2] * nn[2] / l2;
      m[3] = nn[0] * nn[1] / l2; m[4] = nn[0] * nn[2] / l2; m[5] = nn[1] * nn[2] / l2;
    } else {
      for (int c = 0; c < 6; ++c) m[c] = 0.0;
    }
  }
  std::vector<std::vector<Pair>> parts(std::max(1, nthreads));
  parallel_for(n, nthreads, [&](int t, i64 a, i64 b) {
    for (i64 i = a; i < b; ++i) {
      i64 q[3][3];
      std::memcpy(q, &Q[size_t(i) * 9], sizeof q);
      i64 mn[3], mx[3], vlo[3], vhi[3];
      for (int c = 0; c < 3; ++c) {
        mn[c] = std::min({q[0][c], q[1][c], q[2][c]});
        mx[c] = std::max({q[0][c], q[1][c], q[2][c]});
      }
      candidate_range(mn, mx, L.s, rg, vlo, vhi);
      for (i64 z = vlo[2]; z <= vhi[2]; ++z)
        for (i64 y = vlo[1]; y <= vhi[1]; ++y)
          for (i64 x = vlo[0]; x <= vhi[0]; ++x) {
            i64 lo[3] = {x * L.s, y * L.s, z * L.s};
            if (!tri_touch(q, lo, L.s)) continue;
            parts[t].push_back({morton(x, y, z, L.log2R), i, tri_area(q, lo, L.s)});
          }
    }
  });
  *status = OK;
  return reduce_pairs(parts, M);
}

}  // extern "C"

namespace {
// Every (segment, voxel) touch of the fibers, with the weight; M receives the segment moments.
int fiber_pairs(const double* bmin, double extent, int log2R, const float* pts, i64 m, const i64* offsets, i64 F,
                double radius, const i64* region, int nthreads, std::vector<std::vector<Pair>>& parts,
                std::vector<double>& M) {
  Lattice L;
  if (!make_lattice(bmin, extent, log2R, &L) || m < 0 || F < 0 || !(radius >= 0) || !std::isfinite(radius))
    return E_ARG;
  if (offsets[0] != 0 || offsets[F] != m) return E_ARG;
  for (i64 f = 0; f < F; ++f)
    if (offsets[f + 1] < offsets[f]) return E_ARG;
  double rr = std::nearbyint(radius * L.inv);
  if (rr > 8388608.0) return E_ARG;
  i64 rho = i64(rr);
  std::vector<i64> Q(size_t(m) * 3);
  for (i64 i = 0; i < m; ++i) {
    int st = snap(L, pts + 3 * i, &Q[size_t(i) * 3]);
    if (st) return st;
  }
  std::vector<char> is_start(size_t(m), 0);
  for (i64 f = 0; f < F; ++f)
    for (i64 i = offsets[f]; i + 1 < offsets[f + 1]; ++i) is_start[size_t(i)] = 1;
  M.assign(size_t(m) * 6, 0.0);
  for (i64 i = 0; i < m; ++i) {
    if (!is_start[size_t(i)]) continue;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = double(Q[size_t(i + 1) * 3 + a] - Q[size_t(i) * 3 + a]);
    double l2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (l2 == 0) continue;
    double* mm = &M[size_t(i) * 6];
    mm[0] = 1.0 - d[0] * d[0] / l2; mm[1] = 1.0 - d[1] * d[1] / l2; mm[2] = 1.0 - d[2] * d[2] / l2;
    mm[3] = -d[0] * d[1] / l2; mm[4] = -d[0] * d[2] / l2; mm[5] = -d[1] * d[2] / l2;
  }
  Region rg = make_region(L, region);
  parts.assign(std::max(1, nthreads), {});
  parallel_for(m, nthreads, [&](int t, i64 a, i64 b) {
    for (i64 i = a; i < b; ++i) {
      if (!is_start[size_t(i)]) continue;
      const i64* A = &Q[size_t(i) * 3];
      const i64* B = &Q[size_t(i + 1) * 3];
      i64 mn[3], mx[3], vlo[3], vhi[3];
      for (int c = 0; c < 3; ++c) {
        mn[c] = std::min(A[c], B[c]) - rho;
        mx[c] = std::max(A[c], B[c]) + rho;
      }
      candidate_range(mn, mx, L.s, rg, vlo, vhi);
      for (i64 z = vlo[2]; z <= vhi[2]; ++z)
        for (i64 y = vlo[1]; y <= vhi[1]; ++y)
          for (i64 x = vlo[0]; x <= vhi[0]; ++x) {
            i64 lo[3] = {x * L.s, y * L.s, z * L.s};
            i64 c[3], d[3];
            for (int k = 0; k < 3; ++k) { c[k] = A[k] - lo[k]; d[k] = B[k] - A[k]; }
            if (!cap_touch(c, d, L.s, rho)) continue;
            parts[t].push_back({morton(x, y, z, L.log2R), i, seg_length(c, d, L.s)});
          }
    }
  });
  return OK;
}

struct PairList {
  std::vector<u64> keys;
  std::vector<i64> prim;
};
}  // namespace

extern "C" {

// Voxelize fibers: pts[m][3] polylines with CSR offsets[F+1]; segment (i, i+1) exists when
// both points belong to the same fiber, and its primitive id is i.  radius in world units.
void* vxo_voxelize_fibers(const double* bmin, double extent, int log2R, const float* pts, i64 m,
                          const i64* offsets, i64 F, double radius, const i64* region, int nthreads,
                          int* status) {
  std::vector<std::vector<Pair>> parts;
  std::vector<double> M;
  *status = fiber_pairs(bmin, extent, log2R, pts, m, offsets, F, radius, region, nthreads, parts, M);
  if (*status) return nullptr;
  return reduce_pairs(parts, M);
}

// The touching (segment, voxel) pairs themselves, for the fit oracle.
void* vxo_voxelize_fibers_pairs(const double* bmin, double extent, int log2R, const float* pts, i64 m,
                                const i64* offsets, i64 F, double radius, int nthreads, int* status) {
  std::vector<std::vector<Pair>> parts;
  std::vector<double> M;
  *status = fiber_pairs(bmin, extent, log2R, pts, m, offsets, F, radius, nullptr, nthreads, parts, M);
  if (*status) return nullptr;
  PairList* r = new PairList;
  for (auto& part : parts)
    for (const Pair& p : part) {
      r->keys.push_back(p.key);
      r->prim.push_back(p.prim);
    }
  return r;
}
i64 vxo_pairs_size(void* r) { return i64(static_cast<PairList*>(r)->keys.size()); }
void vxo_pairs_copy(void* rp, u64* keys, i64* prim) {
  PairList* r = static_cast<PairList*>(rp);
  std::memcpy(keys, r->keys.data(), r->keys.size() * sizeof(u64));
  std::memcpy(prim, r->prim.data(), r->prim.size() * sizeof(i64));
}
void vxo_pairs_free(void* r) { delete static_cast<PairList*>(r); }

i64 vxo_result_size(void* r) { return i64(static_cast<Result*>(r)->keys.size()); }
i64 vxo_result_npairs(void* r) { return static_cast<Result*>(r)->n_pairs; }
void vxo_result_copy(void* rp, u64* keys, uint32_t* count, double* w, double* S) {
  Result* r = static_cast<Result*>(rp);
  size_t n = r->keys.size();
  std::memcpy(keys, r->keys.data(), n * sizeof(u64));
  std::memcpy(count, r->count.data(), n * sizeof(uint32_t));
  std::memcpy(w, r->w.data(), n * sizeof(double));
  std::memcpy(S, r->S.data(), n * 6 * sizeof(double));
}
void vxo_result_free(void* r) { delete static_cast<Result*>(r); }

// ---------------------------------------------------------------------------------------------
// Sec. 4.4 lobe merging, deterministic reading.
// Distance between two normalised lobes A = S_a / w_a, B = S_b / w_b, Delta = A - B:
//   D = 2 tr(Delta^2) + (tr Delta)^2 = (15 / 4 pi) * integral over the sphere of (w^T Delta w)^2,
// i.e. the L2 distance between their projected-area-squared functions.  Ward's agglomerative
// rule merges the pair with the least w_a w_b / (w_a + w_b) * D (ties to the smallest (a, b)),
// until K clusters remain; then `iters` weighted Lloyd passes: each input lobe joins the
// centroid (S / w) nearest in D (ties to the lowest index), centroids are recomputed as
// sum S / sum w, empty clusters are dropped.  Output lobes sorted by descending weight.
// ---------------------------------------------------------------------------------------------
namespace {
double lobe_dist(const double* A, const double* B) {
  double d[6];
  for (int c = 0; c < 6; ++c) d[c] = A[c] - B[c];
  double tr = d[0] + d[1] + d[2];
  double tr2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 2.0 * (d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
  return 2.0 * tr2 + tr * tr;
}
}  // namespace

double vxo_lobe_dist(const double* A, const double* B) { return lobe_dist(A, B); }

// One level: parent p gathers child voxels [cstart[p], cstart[p+1]) of the level below, each
// with cnl[c] lobes (cw[c*Kc + k], cS[(c*Kc + k)*6 + j]).  Writes pnl[p] <= K lobes to
// pw[p*K + k], pS[(p*K + k)*6 + j].  gap_rel[p] / gap_abs[p]: the smallest margin of any
// discrete decision taken for p (relative to the runner-up, and relative to p's weight);
// +inf when no decision was needed.
void vxo_cluster_level(i64 n_par, const i64* cstart, const int32_t* cnl, const double* cw, const double* cS,
                       int Kc, int K, int iters, int32_t* pnl, double* pw, double* pS, double* gap_rel,
                       double* gap_abs, int nthreads) {
  parallel_for(n_par, nthreads, [&](int, i64 a, i64 b) {
    std::vector<double> lw, lS;
    for (i64 p = a; p < b; ++p) {
      lw.clear(); lS.clear();
      for (i64 c = cstart[p]; c < cstart[p + 1]; ++c)
        for (int k = 0; k < cnl[c]; ++k) {
          double w = cw[size_t(c) * Kc + k];
          if (!(w > 0)) continue;
          lw.push_back(w);
          for (int j = 0; j < 6; ++j) lS.push_back(cS[(size_t(c) * Kc + k) * 6 + j]);
        }
      int n = int(lw.size());
      double W = 0;
      for (double w : lw) W += w;
      double grel = INFINITY, gabs = INFINITY;
      std::vector<double> cwv(lw), cSv(lS);          // clusters: weight and summed S
      std::vector<int> order;
      if (n > K) {
        // Ward agglomeration
        while (int(cwv.size()) > K) {
          int m = int(cwv.size());
          double best = INFINITY, second = INFINITY;
          int bi = -1, bj = -1;
          for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) {
              double Ai[6], Aj[6];
              for (int c = 0; c < 6; ++c) { Ai[c] = cSv[i * 6 + c] / cwv[i]; Aj[c] = cSv[j * 6 + c] / cwv[j]; }
              double cost = cwv[i] * cwv[j] / (cwv[i] + cwv[j]) * lobe_dist(Ai, Aj);
              if (cost < best) { second = best; best = cost; bi = i; bj = j; }
              else if (cost < second) second = cost;
            }
          if (second < INFINITY) {
            grel = std::min(grel, second > 0 ? (second - best) / second : 0.0);
            gabs = std::min(gabs, (second - best) / W);
          }
          cwv[bi] += cwv[bj];
          for (int c = 0; c < 6; ++c) cSv[bi * 6 + c] += cSv[bj * 6 + c];
          cwv.erase(cwv.begin() + bj);
          cSv.erase(cSv.begin() + bj * 6, cSv.begin() + bj * 6 + 6);
        }
        // weighted Lloyd passes over the original lobes
        for (int it = 0; it < iters; ++it) {
          int k = int(cwv.size());
          std::vector<double> cent(size_t(k) * 6);
          for (int i = 0; i < k; ++i)
            for (int c = 0; c < 6; ++c) cent[i * 6 + c] = cSv[i * 6 + c] / cwv[i];
          std::vector<double> nw(k, 0.0), nS(size_t(k) * 6, 0.0);
          for (int l = 0; l < n; ++l) {
            double A[6];
            for (int c = 0; c < 6; ++c) A[c] = lS[l * 6 + c] / lw[l];
            double best = INFINITY, second = INFINITY;
            int bi = -1;
            for (int i = 0; i < k; ++i) {
              double d = lobe_dist(A, &cent[i * 6]);
              if (d < best) { second = best; best = d; bi = i; }
              else if (d < second) second = d;
            }
            if (second < INFINITY) {
              grel = std::min(grel, second > 0 ? (second - best) / second : 0.0);
              gabs = std::min(gabs, lw[l] * (second - best) / W);
            }
            nw[bi] += lw[l];
            for (int c = 0; c < 6; ++c) nS[bi * 6 + c] += lS[l * 6 + c];
          }
          cwv.clear(); cSv.clear();
          for (int i = 0; i < k; ++i) {
            if (!(nw[i] > 0)) continue;
            cwv.push_back(nw[i]);
            for (int c = 0; c < 6; ++c) cSv.push_back(nS[i * 6 + c]);
          }
        }
      }
      int k = int(cwv.size());
      order.resize(k);
      for (int i = 0; i < k; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cwv[x] > cwv[y]; });
      pnl[p] = k;
      for (int i = 0; i < K; ++i) {
        pw[size_t(p) * K + i] = i < k ? cwv[order[i]] : 0.0;
        for (int c = 0; c < 6; ++c) pS[(size_t(p) * K + i) * 6 + c] = i < k ? cSv[order[i] * 6 + c] : 0.0;
      }
      gap_rel[p] = grel;
      gap_abs[p] = gabs;
    }
  });
}

}  // extern "C"
