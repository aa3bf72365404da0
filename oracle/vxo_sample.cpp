// vxo_sample.cpp -- FP64 oracle of the paper's sampling voxelizer (TEST INFRASTRUCTURE ONLY).
//
// Sec. 3.2 (sparse data sampling) generates points on the primitives from kernel indices
// instead of random numbers and stores each in the voxel that contains it:
//   * fibers: every segment between control points i and i+1 is the uniform Catmull-Rom span
//     through points i-1, i, i+1, i+2 (the end points repeated at a fiber's ends), evaluated at
//     t = j / m (j = 0..m) and joined by chords; each chord carries n equally spaced samples at
//     fractions (k + 1/2) / n, each weighing chord length / n, oriented along the chord
//     (moment I - t t^T);
//   * triangles: a triangle of area A receives n_T = max(1, floor(N A / A_max)) samples (the
//     count weighted by the area relative to the largest triangle), sample k at
//     (u1, u2) = ((k + 1/2) / n_T, radical inverse of k in base 2) mapped to barycentric
//     coordinates by Heitz's low-distortion triangle map (the mapped point b0 P0 + b1 P1 +
//     (1 - b0 - b1) P2), each weighing A / n_T with the triangle's normal (moment n n^T).
// Every voxel then holds the number of its samples, their summed weight and their summed
// moments.  Positions are computed in grid units, g = (P - bmin) R / extent, in FP64 with the
// operation order spelled out (contraction off, explicit fused multiply-adds), so the voxel of
// every sample is a well-defined function of the inputs; the floor of n_T's bound is decided by
// comparing squares (no square root decides an integer).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

typedef long long i64;
typedef unsigned long long u64;

namespace {

u64 spread3(u64 v) {
  u64 r = 0;
  for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
  return r;
}
u64 morton(i64 x, i64 y, i64 z) { return spread3(u64(x)) | (spread3(u64(y)) << 1) | (spread3(u64(z)) << 2); }

struct Sample {
  u64 key;
  double w;
  double M[6];   // xx yy zz xy xz yz
};

struct SampleResult {
  std::vector<u64> keys;
  std::vector<uint32_t> count;
  std::vector<double> w, S;
  i64 n_samples = 0;
};

// the voxel of grid point g, or false when it lies outside [0, R)^3
bool voxel_of(const double g[3], i64 R, u64& key) {
  i64 v[3];
  for (int a = 0; a < 3; ++a) {
    const double f = std::floor(g[a]);
    if (!(f >= 0.0 && f < double(R))) return false;
    v[a] = i64(f);
  }
  key = morton(v[0], v[1], v[2]);
  return true;
}

void to_grid(const float* p, const double* bmin, double vs, double g[3]) {
  for (int a = 0; a < 3; ++a) g[a] = (double(p[a]) - bmin[a]) * vs;
}

// bit-reversed k as a fraction of 2^32 (exact)
double radical_inverse2(uint32_t k) {
  uint32_t r = 0;
  for (int b = 0; b < 32; ++b) r |= ((k >> b) & 1u) << (31 - b);
  return double(r) * 0x1p-32;
}

SampleResult* aggregate(std::vector<Sample>& smp) {
  std::vector<i64> order(smp.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](i64 a, i64 b) { return smp[a].key < smp[b].key; });
  auto* r = new SampleResult;
  r->n_samples = i64(smp.size());
  for (i64 idx : order) {
    const Sample& s = smp[idx];
    if (r->keys.empty() || r->keys.back() != s.key) {
      r->keys.push_back(s.key);
      r->count.push_back(0);
      r->w.push_back(0.0);
      for (int t = 0; t < 6; ++t) r->S.push_back(0.0);
    }
    const size_t v = r->keys.size() - 1;
    r->count[v] += 1;
    r->w[v] += s.w;
    for (int t = 0; t < 6; ++t) r->S[6 * v + t] += s.w * s.M[t];
  }
  return r;
}

}  // namespace

extern "C" {

// fibers: pts float [m][3], offsets [F + 1]; sub = m chords per segment, per = n samples per chord
void* vxo_sample_fibers(const double* bmin, double extent, int log2R, const float* pts, i64 n_pts,
                        const i64* offsets, i64 F, int sub, int per, int* status) {
  *status = 0;
  if (sub < 1 || per < 1) { *status = 1; return nullptr; }
  const i64 R = i64(1) << log2R;
  const double vs = std::ldexp(1.0, log2R) / extent;
  std::vector<Sample> smp;
  for (i64 f = 0; f < F; ++f) {
    const i64 a = offsets[f], b = offsets[f + 1];
    for (i64 i = a; i + 1 < b; ++i) {
      double P[4][3];
      to_grid(pts + 3 * (i > a ? i - 1 : i), bmin, vs, P[0]);
      to_grid(pts + 3 * i, bmin, vs, P[1]);
      to_grid(pts + 3 * (i + 1), bmin, vs, P[2]);
      to_grid(pts + 3 * (i + 2 < b ? i + 2 : i + 1), bmin, vs, P[3]);
      double c0[3], c1[3], c2[3], c3[3];
      for (int x = 0; x < 3; ++x) {
        c0[x] = P[1][x];
        c1[x] = 0.5 * (P[2][x] - P[0][x]);
        c2[x] = ((P[0][x] - 2.5 * P[1][x]) + 2.0 * P[2][x]) - 0.5 * P[3][x];
        c3[x] = 0.5 * (P[3][x] - P[0][x]) + 1.5 * (P[1][x] - P[2][x]);
      }
      auto curve = [&](double t, double out[3]) {
        for (int x = 0; x < 3; ++x) out[x] = std::fma(std::fma(std::fma(c3[x], t, c2[x]), t, c1[x]), t, c0[x]);
      };
      for (int j = 0; j < sub; ++j) {
        double A[3], B[3], d[3];
        curve(double(j) / double(sub), A);
        curve(double(j + 1) / double(sub), B);
        for (int x = 0; x < 3; ++x) d[x] = B[x] - A[x];
        const double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double M[6] = {0, 0, 0, 0, 0, 0};
        if (len > 0.0) {
          const double t[3] = {d[0] / len, d[1] / len, d[2] / len};
          M[0] = 1.0 - t[0] * t[0]; M[1] = 1.0 - t[1] * t[1]; M[2] = 1.0 - t[2] * t[2];
          M[3] = -t[0] * t[1]; M[4] = -t[0] * t[2]; M[5] = -t[1] * t[2];
        }
        for (int k = 0; k < per; ++k) {
          const double fr = (double(k) + 0.5) / double(per);
          double X[3];
          for (int x = 0; x < 3; ++x) X[x] = std::fma(fr, d[x], A[x]);
          Sample s;
          if (!voxel_of(X, R, s.key)) continue;
          s.w = len / double(per);
          std::memcpy(s.M, M, sizeof M);
          smp.push_back(s);
        }
      }
    }
  }
  return aggregate(smp);
}

// samples of triangle t: n_T = max(1, floor(N A_t / A_max)), decided on squared areas
static i64 tri_samples(double q, double qmax, int N) {
  if (!(qmax > 0.0)) return 1;
  const double nn = double(N) * double(N) * q;
  i64 k = i64(std::floor(double(N) * std::sqrt(q / qmax)));
  if (k < 0) k = 0;
  while (double(k + 1) * double(k + 1) * qmax <= nn) ++k;
  while (k > 0 && double(k) * double(k) * qmax > nn) --k;
  return k > 1 ? k : 1;
}

// twice the area vector of a triangle in grid units (no fused operations)
static void tri_cross(const double g0[3], const double g1[3], const double g2[3], double c[3]) {
  double e0[3], e1[3];
  for (int x = 0; x < 3; ++x) { e0[x] = g1[x] - g0[x]; e1[x] = g2[x] - g0[x]; }
  c[0] = e0[1] * e1[2] - e0[2] * e1[1];
  c[1] = e0[2] * e1[0] - e0[0] * e1[2];
  c[2] = e0[0] * e1[1] - e0[1] * e1[0];
}

void* vxo_sample_triangles(const double* bmin, double extent, int log2R, const float* tris, i64 n, int N,
                           int* status) {
  *status = 0;
  if (N < 1) { *status = 1; return nullptr; }
  const i64 R = i64(1) << log2R;
  const double vs = std::ldexp(1.0, log2R) / extent;
  std::vector<double> q(n);
  double qmax = 0.0;
  for (i64 t = 0; t < n; ++t) {
    double g[3][3], c[3];
    for (int v = 0; v < 3; ++v) to_grid(tris + 9 * t + 3 * v, bmin, vs, g[v]);
    tri_cross(g[0], g[1], g[2], c);
    q[t] = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    qmax = std::max(qmax, q[t]);
  }
  std::vector<Sample> smp;
  for (i64 t = 0; t < n; ++t) {
    double g[3][3], c[3];
    for (int v = 0; v < 3; ++v) to_grid(tris + 9 * t + 3 * v, bmin, vs, g[v]);
    tri_cross(g[0], g[1], g[2], c);
    const i64 nt = tri_samples(q[t], qmax, N);
    const double A2 = std::sqrt(q[t]);
    double M[6] = {0, 0, 0, 0, 0, 0};
    if (A2 > 0.0) {
      const double nn[3] = {c[0] / A2, c[1] / A2, c[2] / A2};
      M[0] = nn[0] * nn[0]; M[1] = nn[1] * nn[1]; M[2] = nn[2] * nn[2];
      M[3] = nn[0] * nn[1]; M[4] = nn[0] * nn[2]; M[5] = nn[1] * nn[2];
    }
    double d0[3], d1[3];
    for (int x = 0; x < 3; ++x) { d0[x] = g[0][x] - g[2][x]; d1[x] = g[1][x] - g[2][x]; }
    for (i64 k = 0; k < nt; ++k) {
      const double u1 = (double(k) + 0.5) / double(nt);
      const double u2 = radical_inverse2(uint32_t(k));
      double b0, b1;
      if (u2 > u1) { b0 = 0.5 * u1; b1 = u2 - b0; }
      else { b1 = 0.5 * u2; b0 = u1 - b1; }
      double X[3];
      for (int x = 0; x < 3; ++x) X[x] = std::fma(b0, d0[x], std::fma(b1, d1[x], g[2][x]));
      Sample s;
      if (!voxel_of(X, R, s.key)) continue;
      s.w = 0.5 * A2 / double(nt);
      std::memcpy(s.M, M, sizeof M);
      smp.push_back(s);
    }
  }
  return aggregate(smp);
}

i64 vxo_sresult_size(void* r) { return i64(static_cast<SampleResult*>(r)->keys.size()); }
i64 vxo_sresult_nsamples(void* r) { return static_cast<SampleResult*>(r)->n_samples; }
void vxo_sresult_copy(void* rp, u64* keys, uint32_t* count, double* w, double* S) {
  auto* r = static_cast<SampleResult*>(rp);
  std::memcpy(keys, r->keys.data(), r->keys.size() * sizeof(u64));
  std::memcpy(count, r->count.data(), r->count.size() * sizeof(uint32_t));
  std::memcpy(w, r->w.data(), r->w.size() * sizeof(double));
  std::memcpy(S, r->S.data(), r->S.size() * sizeof(double));
}
void vxo_sresult_free(void* r) { delete static_cast<SampleResult*>(r); }

// Heitz's map and the sample counts on their own, for the pins
void vxo_heitz_map(double u1, double u2, double* b) {
  if (u2 > u1) { b[0] = 0.5 * u1; b[1] = u2 - b[0]; }
  else { b[1] = 0.5 * u2; b[0] = u1 - b[1]; }
}
i64 vxo_tri_sample_count(double q, double qmax, int N) { return tri_samples(q, qmax, N); }

}  // extern "C"
