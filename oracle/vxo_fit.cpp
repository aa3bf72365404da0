// vxo_fit.cpp -- FP64 oracle of the differentiable lobe fit (TEST INFRASTRUCTURE ONLY).
//
// Fit at pyramid levels lo..hi: every voxel u with w_u > 0 gets two lobes given by lower
// triangular matrices L_1, L_2 (6 parameters each, row-major lower triangle
// L00 L10 L11 L20 L21 L22), whose projected area in direction omega is
// f_u(omega) = |L_1^T omega| + |L_2^T omega|.  The target is the projected area of u's
// children (Sec. 4.1: sigma(omega) = sqrt(omega^T S omega) for an SGGX S), weighted by their
// density: tau_u(omega) = sum_c w_c sqrt(omega^T (S_c / w_c) omega) / sum_c w_c over the
// children c with w_c > 0.  Loss = sum over levels and voxels of the mean over 128 Fibonacci
// directions of (f_u - tau_u)^2.
//
// The pair set (which segment touches which leaf voxel) comes from the exact test on the
// lattice-snapped points `pts_snap`; the weights (clipped centreline lengths) and tangents
// are evaluated in FP64 from the continuous points `pts_cont`, so that the loss is a smooth
// function of them between clip-plane crossings and can be differentiated and checked by
// finite differences.  Gradients: analytic, to every L and to every control point.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

typedef long long i64;
typedef unsigned long long u64;

extern "C" void* vxo_voxelize_fibers_pairs(const double* bmin, double extent, int log2R, const float* pts, i64 m,
                                           const i64* offsets, i64 F, double radius, int nthreads, int* status);
extern "C" i64 vxo_pairs_size(void* r);
extern "C" void vxo_pairs_copy(void* r, u64* keys, i64* prim);
extern "C" void vxo_pairs_free(void* r);

namespace {

constexpr int NDIR = 128;

struct Dirs {
  double w[NDIR][3];
  Dirs() {
    const double ga = M_PI * (3.0 - std::sqrt(5.0));
    for (int k = 0; k < NDIR; ++k) {
      double z = 1.0 - (2.0 * k + 1.0) / NDIR;
      double r = std::sqrt(std::max(0.0, 1.0 - z * z));
      w[k][0] = r * std::cos(k * ga);
      w[k][1] = r * std::sin(k * ga);
      w[k][2] = z;
    }
  }
};

double quad(const double* S, const double* o) {
  return S[0] * o[0] * o[0] + S[1] * o[1] * o[1] + S[2] * o[2] * o[2] +
         2.0 * (S[3] * o[0] * o[1] + S[4] * o[0] * o[2] + S[5] * o[1] * o[2]);
}

// y = L^T omega for the lower-triangular parameters l = (L00, L10, L11, L20, L21, L22)
void lt_times(const double* l, const double* o, double y[3]) {
  y[0] = l[0] * o[0] + l[1] * o[1] + l[3] * o[2];
  y[1] = l[2] * o[1] + l[4] * o[2];
  y[2] = l[5] * o[2];
}

// Clipped length of segment (A, B) (voxel units) inside [lo, lo+1)^3 and its gradient.
// Returns the length; gA, gB receive d(length)/dA, d(length)/dB (zero when empty).
double clip_len(const double* A, const double* B, const double* lo, double* gA, double* gB) {
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = B[a] - A[a];
  double t0 = 0.0, t1 = 1.0;
  int e0 = -1, e1 = -1;       // axis fixing the entry / exit parameter (-1: the segment end)
  for (int a = 0; a < 3; ++a) gA[a] = gB[a] = 0.0;     // an empty piece has no gradient
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (!(A[a] >= lo[a] && A[a] < lo[a] + 1.0)) return 0.0;
      continue;
    }
    double ta = (lo[a] - A[a]) / d[a], tb = (lo[a] + 1.0 - A[a]) / d[a];
    double tin = std::min(ta, tb), tout = std::max(ta, tb);
    if (tin > t0) { t0 = tin; e0 = a; }
    if (tout < t1) { t1 = tout; e1 = a; }
  }
  if (!(t1 > t0)) return 0.0;
  double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double u[3] = {d[0] / len, d[1] / len, d[2] / len};
  // length = u . (B' - A'), B' = A + t1 d, A' = A + t0 d; a clipped end moves inside its plane:
  // d(end) = P (moving point), P = I - d e^T / d_e for a plane end, identity for a segment end.
  // moving point of A' = (1 - t0) dA + t0 dB, of B' = (1 - t1) dA + t1 dB.
  auto proj_u = [&](int e, double v[3]) {        // u^T P as a row vector
    if (e < 0) { for (int a = 0; a < 3; ++a) v[a] = u[a]; return; }
    for (int a = 0; a < 3; ++a) v[a] = u[a];
    v[e] -= len / d[e];                            // u . d / d_e = len / d_e
  };
  double pe[3], ps[3];
  proj_u(e1, pe);
  proj_u(e0, ps);
  for (int a = 0; a < 3; ++a) {
    gA[a] = pe[a] * (1.0 - t1) - ps[a] * (1.0 - t0);
    gB[a] = pe[a] * t1 - ps[a] * t0;
  }
  return (t1 - t0) * len;
}

struct FitProblem {
  // pyramid (FP64) levels 0..hi
  std::vector<std::vector<u64>> keys;
  std::vector<std::vector<double>> w;        // [n]
  std::vector<std::vector<double>> S;        // [n][6]
  std::vector<std::vector<i64>> cstart;      // level L>=1: children [cstart[u], cstart[u+1]) in level L-1
};

int find_key(const std::vector<u64>& k, u64 key) {
  auto it = std::lower_bound(k.begin(), k.end(), key);
  if (it == k.end() || *it != key) return -1;
  return int(it - k.begin());
}

}  // namespace

extern "C" {

// Evaluate the fit loss and its analytic gradient.
//   pts_snap: float [m][3] (pair set), pts_cont: double [m][3] (weights, tangents), world units
//   L_all: double, for levels lo..hi in order, [n_L][12]; the caller sizes it from the pyramid
//          of the pair set (vxo_fit_levels gives n_L).
//   loss_vox: double, per voxel of levels lo..hi (same layout as L_all / 12), may be NULL
//   dL: double like L_all, may be NULL;  dpts: double [m][3] (world units), may be NULL
//   dirs: double [128][3], the direction set, or NULL for the Fibonacci set in FP64
// Returns the total loss; *status = 0 on success.
double vxo_fit_eval(const double* bmin, double extent, int log2R, const float* pts_snap, const double* pts_cont,
                    i64 m, const i64* offsets, i64 F, double radius, int lo, int hi, const double* L_all,
                    double* loss_vox, double* dL, double* dpts, const double* dirs, int nthreads, int* status) {
  *status = 0;
  void* pr = vxo_voxelize_fibers_pairs(bmin, extent, log2R, pts_snap, m, offsets, F, radius, nthreads, status);
  if (*status) return 0.0;
  i64 np = vxo_pairs_size(pr);
  std::vector<u64> pk(np);
  std::vector<i64> pp(np);
  vxo_pairs_copy(pr, pk.data(), pp.data());
  vxo_pairs_free(pr);
  const double vs = double(i64(1) << log2R) / extent;     // voxel units per world unit
  auto vox = [&](i64 i, int a) { return (pts_cont[3 * i + a] - bmin[a]) * vs; };
  // leaf sums from the continuous geometry
  FitProblem P;
  P.keys.resize(hi + 1);
  P.w.resize(hi + 1);
  P.S.resize(hi + 1);
  P.cstart.resize(hi + 1);
  std::vector<double> pw(np), pM(np * 6);
  std::vector<int> pv(np);
  {
    std::vector<u64> uk(pk);
    std::sort(uk.begin(), uk.end());
    uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
    P.keys[0] = uk;
    P.w[0].assign(uk.size(), 0.0);
    P.S[0].assign(uk.size() * 6, 0.0);
  }
  for (i64 j = 0; j < np; ++j) {
    const i64 i = pp[j];
    double A[3], B[3], lo3[3];
    u64 k = pk[j];
    i64 c[3] = {0, 0, 0};
    for (int b = 0; b < log2R; ++b)
      for (int a = 0; a < 3; ++a) c[a] |= i64((k >> (3 * b + a)) & 1) << b;
    for (int a = 0; a < 3; ++a) { A[a] = vox(i, a); B[a] = vox(i + 1, a); lo3[a] = double(c[a]); }
    double gA[3], gB[3];
    pw[j] = clip_len(A, B, lo3, gA, gB);
    double d[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    double l2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double* M = &pM[j * 6];
    if (l2 > 0) {
      M[0] = 1 - d[0] * d[0] / l2; M[1] = 1 - d[1] * d[1] / l2; M[2] = 1 - d[2] * d[2] / l2;
      M[3] = -d[0] * d[1] / l2; M[4] = -d[0] * d[2] / l2; M[5] = -d[1] * d[2] / l2;
    } else {
      for (int t = 0; t < 6; ++t) M[t] = 0;
    }
    int v = find_key(P.keys[0], k);
    pv[j] = v;
    P.w[0][v] += pw[j];
    for (int t = 0; t < 6; ++t) P.S[0][v * 6 + t] += pw[j] * M[t];
  }
  // pyramid sums
  for (int L = 1; L <= hi; ++L) {
    const auto& ck = P.keys[L - 1];
    auto& K = P.keys[L];
    auto& cs = P.cstart[L];
    for (size_t i = 0; i < ck.size(); ++i) {
      if (i == 0 || (ck[i] >> 3) != (ck[i - 1] >> 3)) {
        K.push_back(ck[i] >> 3);
        cs.push_back(i64(i));
      }
    }
    cs.push_back(i64(ck.size()));
    P.w[L].assign(K.size(), 0.0);
    P.S[L].assign(K.size() * 6, 0.0);
    for (size_t u = 0; u < K.size(); ++u)
      for (i64 c = cs[u]; c < cs[u + 1]; ++c) {
        P.w[L][u] += P.w[L - 1][c];
        for (int t = 0; t < 6; ++t) P.S[L][u * 6 + t] += P.S[L - 1][c * 6 + t];
      }
  }
  // loss and gradients w.r.t. L and w.r.t. the children's (S, w)
  static const Dirs D;
  const double* dir0 = dirs ? dirs : &D.w[0][0];
  std::vector<std::vector<double>> gS(hi + 1), gw(hi + 1);
  for (int L = 0; L <= hi; ++L) {
    gS[L].assign(P.keys[L].size() * 6, 0.0);
    gw[L].assign(P.keys[L].size(), 0.0);
  }
  double total = 0.0;
  i64 off = 0;
  for (int L = lo; L <= hi; ++L) {
    const i64 n = i64(P.keys[L].size());
    for (i64 u = 0; u < n; ++u) {
      const double* lu = L_all + (off + u) * 12;
      double lv = 0.0;
      if (P.w[L][u] > 0) {
        const i64 c0 = P.cstart[L][u], c1 = P.cstart[L][u + 1];
        const double W = P.w[L][u];
        double gl[12] = {0};
        for (int k = 0; k < NDIR; ++k) {
          const double* o = dir0 + 3 * k;
          double tau = 0.0;
          for (i64 c = c0; c < c1; ++c) {
            double wc = P.w[L - 1][c];
            if (!(wc > 0)) continue;
            tau += std::sqrt(std::max(0.0, wc * quad(&P.S[L - 1][c * 6], o)));
          }
          tau /= W;
          double f = 0.0, y[2][3], ny[2];
          for (int j = 0; j < 2; ++j) {
            lt_times(lu + 6 * j, o, y[j]);
            ny[j] = std::sqrt(y[j][0] * y[j][0] + y[j][1] * y[j][1] + y[j][2] * y[j][2]);
            f += ny[j];
          }
          const double r = f - tau;
          lv += r * r / NDIR;
          const double g = 2.0 * r / NDIR;            // d loss / d f ; d loss / d tau = -g
          for (int j = 0; j < 2; ++j) {
            if (!(ny[j] > 0)) continue;
            // d|y|/dL_ab = y_b o_a / |y| for a >= b
            const double* yy = y[j];
            double* gj = gl + 6 * j;
            gj[0] += g * yy[0] * o[0] / ny[j];
            gj[1] += g * yy[0] * o[1] / ny[j];
            gj[2] += g * yy[1] * o[1] / ny[j];
            gj[3] += g * yy[0] * o[2] / ny[j];
            gj[4] += g * yy[1] * o[2] / ny[j];
            gj[5] += g * yy[2] * o[2] / ny[j];
          }
          // tau = sum_c q_c / W, q_c = sqrt(w_c o^T S_c o), W = sum_c w_c
          for (i64 c = c0; c < c1; ++c) {
            double wc = P.w[L - 1][c];
            if (!(wc > 0)) continue;
            double qs = quad(&P.S[L - 1][c * 6], o);
            double q = std::sqrt(std::max(0.0, wc * qs));
            double dtau_dw = -tau / W;
            if (q > 0) {
              double k2 = wc / (2.0 * q * W);      // d tau / d (o^T S_c o)
              double* G = &gS[L - 1][c * 6];
              G[0] += -g * k2 * o[0] * o[0];
              G[1] += -g * k2 * o[1] * o[1];
              G[2] += -g * k2 * o[2] * o[2];
              G[3] += -g * k2 * 2 * o[0] * o[1];
              G[4] += -g * k2 * 2 * o[0] * o[2];
              G[5] += -g * k2 * 2 * o[1] * o[2];
              dtau_dw += qs / (2.0 * q * W);
            }
            gw[L - 1][c] += -g * dtau_dw;
          }
        }
        if (dL)
          for (int t = 0; t < 12; ++t) dL[(off + u) * 12 + t] = gl[t];
      } else if (dL) {
        for (int t = 0; t < 12; ++t) dL[(off + u) * 12 + t] = 0.0;
      }
      if (loss_vox) loss_vox[off + u] = lv;
      total += lv;
    }
    off += n;
  }
  if (dpts) {
    // top-down: a voxel's (S, w) feed every ancestor's sums
    for (int L = hi - 1; L >= 0; --L)
      for (size_t u = 0; u < P.keys[L + 1].size(); ++u)
        for (i64 c = P.cstart[L + 1][u]; c < P.cstart[L + 1][u + 1]; ++c) {
          gw[L][c] += gw[L + 1][u];
          for (int t = 0; t < 6; ++t) gS[L][c * 6 + t] += gS[L + 1][u * 6 + t];
        }
    for (i64 i = 0; i < 3 * m; ++i) dpts[i] = 0.0;
    for (i64 j = 0; j < np; ++j) {
      const i64 i = pp[j];
      const int v = pv[j];
      double A[3], B[3], lo3[3], gA[3], gB[3];
      u64 k = pk[j];
      i64 c[3] = {0, 0, 0};
      for (int b = 0; b < log2R; ++b)
        for (int a = 0; a < 3; ++a) c[a] |= i64((k >> (3 * b + a)) & 1) << b;
      for (int a = 0; a < 3; ++a) { A[a] = vox(i, a); B[a] = vox(i + 1, a); lo3[a] = double(c[a]); }
      const double wl = clip_len(A, B, lo3, gA, gB);
      const double* M = &pM[j * 6];
      const double* G = &gS[0][size_t(v) * 6];
      // d loss / d w_pv
      double gwp = gw[0][v];
      for (int t = 0; t < 6; ++t) gwp += G[t] * M[t];
      // d loss / d M (6-vector), then through t = d / |d| to d = B - A
      double gM[6];
      for (int t = 0; t < 6; ++t) gM[t] = wl * G[t];
      double d[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      double len = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double gd[3] = {0, 0, 0};
      if (len > 0) {
        double t[3] = {d[0] / len, d[1] / len, d[2] / len};
        // M = (1 - tx^2, 1 - ty^2, 1 - tz^2, -tx ty, -tx tz, -ty tz)
        double gt[3];
        gt[0] = -2 * t[0] * gM[0] - t[1] * gM[3] - t[2] * gM[4];
        gt[1] = -2 * t[1] * gM[1] - t[0] * gM[3] - t[2] * gM[5];
        gt[2] = -2 * t[2] * gM[2] - t[0] * gM[4] - t[1] * gM[5];
        double dot = gt[0] * t[0] + gt[1] * t[1] + gt[2] * t[2];
        for (int a = 0; a < 3; ++a) gd[a] = (gt[a] - dot * t[a]) / len;
      }
      for (int a = 0; a < 3; ++a) {
        dpts[3 * i + a] += (gwp * gA[a] - gd[a]) * vs;
        dpts[3 * (i + 1) + a] += (gwp * gB[a] + gd[a]) * vs;
      }
    }
  }
  return total;
}

// Sizes of the pyramid levels 0..hi of the pair set (so the caller can size L_all).
int vxo_fit_levels(const double* bmin, double extent, int log2R, const float* pts_snap, i64 m, const i64* offsets,
                   i64 F, double radius, int hi, i64* n_levels, int nthreads) {
  int status = 0;
  void* pr = vxo_voxelize_fibers_pairs(bmin, extent, log2R, pts_snap, m, offsets, F, radius, nthreads, &status);
  if (status) return status;
  i64 np = vxo_pairs_size(pr);
  std::vector<u64> pk(np);
  std::vector<i64> pp(np);
  vxo_pairs_copy(pr, pk.data(), pp.data());
  vxo_pairs_free(pr);
  std::sort(pk.begin(), pk.end());
  pk.erase(std::unique(pk.begin(), pk.end()), pk.end());
  for (int L = 0; L <= hi; ++L) {
    n_levels[L] = i64(pk.size());
    for (auto& k : pk) k >>= 3;
    pk.erase(std::unique(pk.begin(), pk.end()), pk.end());
  }
  return 0;
}

}  // extern "C"
