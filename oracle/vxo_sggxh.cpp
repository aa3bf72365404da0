// vxo_sggxh.cpp -- FP64 oracle of the paper's SGGX-H lobe reduction (TEST INFRASTRUCTURE ONLY).
//
// Sec. 4.4 compares lobes through histograms of samples drawn from them (N = 5000 samples per
// lobe, 5 bins per dimension) under a Wasserstein distance, repeatedly merges the two closest
// lobes by pooling their samples, and stops at the lobe cap.  The readings taken here:
//   * a lobe (w, S) is the SGGX of S / w, floored by 1e-3 of its trace on the diagonal (the
//     paper's small uniform deviation for near-degenerate lobes); its distribution of normals is
//     that of the ellipsoid x^T S x = 1: with S = L L^T (Cholesky) and u uniform on the sphere,
//     the point L^-T u has normal L u and its area element is proportional to |L u|, so a
//     sample is n = L u / |L u| with u accepted with probability |L u| / sqrt(tr S);
//   * uniform points on the sphere by rejection from the cube [-1, 1]^3 (u = v / |v|, |v| <= 1),
//     acceptance U^2 tr(S) |v|^2 <= |L v|^2, so only +, *, / and square roots (correctly rounded
//     in IEEE double) decide a sample's bin;
//   * random numbers: counter-based SplitMix64 (Steele, Lea, Flood 2014): draw d of sample k of
//     stream `key` is the SplitMix64 output number (k 2^32 + d) of seed `key`; a lobe's stream is
//     keyed by its level, its voxel's Morton key and its slot among the voxel's input lobes;
//   * histogram: bin floor((n_a + 1) * 2.5) in [0, 4] per axis, counts of N accepted samples;
//   * distance: the Wasserstein-1 distance between the histograms' marginals along x, y and z,
//     summed (bin width 0.4): for lobes holding m_i, m_j pooled sample sets of N samples,
//         W = 0.4 / N * sum_axis sum_b |C_i(b) m_j - C_j(b) m_i| / (m_i m_j)
//     with C the cumulative counts of bins 0..b (b < 4); compared exactly in integers;
//   * merge: the closest pair (ties to the lowest (i, j) in slot order), w and S added, the
//     counts pooled; repeat while more than K lobes remain; lobes sorted by descending weight.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

typedef long long i64;
typedef unsigned long long u64;

namespace {

const u64 kGamma = 0x9E3779B97F4A7C15ull;

u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// SplitMix64 output number c of seed `key`: the state advanced c + 1 times, then mixed
u64 splitmix_at(u64 key, u64 c) { return mix64(key + kGamma * (c + 1)); }

u64 draw(u64 key, u64 k, u64 d) { return splitmix_at(key, (k << 32) | d); }

double unit(u64 x) { return double(x >> 11) * 0x1p-53; }

u64 lobe_key(int level, u64 voxel_key, int slot) {
  return mix64(mix64(voxel_key + kGamma * u64(level + 1)) + kGamma * u64(slot + 1));
}

const int kMaxAttempts = 10000;

// N samples of the lobe (w, S): emit(n) for each accepted unit normal n, in sample order
template <class Emit>
void sample_lobe(const double* S, double w, u64 key, int N, Emit&& emit) {
  double a00 = S[0] / w, a11 = S[1] / w, a22 = S[2] / w;
  const double a10 = S[3] / w, a20 = S[4] / w, a21 = S[5] / w;
  const double e = 1e-3 * ((a00 + a11) + a22);
  a00 = a00 + e;
  a11 = a11 + e;
  a22 = a22 + e;
  const double tr = (a00 + a11) + a22;
  const double l00 = std::sqrt(a00);
  const double l10 = a10 / l00, l20 = a20 / l00;
  double d1 = a11 - l10 * l10;
  if (!(d1 > 0.0)) d1 = e;
  const double l11 = std::sqrt(d1);
  const double l21 = (a21 - l20 * l10) / l11;
  double d2 = (a22 - l20 * l20) - l21 * l21;
  if (!(d2 > 0.0)) d2 = e;
  const double l22 = std::sqrt(d2);
  for (int k = 0; k < N; ++k) {
    for (int at = 0; at < kMaxAttempts; ++at) {
      const u64 d = 4 * u64(at);
      const double x = 2.0 * unit(draw(key, k, d)) - 1.0;
      const double y = 2.0 * unit(draw(key, k, d + 1)) - 1.0;
      const double z = 2.0 * unit(draw(key, k, d + 2)) - 1.0;
      const double r2 = (x * x + y * y) + z * z;
      if (r2 > 1.0 || r2 == 0.0) continue;
      const double p0 = l00 * x;
      const double p1 = l10 * x + l11 * y;
      const double p2 = (l20 * x + l21 * y) + l22 * z;
      const double q = (p0 * p0 + p1 * p1) + p2 * p2;
      const double U = unit(draw(key, k, d + 3));
      if (((U * U) * tr) * r2 > q) continue;
      const double len = std::sqrt(q);
      emit(p0 / len, p1 / len, p2 / len);
      break;
    }
  }
}

// counts[125] (bin x * 25 + y * 5 + z) of N samples of the lobe (w, S)
void lobe_hist(const double* S, double w, u64 key, int N, int32_t* counts) {
  std::fill(counts, counts + 125, 0);
  sample_lobe(S, w, key, N, [&](double n0, double n1, double n2) {
    const double n[3] = {n0, n1, n2};
    int b[3];
    for (int c = 0; c < 3; ++c) {
      const double f = std::floor((n[c] + 1.0) * 2.5);
      b[c] = !(f >= 0.0) ? 0 : (f > 4.0 ? 4 : int(f));     // a non-finite lobe lands in bin 0
    }
    counts[b[0] * 25 + b[1] * 5 + b[2]] += 1;
  });
}

struct Lobe {
  double w;
  double S[6];
  i64 m;           // pooled sample sets
  i64 C[3][4];     // cumulative marginal counts
  bool on;
};

void marginals(const int32_t* h, i64 C[3][4]) {
  i64 mg[3][5] = {};
  for (int x = 0; x < 5; ++x)
    for (int y = 0; y < 5; ++y)
      for (int z = 0; z < 5; ++z) {
        const i64 c = h[x * 25 + y * 5 + z];
        mg[0][x] += c;
        mg[1][y] += c;
        mg[2][z] += c;
      }
  for (int a = 0; a < 3; ++a) {
    i64 run = 0;
    for (int b = 0; b < 4; ++b) {
      run += mg[a][b];
      C[a][b] = run;
    }
  }
}

i64 pair_num(const Lobe& A, const Lobe& B) {
  i64 s = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 4; ++b) s += std::llabs(A.C[a][b] * B.m - B.C[a][b] * A.m);
  return s;
}

// Merge to at most K lobes.  Returns the surviving slots sorted by descending weight (ties in
// slot order); owner[i] is the slot input i was merged into.
std::vector<int> reduce(std::vector<Lobe>& L, int K, std::vector<int>& owner) {
  const int n = int(L.size());
  owner.resize(n);
  std::iota(owner.begin(), owner.end(), 0);
  int active = n;
  while (active > K) {
    int bi = -1, bj = -1;
    i64 bn = 0, bd = 1;
    for (int i = 0; i < n; ++i) {
      if (!L[i].on) continue;
      for (int j = i + 1; j < n; ++j) {
        if (!L[j].on) continue;
        const i64 nn = pair_num(L[i], L[j]), dd = L[i].m * L[j].m;
        if (bi < 0 || nn * bd < bn * dd) {     // strictly closer: ties keep the first pair
          bi = i;
          bj = j;
          bn = nn;
          bd = dd;
        }
      }
    }
    Lobe& A = L[bi];
    const Lobe& B = L[bj];
    A.w += B.w;
    for (int c = 0; c < 6; ++c) A.S[c] += B.S[c];
    A.m += B.m;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 4; ++b) A.C[a][b] += B.C[a][b];
    L[bj].on = false;
    for (int& o : owner)
      if (o == bj) o = bi;
    --active;
  }
  std::vector<int> order;
  for (int i = 0; i < n; ++i)
    if (L[i].on) order.push_back(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return L[a].w > L[b].w; });
  return order;
}

}  // namespace

extern "C" {

u64 vxo_splitmix_at(u64 key, u64 c) { return splitmix_at(key, c); }
u64 vxo_sggxh_lobe_key(int level, u64 voxel_key, int slot) { return lobe_key(level, voxel_key, slot); }

void vxo_sggxh_hist(const double* S, double w, u64 key, int N, int32_t* counts) { lobe_hist(S, w, key, N, counts); }

// the accepted normals themselves, out [N][3] (fewer when a sample ran out of attempts; returns
// how many)
int vxo_sggxh_samples(const double* S, double w, u64 key, int N, double* out) {
  int m = 0;
  sample_lobe(S, w, key, N, [&](double n0, double n1, double n2) {
    out[3 * m] = n0;
    out[3 * m + 1] = n1;
    out[3 * m + 2] = n2;
    ++m;
  });
  return m;
}

// Reduce given histograms (n lobes, counts [n][125] of N samples each) to K lobes: out_nl, out_w
// [K], out_S [K][6], out_of [n] = the output lobe each input went to
void vxo_sggxh_reduce(int n, const double* w, const double* S, const int32_t* counts, int K, int* out_nl,
                      double* out_w, double* out_S, int* out_of) {
  std::vector<Lobe> L(n);
  for (int i = 0; i < n; ++i) {
    L[i].w = w[i];
    std::memcpy(L[i].S, S + 6 * i, sizeof L[i].S);
    L[i].m = 1;
    marginals(counts + 125 * i, L[i].C);
    L[i].on = true;
  }
  std::vector<int> owner;
  const std::vector<int> order = reduce(L, K, owner);
  *out_nl = int(order.size());
  for (int o = 0; o < int(order.size()); ++o) {
    out_w[o] = L[order[o]].w;
    std::memcpy(out_S + 6 * o, L[order[o]].S, 6 * sizeof(double));
    for (int i = 0; i < n; ++i)
      if (owner[i] == order[o]) out_of[i] = o;
  }
}

// One level: parent p gathers the lobes of its children cstart[p] .. cstart[p+1]-1 (child c has
// cnl[c] lobes, cw [c][Kc], cS [c][Kc][6]), drops those of zero weight, samples the rest (stream
// keyed by level, pkeys[p] and the slot) and reduces them to K.  Outputs as for the reduce.
void vxo_sggxh_level(i64 n_par, const u64* pkeys, const i64* cstart, const int32_t* cnl, const double* cw,
                     const double* cS, int Kc, int level, int K, int N, int32_t* out_nl, double* out_w,
                     double* out_S) {
  std::vector<int32_t> h(125);
  for (i64 p = 0; p < n_par; ++p) {
    std::vector<Lobe> L;
    for (i64 c = cstart[p]; c < cstart[p + 1]; ++c)
      for (int k = 0; k < cnl[c]; ++k) {
        const double w = cw[c * Kc + k];
        if (!(w > 0.0)) continue;
        Lobe l;
        l.w = w;
        std::memcpy(l.S, cS + (c * Kc + k) * 6, sizeof l.S);
        l.m = 1;
        lobe_hist(l.S, w, lobe_key(level, pkeys[p], int(L.size())), N, h.data());
        marginals(h.data(), l.C);
        l.on = true;
        L.push_back(l);
      }
    std::vector<int> owner;
    const std::vector<int> order = reduce(L, K, owner);    // at or under the cap: only sorted
    out_nl[p] = int32_t(order.size());
    for (int o = 0; o < K; ++o) {
      const bool v = o < int(order.size());
      out_w[p * K + o] = v ? L[order[o]].w : 0.0;
      for (int c = 0; c < 6; ++c) out_S[(p * K + o) * 6 + c] = v ? L[order[o]].S[c] : 0.0;
    }
  }
}

}  // extern "C"
