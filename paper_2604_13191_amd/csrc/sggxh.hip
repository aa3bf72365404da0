// sggxh.hip -- the paper's SGGX-H lobe reduction (Sec. 4.4) on the GPU.
//
// A coarse voxel gathers the lobes of its children (the leaf's voxel is one lobe), drops those of
// zero weight and, when more than K remain, compares them through histograms of samples drawn
// from their normal distributions and merges the closest pair (pooling the samples) until K are
// left:
//   * lobe (w, S): the SGGX of S / w, its diagonal raised by 1e-3 of its trace; with S = L L^T
//     (Cholesky), a sample is n = L u / |L u| for u uniform on the sphere, accepted with
//     probability |L u| / sqrt(tr S) (the normals of the ellipsoid x^T S x = 1 weighted by area);
//     u from the cube [-1, 1]^3 by rejection, so only correctly rounded IEEE double operations
//     decide a sample's bin;
//   * random numbers: draw d of sample k of a lobe is SplitMix64 output number k 2^32 + d of the
//     lobe's seed, keyed by the level, the voxel's Morton key and the lobe's slot;
//   * histogram: 5 bins per axis, floor((n_a + 1) 2.5); only the three axis marginals are kept
//     (the distance uses nothing else);
//   * distance: Wasserstein-1 between the axis marginals, summed over the axes; for lobes pooling
//     m_i, m_j sample sets it is proportional to sum |C_i(b) m_j - C_j(b) m_i| / (m_i m_j) over
//     the cumulative counts C, compared exactly in 64-bit integers; ties to the first pair in
//     slot order;
//   * merge: w and S added (FP32), counts pooled; the survivors sorted by descending weight.
// One 64-lane block per coarse voxel: the samples of a lobe are spread over the lanes and counted
// with integer LDS atomics (exact, order-free), a lane holds one row of the pair table in a merge
// round, and a wave reduction picks the pair.
#pragma clang fp contract(off)

#include "vx_internal.hpp"

namespace vx {
namespace {

constexpr int kMaxLobes = 64;        // 8 children x K <= 8
constexpr int kMaxAttempts = 10000;
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t k, uint64_t d) {
  return mix64(key + kGamma * (((k << 32) | d) + 1));
}
__device__ __forceinline__ double unit(uint64_t x) { return double(x >> 11) * 0x1p-53; }
__device__ __forceinline__ uint64_t lobe_key(int level, uint64_t voxel_key, int slot) {
  return mix64(mix64(voxel_key + kGamma * uint64_t(level + 1)) + kGamma * uint64_t(slot + 1));
}

struct Chol {
  double l00, l10, l11, l20, l21, l22, tr;
};

// lobe (w, S) with S = (xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ Chol lobe_chol(float wf, float xx, float yy, float zz, float xy, float xz, float yz) {
  const double w = double(wf);
  double a00 = double(xx) / w, a11 = double(yy) / w, a22 = double(zz) / w;
  const double a10 = double(xy) / w, a20 = double(xz) / w, a21 = double(yz) / w;
  const double e = 1e-3 * ((a00 + a11) + a22);
  a00 = a00 + e;
  a11 = a11 + e;
  a22 = a22 + e;
  Chol c;
  c.tr = (a00 + a11) + a22;
  c.l00 = sqrt(a00);
  c.l10 = a10 / c.l00;
  c.l20 = a20 / c.l00;
  double d1 = a11 - c.l10 * c.l10;
  if (!(d1 > 0.0)) d1 = e;
  c.l11 = sqrt(d1);
  c.l21 = (a21 - c.l20 * c.l10) / c.l11;
  double d2 = (a22 - c.l20 * c.l20) - c.l21 * c.l21;
  if (!(d2 > 0.0)) d2 = e;
  c.l22 = sqrt(d2);
  return c;
}

__device__ __forceinline__ int bin_of(double n) {
  const double f = floor((n + 1.0) * 2.5);
  return !(f >= 0.0) ? 0 : (f > 4.0 ? 4 : int(f));
}

// attempt `at` of sample k of the lobe: true (and the three bins) when it is accepted
__device__ __forceinline__ bool lobe_attempt(const Chol& c, uint64_t key, uint64_t k, int at, int b[3]) {
  const uint64_t d = 4 * uint64_t(at);
  const double x = 2.0 * unit(draw(key, k, d)) - 1.0;
  const double y = 2.0 * unit(draw(key, k, d + 1)) - 1.0;
  const double z = 2.0 * unit(draw(key, k, d + 2)) - 1.0;
  const double r2 = (x * x + y * y) + z * z;
  if (r2 > 1.0 || r2 == 0.0) return false;
  const double p0 = c.l00 * x;
  const double p1 = c.l10 * x + c.l11 * y;
  const double p2 = (c.l20 * x + c.l21 * y) + c.l22 * z;
  const double q = (p0 * p0 + p1 * p1) + p2 * p2;
  const double U = unit(draw(key, k, d + 3));
  if (((U * U) * c.tr) * r2 > q) return false;
  const double len = sqrt(q);
  b[0] = bin_of(p0 / len);
  b[1] = bin_of(p1 / len);
  b[2] = bin_of(p2 / len);
  return true;
}

// (num, den, i, j): is a strictly closer than b, or as close and earlier in (i, j) order?
__device__ __forceinline__ bool pair_before(int64_t na, int64_t da, int ia, int ja, int64_t nb, int64_t db, int ib,
                                            int jb) {
  if (ia < 0) return false;
  if (ib < 0) return true;
  const int64_t l = na * db, r = nb * da;
  if (l != r) return l < r;
  return ia < ib || (ia == ib && ja < jb);
}

// Child lobes come from a vx_lobes level (lob != nullptr) or from the leaf (one lobe per voxel).
template <class Key>
__global__ void __launch_bounds__(64) k_sggxh_level(const Key* __restrict__ ckeys, const int64_t* __restrict__ n_child,
                                                    int64_t cmax, const float* __restrict__ leaf_w,
                                                    const float* __restrict__ leaf_S, int64_t leaf_cap,
                                                    vx_lobes clob, int Kc, const Key* __restrict__ pkeys,
                                                    const int64_t* __restrict__ n_par, int64_t pmax, vx_lobes plob,
                                                    int K, int level, int N, int64_t* stats) {
  __shared__ float sw[kMaxLobes];
  __shared__ float sS[6][kMaxLobes];
  __shared__ int smg[kMaxLobes][15];     // marginal counts: axis * 5 + bin
  __shared__ int64_t sC[kMaxLobes][12];  // cumulative marginals, bins 0..3
  __shared__ int64_t sm[kMaxLobes];
  __shared__ int son[kMaxLobes];
  const int64_t nparents = *n_par, nc = *n_child;
  if (nparents > pmax || nc > cmax) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
      atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_VOXEL_CAPACITY);
    return;
  }
  const int lane = threadIdx.x;
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  for (int64_t p = blockIdx.x; p < nparents; p += gridDim.x) {
    const Key pk = pkeys[p];
    // children: key >> 3 == pk, contiguous from the first key >= pk << 3
    int64_t lo = 0, hi = nc;
    const Key first = Key(pk << 3);
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ckeys[mid] < first) lo = mid + 1; else hi = mid;
    }
    // gather the positive lobes, child-major then lobe order: lane = child * Kc + lobe
    bool have = false;
    float lw = 0.0f;
    float lS[6] = {0, 0, 0, 0, 0, 0};
    {
      const int ci = lane / Kc, k = lane % Kc;
      const int64_t c = lo + ci;
      if (ci < 8 && c < nc && Key(ckeys[c] >> 3) == pk) {
        if (clob.nl == nullptr) {
          if (k == 0) {
            lw = leaf_w[c];
#pragma unroll
            for (int t = 0; t < 6; ++t) lS[t] = leaf_S[t * leaf_cap + c];
            have = lw > 0.0f;
          }
        } else if (k < int(clob.nl[c])) {
          lw = clob.w[int64_t(k) * clob.cap + c];
#pragma unroll
          for (int t = 0; t < 6; ++t) lS[t] = clob.S[(int64_t(t) * Kc + k) * clob.cap + c];
          have = lw > 0.0f;
        }
      }
    }
    const uint64_t hv = __ballot(have);
    const int n = __popcll(hv);
    const int slot = __popcll(hv & lt);
    if (have) {
      sw[slot] = lw;
#pragma unroll
      for (int t = 0; t < 6; ++t) sS[t][slot] = lS[t];
    }
    if (lane < kMaxLobes) son[lane] = lane < n;
    __syncthreads();
    if (n > K) {
      // marginal counts of N samples per lobe (integer atomics: exact and order-free)
      for (int i = lane; i < kMaxLobes * 15; i += 64) smg[i / 15][i % 15] = 0;
      __syncthreads();
      // The n N samples are dealt to the lanes in turn, and a lane moves to its next sample as
      // soon as one is accepted, so the lanes' attempts do not wait for one another sample by
      // sample (acceptance runs from about a quarter to a half per attempt).
      {
        const int total = n * N;
        int t = lane, at = 0, cj = -1;
        Chol c{};
        uint64_t key = 0;
        while (t < total) {
          const int j = t / N, k = t - j * N;
          if (j != cj) {
            c = lobe_chol(sw[j], sS[0][j], sS[1][j], sS[2][j], sS[3][j], sS[4][j], sS[5][j]);
            key = lobe_key(level, uint64_t(pk), j);
            cj = j;
          }
          int b[3];
          const bool ok = lobe_attempt(c, key, uint64_t(k), at, b);
          if (ok) {
            atomicAdd(&smg[j][b[0]], 1);
            atomicAdd(&smg[j][5 + b[1]], 1);
            atomicAdd(&smg[j][10 + b[2]], 1);
          }
          if (ok || at + 1 >= kMaxAttempts) {
            t += 64;
            at = 0;
          } else {
            ++at;
          }
        }
      }
      __syncthreads();
      if (lane < n) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          int64_t run = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            run += smg[lane][5 * a + b];
            sC[lane][4 * a + b] = run;
          }
        }
        sm[lane] = 1;
      }
      __syncthreads();
      // closest pair by rows: lane i scans j > i; ties keep the first j, then the first row
      for (int active = n; active > K; --active) {
        int64_t bn = 0, bd = 1;
        int bi = -1, bj = -1;
        if (lane < n && son[lane]) {
          const int i = lane;
          int64_t Ci[12];
#pragma unroll
          for (int t = 0; t < 12; ++t) Ci[t] = sC[i][t];
          const int64_t mi = sm[i];
          for (int j = i + 1; j < n; ++j) {
            if (!son[j]) continue;
            const int64_t mj = sm[j];
            int64_t num = 0;
#pragma unroll
            for (int t = 0; t < 12; ++t) {
              const int64_t d = Ci[t] * mj - sC[j][t] * mi;
              num += d < 0 ? -d : d;
            }
            const int64_t den = mi * mj;
            if (bi < 0 || num * bd < bn * den) {
              bi = i;
              bj = j;
              bn = num;
              bd = den;
            }
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const int64_t on = __shfl_xor(bn, o, 64), od = __shfl_xor(bd, o, 64);
          const int oi = __shfl_xor(bi, o, 64), oj = __shfl_xor(bj, o, 64);
          if (pair_before(on, od, oi, oj, bn, bd, bi, bj)) {
            bn = on;
            bd = od;
            bi = oi;
            bj = oj;
          }
        }
        // every lane holds the same pair now
        if (lane == 0) {
          sw[bi] = sw[bi] + sw[bj];
#pragma unroll
          for (int t = 0; t < 6; ++t) sS[t][bi] = sS[t][bi] + sS[t][bj];
          sm[bi] += sm[bj];
#pragma unroll
          for (int t = 0; t < 12; ++t) sC[bi][t] += sC[bj][t];
          son[bj] = 0;
        }
        __syncthreads();
      }
    }
    // survivors by descending weight (ties in slot order)
    const int m = n > K ? K : n;
    if (lane < n && son[lane]) {
      const float w = sw[lane];
      int rank = 0;
      for (int t = 0; t < n; ++t)
        if (son[t] && (sw[t] > w || (sw[t] == w && t < lane))) ++rank;
      plob.w[int64_t(rank) * plob.cap + p] = w;
#pragma unroll
      for (int t = 0; t < 6; ++t) plob.S[(int64_t(t) * K + rank) * plob.cap + p] = sS[t][lane];
    }
    if (lane >= m && lane < K) {
      plob.w[int64_t(lane) * plob.cap + p] = 0.0f;
#pragma unroll
      for (int t = 0; t < 6; ++t) plob.S[(int64_t(t) * K + lane) * plob.cap + p] = 0.0f;
    }
    if (lane == 0) plob.nl[p] = uint8_t(m);
    __syncthreads();
  }
}

}  // namespace

vx_status sggxh_run(const vx_grid* g, const vx_voxels* leaf, const vx_voxels* out, const int64_t* n_levels,
                    int levels, int K, int N, const vx_lobes* lobes, int64_t* stats, hipStream_t s) {
  const bool key64 = g->log2_res > 10;
  launch_fill_i64(stats, VX_NSTAT, 0, s);
  for (int l = 1; l < levels; ++l) {
    const vx_voxels& C = l == 1 ? *leaf : out[l - 2];
    const vx_voxels& P = out[l - 1];
    const vx_lobes clob = l == 1 ? vx_lobes{nullptr, nullptr, nullptr, 0} : lobes[l - 2];
    const int Kc = l == 1 ? 1 : K;
    const int64_t cmax = l == 1 ? C.cap : (C.cap < clob.cap ? C.cap : clob.cap);
    const int64_t pmax = P.cap < lobes[l - 1].cap ? P.cap : lobes[l - 1].cap;
    const int grid = int(pmax < 16384 ? (pmax < 1 ? 1 : pmax) : 16384);
    VX_TIMED("sggxh_level", s);
#define VX_SH(Ky)                                                                                                \
  hipLaunchKernelGGL(k_sggxh_level<Ky>, dim3(grid), dim3(64), 0, s, (const Ky*)C.keys, n_levels + l - 1, cmax,  \
                     leaf->w, leaf->S, leaf->cap, clob, Kc, (const Ky*)P.keys, n_levels + l, pmax, lobes[l - 1], K, \
                     l, N, stats)
    if (key64) VX_SH(uint64_t); else VX_SH(uint32_t);
#undef VX_SH
  }
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

}  // namespace vx
