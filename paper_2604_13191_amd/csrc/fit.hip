// fit.hip -- differentiable two-lobe fit over the pyramid, forward and hand-written backward.
//
// For every voxel u of levels lo..hi with w_u > 0, two lobes given by lower-triangular L_1, L_2
// (6 parameters each: L00 L10 L11 L20 L21 L22) have projected area
// f_u(omega) = |L_1^T omega| + |L_2^T omega|; the target is the density-weighted projected area
// of u's children, tau_u(omega) = sum_c sqrt(w_c omega^T S_c omega) / sum_c w_c (Sec. 4.1 gives
// sigma(omega) = sqrt(omega^T S omega) for an SGGX S = S_c / w_c).  The loss is the sum over
// voxels of the mean over the direction set of (f_u - tau_u)^2.
//
// Backward: d loss / d L per voxel; d loss / d (S_c, w_c) per child, accumulated top-down so
// that every leaf voxel holds the gradient of all its ancestors' sums; then, per fiber segment,
// through the clipped lengths (weights) and the tangent (moment I - t t^T) to the control
// points.  Intermediates are recomputed instead of stored: the per-direction profiles are
// re-evaluated in the backward kernel, and the (segment, voxel) pairs are re-emitted in
// primitive order by the voxelize front half.
#include "geom.hpp"
#include "vx_internal.hpp"

namespace vx {

template <class Key>
__device__ __forceinline__ int64_t key_lower_bound(const Key* __restrict__ keys, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (uint64_t(keys[mid]) < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ float quadf(const float* S, float x, float y, float z) {
  return S[0] * x * x + S[1] * y * y + S[2] * z * z + 2.0f * (S[3] * x * y + S[4] * x * z + S[5] * y * z);
}

constexpr int kMaxChild = 8;

// children of voxel u in the level below: [cstart[u], cstart[u + 1]), at most 8
__device__ __forceinline__ int child_range(const int64_t* __restrict__ cstart, int64_t u, int64_t& first) {
  first = cstart[u];
  const int64_t n = cstart[u + 1] - first;
  return int(n < kMaxChild ? n : kMaxChild);
}

// ---------------------------------------------------------------------------------------------
// Layout of both passes: 16 lanes per voxel (four voxels per wave), each lane taking every 16th
// direction; a voxel's children (w, S) are staged in LDS by its group, the directions of the set
// once per block.  Sums over a group's lanes are butterfly reductions over 16 lanes.
// ---------------------------------------------------------------------------------------------
constexpr int kGroup = 16;                      // lanes per voxel
constexpr int kGroups = kBlock / kGroup;        // voxels in flight per block
constexpr int kMaxDir = 256;

template <class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = kGroup / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kGroup);
  return v;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// the children of voxel u staged by the group: cw[c], cS[c][6]; returns their number
template <class T>
__device__ __forceinline__ int stage_children(const vx_voxels& ch, const int64_t* cstart, int64_t u, bool active,
                                              int gl, T* cw, T (*cS)[6], int64_t& first) {
  int nc = 0;
  first = 0;
  if (active) nc = child_range(cstart, u, first);
  if (active && gl < nc) {
    const int64_t cc = first + gl;
    cw[gl] = T(ch.w[cc]);
#pragma unroll
    for (int t = 0; t < 6; ++t) cS[gl][t] = T(ch.S[int64_t(t) * ch.cap + cc]);
  }
  wave_sync_lds();
  return nc;
}

// ---------------------------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_fit_fwd(vx_voxels par, const int64_t* n_par_p, int64_t rows, vx_voxels ch,
                                                    const int64_t* __restrict__ cstart, const float* __restrict__ Lp,
                                                    const float* __restrict__ dirs, int ndir,
                                                    float* __restrict__ loss_vox) {
  __shared__ float sdir[kMaxDir][3];
  __shared__ float scw[kGroups][kMaxChild];
  __shared__ float scS[kGroups][kMaxChild][6];
  for (int k = threadIdx.x; k < ndir; k += kBlock)
    for (int a = 0; a < 3; ++a) sdir[k][a] = dirs[3 * k + a];
  __syncthreads();
  const int grp = threadIdx.x / kGroup, gl = threadIdx.x % kGroup;
  const int64_t n_par = *n_par_p < rows ? *n_par_p : rows;   // never past the parameter rows
  // the four groups of a wave advance together (uniform trip count per wave)
  const int wgrp0 = (threadIdx.x >> 6) * (64 / kGroup);
  for (int64_t u0 = int64_t(blockIdx.x) * kGroups + wgrp0; u0 < n_par; u0 += int64_t(gridDim.x) * kGroups) {
    const int64_t u = u0 + (grp - wgrp0);
    const bool in = u < n_par;
    const float W = in ? par.w[u] : 0.f;
    const bool active = in && W > 0.f;
    int64_t first;
    const int nc = stage_children(ch, cstart, u, active, gl, scw[grp], scS[grp], first);
    float acc = 0.f;
    if (active) {
      float l[12];
      for (int t = 0; t < 12; ++t) l[t] = Lp[u * 12 + t];
      const float invW = 1.0f / W;
      for (int k = gl; k < ndir; k += kGroup) {
        const float x = sdir[k][0], y = sdir[k][1], z = sdir[k][2];
        float tau = 0.f;
        for (int c = 0; c < nc; ++c)
          if (scw[grp][c] > 0.f) tau += sqrtf(fmaxf(scw[grp][c] * quadf(scS[grp][c], x, y, z), 0.f));
        tau *= invW;
        float f = 0.f;
        for (int j = 0; j < 2; ++j) {
          const float* lj = l + 6 * j;
          const float y0 = lj[0] * x + lj[1] * y + lj[3] * z, y1 = lj[2] * y + lj[4] * z, y2 = lj[5] * z;
          f += sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
        }
        const float r = f - tau;
        acc = fmaf(r, r, acc);
      }
    }
    acc = group_sum(acc);
    if (in && gl == 0) loss_vox[u] = active ? acc / float(ndir) : 0.f;
    wave_sync_lds();                                  // the group's LDS slots are reused next
  }
}

// deterministic sum of the per-voxel losses of all levels into loss[0]: fixed per-block chunks
// of every level, then one block adds the block sums in order
struct LossLevels {
  const float* p[24];
  const int64_t* n[24];
  int64_t rows[24];       // the forward wrote at most this many per-voxel losses
  int count;
};

__global__ void __launch_bounds__(kBlock) k_fit_partial(LossLevels lv, float* __restrict__ part) {
  __shared__ float red[kWaves];
  float acc = 0.f;
  for (int i = 0; i < lv.count; ++i) {
    const int64_t n = *lv.n[i] < lv.rows[i] ? *lv.n[i] : lv.rows[i];
    const int64_t chunk = (n + kGrid - 1) / kGrid;
    const int64_t b0 = int64_t(blockIdx.x) * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    for (int64_t j = b0 + threadIdx.x; j < b1; j += kBlock) acc += lv.p[i][j];
  }
  acc = wave_sum(acc);
  if (lane_id() == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < kWaves; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(1024) k_fit_total(const float* __restrict__ part, float* loss) {
  __shared__ float red[16];
  float acc = threadIdx.x < kGrid ? part[threadIdx.x] : 0.f;
  acc = wave_sum(acc);
  if (lane_id() == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < 16; ++w) t += red[w];
    loss[0] = t;
  }
}

// ---------------------------------------------------------------------------------------------
// backward per voxel: lobe gradients and the gradient of the target w.r.t. the children's sums.
// FP64: the derivative of the target along a child's own (w, S) direction nearly cancels (the
// target is invariant when all children scale alike), so the parts must be accurate.
// gch: [7][gcap] (S components, then w) for the level below.  DPL: directions per lane.
// ---------------------------------------------------------------------------------------------
// 1 / sqrt(x), x > 0: the hardware estimate refined by one Newton step,
// r' = r (3/2 - x r^2 / 2), which squares the estimate's relative error
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * r;
  return fma(r, fma(-h, r, 0.5), r);
}
// sqrt(x) for x >= 0 as x / sqrt(x)
__device__ __forceinline__ double sqrt_nr(double x) { return x > 0.0 ? x * rsqrt_nr(x) : 0.0; }

__device__ __forceinline__ double quadd(const double* S, double x, double y, double z) {
  return S[0] * x * x + S[1] * y * y + S[2] * z * z + 2.0 * (S[3] * x * y + S[4] * x * z + S[5] * y * z);
}

template <int DPL>
__global__ void __launch_bounds__(kBlock) k_fit_bwd(vx_voxels par, const int64_t* n_par_p, int64_t rows,
                                                    const double* __restrict__ c64, int64_t ccap,
                                                    const int64_t* __restrict__ cstart, const float* __restrict__ Lp,
                                                    const float* __restrict__ dirs, int ndir,
                                                    const float* __restrict__ dloss, float* __restrict__ dLp,
                                                    double* __restrict__ gch, int64_t gcap) {
  // directions and the children's FP64 sums staged once, not converted in the inner loops
  __shared__ double sdir[kMaxDir][3];
  __shared__ double scw[kGroups][kMaxChild];
  __shared__ double scS[kGroups][kMaxChild][6];
  for (int k = threadIdx.x; k < ndir; k += kBlock)
    for (int a = 0; a < 3; ++a) sdir[k][a] = dirs[3 * k + a];
  __syncthreads();
  const int grp = threadIdx.x / kGroup, gl = threadIdx.x % kGroup;
  const int64_t n_par = *n_par_p < rows ? *n_par_p : rows;
  const double g0 = double(dloss[0]);
  const double g2 = 2.0 / double(ndir) * g0;
  const int wgrp0 = (threadIdx.x >> 6) * (64 / kGroup);
  for (int64_t u0 = int64_t(blockIdx.x) * kGroups + wgrp0; u0 < n_par; u0 += int64_t(gridDim.x) * kGroups) {
    const int64_t u = u0 + (grp - wgrp0);
    const bool in = u < n_par;
    const float Wf = in ? par.w[u] : 0.f;
    const bool active = in && Wf > 0.f && c64 != nullptr;   // no FP64 sums: no points, nothing to fit
    int64_t first = 0;
    int nc = 0;
    if (active) nc = child_range(cstart, u, first);
    if (active && gl < nc) {
      const int64_t cc = first + gl;
      scw[grp][gl] = c64[6 * ccap + cc];
#pragma unroll
      for (int t = 0; t < 6; ++t) scS[grp][gl][t] = c64[int64_t(t) * ccap + cc];
    }
    wave_sync_lds();
    const double* cw = scw[grp];
    double l[12], gl12[12], dg[DPL], dt[DPL];
#pragma unroll
    for (int t = 0; t < 12; ++t) {
      l[t] = active ? double(Lp[u * 12 + t]) : 0.0;
      gl12[t] = 0.0;
    }
    // the parent's weight as the FP64 sum of its children's
    double Wd = 0.0;
    for (int c = 0; c < nc; ++c) Wd += cw[c];
    const double invW = active && Wd > 0.0 ? 1.0 / Wd : 0.0;
    // pass 1 (this lane's directions): target, fit, residual; lobe gradients
#pragma unroll
    for (int i = 0; i < DPL; ++i) {
      const int k = gl + kGroup * i;
      dg[i] = 0.0;
      dt[i] = 0.0;
      if (!active || k >= ndir) continue;
      const double x = sdir[k][0], y = sdir[k][1], z = sdir[k][2];
      double tau = 0.0;
      for (int c = 0; c < nc; ++c) {
        const double wc = double(cw[c]);
        if (!(wc > 0.0)) continue;
        tau += sqrt_nr(fmax(wc * quadd(scS[grp][c], x, y, z), 0.0));
      }
      tau *= invW;
      double f = 0.0, yv[2][3], ry[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double* lj = l + 6 * j;
        yv[j][0] = lj[0] * x + lj[1] * y + lj[3] * z;
        yv[j][1] = lj[2] * y + lj[4] * z;
        yv[j][2] = lj[5] * z;
        const double n2 = yv[j][0] * yv[j][0] + yv[j][1] * yv[j][1] + yv[j][2] * yv[j][2];
        ry[j] = n2 > 0.0 ? rsqrt_nr(n2) : 0.0;                 // 1 / |L_j^T w|
        f += n2 * ry[j];
      }
      const double g = (f - tau) * g2;                          // d loss / d f;  d loss / d tau = -g
      dg[i] = g;
      dt[i] = tau;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (!(ry[j] > 0.0)) continue;
        const double sj = g * ry[j];
        double* gj = gl12 + 6 * j;
        gj[0] += sj * yv[j][0] * x;
        gj[1] += sj * yv[j][0] * y;
        gj[2] += sj * yv[j][1] * y;
        gj[3] += sj * yv[j][0] * z;
        gj[4] += sj * yv[j][1] * z;
        gj[5] += sj * yv[j][2] * z;
      }
    }
#pragma unroll
    for (int t = 0; t < 12; ++t) {
      const double v = group_sum(gl12[t]);
      if (active && gl == t) dLp[u * 12 + t] = float(v);
    }
    if (in && !active && gl < 12) dLp[u * 12 + gl] = 0.f;
    // pass 2 (one child at a time): d loss / d (S_c, w_c)
    for (int c = 0; c < kMaxChild; ++c) {
      if (!__any(active && c < nc)) break;                 // uniform over the wave
      double acc[7] = {0, 0, 0, 0, 0, 0, 0};
      const bool on = active && c < nc;
      const double wc = on ? double(cw[c]) : 0.0;
      if (on && wc > 0.0) {
#pragma unroll
        for (int i = 0; i < DPL; ++i) {
          const int k = gl + kGroup * i;
          if (k >= ndir) continue;
          const double x = sdir[k][0], y = sdir[k][1], z = sdir[k][2], g = dg[i];
          const double qs = quadd(scS[grp][c], x, y, z);
          const double q2 = wc * qs;
          double dw = -dt[i] * invW;
          if (q2 > 0.0) {
            const double h = 0.5 * rsqrt_nr(q2) * invW;         // 1 / (2 sqrt(w_c w^T S_c w)) / W
            const double k2 = -g * wc * h;                      // d loss / d (w^T S_c w)
            acc[0] += k2 * x * x;
            acc[1] += k2 * y * y;
            acc[2] += k2 * z * z;
            acc[3] += k2 * 2.0 * x * y;
            acc[4] += k2 * 2.0 * x * z;
            acc[5] += k2 * 2.0 * y * z;
            dw += qs * h;
          }
          acc[6] += -g * dw;
        }
      }
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const double v = group_sum(acc[t]);
        if (on && gl == t) gch[int64_t(t) * gcap + first + c] = v;
      }
    }
    wave_sync_lds();                                  // the group's LDS slots are reused next
  }
}

// top-down: every voxel of level L adds its parent's accumulated gradient (level L+1)
__global__ void __launch_bounds__(kBlock) k_fit_down(const int32_t* __restrict__ pidx, const int64_t* n_p,
                                                     double* __restrict__ g, int64_t gcap,
                                                     const double* __restrict__ gup, int64_t gupcap) {
  const int64_t n = *n_p;
  for (int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x; c < n; c += int64_t(gridDim.x) * kBlock) {
    const int64_t p = pidx[c];
#pragma unroll
    for (int t = 0; t < 7; ++t) g[int64_t(t) * gcap + c] += gup[int64_t(t) * gupcap + p];
  }
}

// leaf lookup table: first and end leaf index of every 16^3 tile (empty tiles: 0, 0)
template <class Key>
__global__ void __launch_bounds__(kBlock) k_tile_index(const Key* __restrict__ keys, const int64_t* n_p,
                                                       int64_t* __restrict__ tfirst, int64_t* __restrict__ tend) {
  const int64_t n = *n_p;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    const uint64_t t = uint64_t(keys[i]) >> (3 * kTileBits);
    if (i == 0 || (uint64_t(keys[i - 1]) >> (3 * kTileBits)) != t) tfirst[t] = i;
    if (i == n - 1 || (uint64_t(keys[i + 1]) >> (3 * kTileBits)) != t) tend[t] = i + 1;
  }
}

// per segment: chain rule over its (segment, voxel) pairs, which the front half emitted
// contiguously in primitive order; seg_grad[p] = (d/dA, d/dB) in world units
template <class Key>
__global__ void __launch_bounds__(kBlock) k_fit_pairs(const int32_t* __restrict__ rec,
                                                      const int64_t* __restrict__ cand_off, int64_t n_prims,
                                                      const uint64_t* __restrict__ masks,
                                                      const int64_t* __restrict__ wave_off,
                                                      const int64_t* __restrict__ ctl, const Key* __restrict__ pkeys,
                                                      vx_voxels leaf, const int64_t* n_leaf_p,
                                                      const double* __restrict__ gleaf, int64_t gcap, int Sb,
                                                      int log2R, double vs, const int64_t* __restrict__ tfirst,
                                                      const int64_t* __restrict__ tend, double* __restrict__ seg_grad) {
  const int64_t n_leaf = *n_leaf_p;
  const int64_t n_cand = ctl[CTL_N_CAND];
  const int64_t n_pairs = ctl[CTL_N_PAIRS];
  const Key* lk = reinterpret_cast<const Key*>(leaf.keys);
  const double inv_s = 1.0 / double(int64_t(1) << Sb);
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < n_prims; p += int64_t(gridDim.x) * kBlock) {
    double gA[3] = {0, 0, 0}, gB[3] = {0, 0, 0};
    const int64_t c0 = cand_off[p], c1 = cand_off[p + 1];
    if (c1 > c0 && c1 <= n_cand) {
      auto pair_index = [&](int64_t c) -> int64_t {
        const int64_t ch = c >> 6;
        const int r = int(c & 63);
        return wave_off[ch] + (r ? __popcll(masks[ch] & ((uint64_t(1) << r) - 1)) : 0);
      };
      int64_t j0 = pair_index(c0), j1 = pair_index(c1);
      if (j0 < 0 || j1 > n_pairs || j0 > j1) j1 = j0;          // front half over capacity: no pairs
      const int32_t* r = rec + p * kRec;
      double A[3], B[3], d[3];
      for (int a = 0; a < 3; ++a) {
        A[a] = double(r[a]) * inv_s;
        B[a] = double(r[3 + a]) * inv_s;
        d[a] = B[a] - A[a];
      }
      const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double t[3] = {0, 0, 0};
      if (len > 0)
        for (int a = 0; a < 3; ++a) t[a] = d[a] / len;
      const double M[6] = {1 - t[0] * t[0], 1 - t[1] * t[1], 1 - t[2] * t[2], -t[0] * t[1], -t[0] * t[2], -t[1] * t[2]};
      double gM[6] = {0, 0, 0, 0, 0, 0};
      for (int64_t j = j0; j < j1; ++j) {
        const uint64_t key = uint64_t(pkeys[j]);
        double lo[3] = {0, 0, 0};
        for (int b = 0; b < log2R; ++b)
          for (int a = 0; a < 3; ++a) lo[a] += double((key >> (3 * b + a)) & 1) * double(int64_t(1) << b);
        double dA[3], dB[3];
        const double w = seg_length_grad(A, B, lo, dA, dB);
        if (!(w > 0.0)) continue;
        int64_t v;
        if (tfirst) {
          const uint64_t t = key >> (3 * kTileBits);
          const int64_t a = tfirst[t], b = tend[t];
          v = a + key_lower_bound(lk + a, b - a, key);
          if (v >= b) continue;
        } else {
          v = key_lower_bound(lk, n_leaf, key);
        }
        if (v >= n_leaf || uint64_t(lk[v]) != key) continue;
        double gS[6];
        for (int q = 0; q < 6; ++q) gS[q] = gleaf[int64_t(q) * gcap + v];
        double gw = gleaf[6 * gcap + v];
        for (int q = 0; q < 6; ++q) {
          gw += gS[q] * M[q];
          gM[q] += w * gS[q];
        }
        for (int a = 0; a < 3; ++a) {
          gA[a] += gw * dA[a];
          gB[a] += gw * dB[a];
        }
      }
      if (len > 0) {
        double gt[3];
        gt[0] = -2 * t[0] * gM[0] - t[1] * gM[3] - t[2] * gM[4];
        gt[1] = -2 * t[1] * gM[1] - t[0] * gM[3] - t[2] * gM[5];
        gt[2] = -2 * t[2] * gM[2] - t[0] * gM[4] - t[1] * gM[5];
        const double dot = gt[0] * t[0] + gt[1] * t[1] + gt[2] * t[2];
        for (int a = 0; a < 3; ++a) {
          const double gd = (gt[a] - dot * t[a]) / len;
          gA[a] -= gd;
          gB[a] += gd;
        }
      }
    }
    for (int a = 0; a < 3; ++a) {
      seg_grad[p * 6 + a] = gA[a] * vs;
      seg_grad[p * 6 + 3 + a] = gB[a] * vs;
    }
  }
}

// a point's gradient: its segment's start end plus the previous segment's far end, added in FP64
// (the two nearly cancel along a straight fiber) and rounded once
__global__ void __launch_bounds__(kBlock) k_fit_points(const double* __restrict__ seg_grad, int64_t n,
                                                       float* __restrict__ dpts) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    for (int a = 0; a < 3; ++a)
      dpts[i * 3 + a] = float(seg_grad[i * 6 + a] + (i > 0 ? seg_grad[(i - 1) * 6 + 3 + a] : 0.0));
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------------------------
// binding of the lobe parameters: row r of a level's parameters belongs to the voxel that was at
// index r when the parameters were made.  A level whose voxel count or keys differ from that
// binding (control points moved across voxels) is flagged, and every kernel stays within the
// parameter rows.
// ---------------------------------------------------------------------------------------------
template <class Key>
__global__ void __launch_bounds__(kBlock) k_fit_bind(const Key* __restrict__ keys, const int64_t* n_p, int64_t rows,
                                                     const Key* __restrict__ bound, int64_t* stats) {
  const int64_t n = *n_p;
  if (blockIdx.x == 0 && threadIdx.x == 0 && n != rows)
    atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_FIT_ROWS);
  if (!bound) return;
  const int64_t m = n < rows ? n : rows;
  bool diff = false;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < m; i += int64_t(gridDim.x) * kBlock)
    diff = diff || keys[i] != bound[i];
  if (__any(diff) && lane_id() == 0)
    atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_FIT_KEYS);
}

// ---------------------------------------------------------------------------------------------
// FP64 sums of the levels below the fitted ones, for the backward pass.  The target's square
// roots are ill-conditioned where a child holds nearly one fiber direction and a direction of
// the set is nearly parallel to it, so the backward differentiates at sums formed in FP64 from
// the re-emitted pairs: sorted by key (stable, so each voxel's pairs stay in primitive order),
// each leaf voxel adds its clipped lengths and moments in FP64, and every level above adds its
// children.  Layout of a level: [7][cap] (S components xx yy zz xy xz yz, then w).
// ---------------------------------------------------------------------------------------------
// start has cap + 2 entries: the first pair of every key (heads past cap are dropped), the end
// at index min(total, cap), and the number of distinct keys at index cap + 1
struct LeafSegOut {
  int64_t* start;
  int64_t cap;
  __device__ void operator()(int64_t i, int64_t ex, int64_t v) const {
    if (v && ex <= cap) start[ex] = i;
  }
};
struct LeafSegTotal {
  int64_t* start;
  int64_t cap;
  const int64_t* n_leaf;
  int64_t* stats;
  __device__ void operator()(int64_t total, int64_t n) const {
    if (total <= cap) start[total] = n;
    start[cap + 1] = total;
    if (total != *n_leaf)
      atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_FIT_KEYS);
  }
};

template <class Key>
__global__ void __launch_bounds__(kBlock) k_fit_leaf64(const Key* __restrict__ pkeys, const uint32_t* __restrict__ pprim,
                                                       const int64_t* __restrict__ sstart, const int32_t* __restrict__ rec,
                                                       const Key* __restrict__ lkeys, const int64_t* n_leaf_p,
                                                       int64_t cap, int Sb, int log2R, double* __restrict__ out,
                                                       int64_t* stats) {
  // within the leaf, its capacity and the keys the pairs hold (sstart[i + 1] is written for i < n)
  int64_t n = *n_leaf_p < cap ? *n_leaf_p : cap;
  n = sstart[cap + 1] < n ? sstart[cap + 1] : n;
  const double inv_s = 1.0 / double(int64_t(1) << Sb);
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    const int64_t a = sstart[i], b = sstart[i + 1];
    double W = 0.0, S[6] = {0, 0, 0, 0, 0, 0};
    if (b > a && pkeys[a] != lkeys[i])
      atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_FIT_KEYS);
    const uint64_t key = uint64_t(lkeys[i]);
    double lo[3] = {0, 0, 0};
    for (int bit = 0; bit < log2R; ++bit)
      for (int ax = 0; ax < 3; ++ax) lo[ax] += double((key >> (3 * bit + ax)) & 1) * double(int64_t(1) << bit);
    for (int64_t j = a; j < b; ++j) {
      const int32_t* r = rec + int64_t(pprim[j]) * kRec;
      double A[3], B[3], d[3], gA[3], gB[3];
      for (int ax = 0; ax < 3; ++ax) {
        A[ax] = double(r[ax]) * inv_s;
        B[ax] = double(r[3 + ax]) * inv_s;
        d[ax] = B[ax] - A[ax];
      }
      const double w = seg_length_grad(A, B, lo, gA, gB);
      if (!(w > 0.0)) continue;
      const double l2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double il2 = 1.0 / l2;
      W += w;
      S[0] += w * (1.0 - d[0] * d[0] * il2);
      S[1] += w * (1.0 - d[1] * d[1] * il2);
      S[2] += w * (1.0 - d[2] * d[2] * il2);
      S[3] -= w * d[0] * d[1] * il2;
      S[4] -= w * d[0] * d[2] * il2;
      S[5] -= w * d[1] * d[2] * il2;
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) out[int64_t(t) * cap + i] = S[t];
    out[6 * cap + i] = W;
  }
}

// level L from level L - 1: every voxel adds its children [cstart[u], cstart[u + 1]) in order
__global__ void __launch_bounds__(kBlock) k_fit_up64(const int64_t* __restrict__ cstart, const int64_t* n_p,
                                                     int64_t cap, const double* __restrict__ in, int64_t icap,
                                                     double* __restrict__ out) {
  const int64_t n = *n_p < cap ? *n_p : cap;
  for (int64_t u = int64_t(blockIdx.x) * kBlock + threadIdx.x; u < n; u += int64_t(gridDim.x) * kBlock) {
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t c = cstart[u]; c < cstart[u + 1]; ++c)
#pragma unroll
      for (int t = 0; t < 7; ++t) acc[t] += in[int64_t(t) * icap + c];
#pragma unroll
    for (int t = 0; t < 7; ++t) out[int64_t(t) * cap + u] = acc[t];
  }
}

__global__ void __launch_bounds__(kBlock) k_copy_pairs(const uint8_t* __restrict__ ksrc, const uint32_t* __restrict__ psrc,
                                                       const int64_t* __restrict__ ctl, int kb,
                                                       uint8_t* __restrict__ kdst, uint32_t* __restrict__ pdst) {
  const int64_t n = ctl[CTL_N_PAIRS];
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    if (kb == 8) reinterpret_cast<uint64_t*>(kdst)[i] = reinterpret_cast<const uint64_t*>(ksrc)[i];
    else reinterpret_cast<uint32_t*>(kdst)[i] = reinterpret_cast<const uint32_t*>(ksrc)[i];
    pdst[i] = psrc[i];
  }
}

// ---------------------------------------------------------------------------------------------
// orchestration
// ---------------------------------------------------------------------------------------------
struct FitWs {
  float* loss_vox[21];
  double* g[21];           // [7][cap_L] per level 0..hi-1
  int64_t* cstart[21];     // [cap_L + 1] per level 1..hi: first child (in level L-1) of every voxel
  int32_t* pidx[21];       // [cap_L] per level 0..hi-1: index of every voxel's parent in level L+1
  int64_t* tfirst;         // [tiles] leaf lookup: first and end leaf index of every 16^3 tile
  int64_t* tend;
  float* part;             // [kGrid] block sums of the loss
  int64_t* partial;        // [kGrid + 1] scan partials
  double* seg_grad;        // [n_pts][6] d loss / d (segment start, segment end), world units
  FrontWs f;
  double* s64[21];         // [7][cap_L] per level 0..hi-1: FP64 sums (S, then w)
  int64_t* sstart;         // [cap_0 + 2] first sorted pair of every leaf voxel, end, key count
  PairBufs pb, pc;         // sort buffers of the re-emitted pairs (a copy, then ping-pong)
  int32_t* hist;           // radix digit histograms
};

// dense table of 16^3 tiles for the leaf lookup of the backward pass (grids up to 2048^3)
static int64_t leaf_tiles(int log2R) {
  return log2R > kTileBits && log2R <= 11 ? int64_t(1) << (3 * (log2R - kTileBits)) : 0;
}

static size_t fit_ws_layout(int64_t n_pts, int64_t max_cand, int64_t max_pairs, const int64_t* caps, int hi,
                            int log2R, void* base, FitWs* w) {
  const bool key64 = log2R > 10;
  Carver cv(base);
  FitWs x;
  for (int L = 0; L <= hi; ++L) x.loss_vox[L] = cv.take<float>(caps[L]);
  for (int L = 0; L < hi; ++L) x.g[L] = cv.take<double>(7 * caps[L]);
  for (int L = 1; L <= hi; ++L) x.cstart[L] = cv.take<int64_t>(caps[L] + 1);
  for (int L = 0; L < hi; ++L) x.pidx[L] = cv.take<int32_t>(caps[L]);
  const int64_t tiles = leaf_tiles(log2R);
  x.tfirst = cv.take<int64_t>(tiles);
  x.tend = cv.take<int64_t>(tiles);
  x.part = cv.take<float>(kGrid);
  x.partial = cv.take<int64_t>(kGrid + 1);
  x.seg_grad = cv.take<double>(6 * n_pts);
  front_ws_carve(cv, n_pts, max_cand, max_pairs, key64, &x.f);
  for (int L = 0; L < hi; ++L) x.s64[L] = cv.take<double>(n_pts > 0 ? 7 * caps[L] : 0);
  x.sstart = cv.take<int64_t>(n_pts > 0 ? caps[0] + 2 : 0);
  const int kb = key64 ? 8 : 4;
  for (PairBufs* pbuf : {&x.pb, &x.pc}) {
    pbuf->keys = cv.take<uint8_t>(max_pairs * kb);
    pbuf->w = cv.take<float>(max_pairs);
    pbuf->prim = cv.take<uint32_t>(max_pairs);
  }
  x.hist = cv.take<int32_t>(max_pairs > 0 ? int64_t(kRadixBuckets) * kGrid : 0);
  if (w) *w = x;
  return cv.off + 256;
}

size_t fit_ws_bytes(int64_t n_pts, int64_t max_cand, int64_t max_pairs, const int64_t* caps, int hi, int log2R) {
  return fit_ws_layout(n_pts, max_cand, max_pairs, caps, hi, log2R, nullptr, nullptr);
}

struct StartTotal {
  int64_t* start;
  __device__ void operator()(int64_t total, int64_t n) const { start[total] = n; }
};
// heads of the parent key: the parent's first child, and every child's parent index
struct ChildOut {
  int64_t* start;
  int32_t* parent;
  __device__ void operator()(int64_t i, int64_t ex, int64_t v) const {
    if (v) start[ex] = i;
    parent[i] = int32_t(ex + v - 1);
  }
};

// first child of every voxel of levels 1..hi: heads of the parent key over each level below
static void child_starts(bool key64, const vx_voxels* levels, const int64_t* n_levels, int hi, const FitWs& w,
                         hipStream_t s) {
  VX_TIMED("fit_children", s);
  for (int L = 1; L <= hi; ++L) {
    if (key64)
      device_scan(HeadIn<uint64_t, 3>{(const uint64_t*)levels[L - 1].keys}, ChildOut{w.cstart[L], w.pidx[L - 1]},
                  StartTotal{w.cstart[L]}, n_levels + L - 1, 0, w.partial, s);
    else
      device_scan(HeadIn<uint32_t, 3>{(const uint32_t*)levels[L - 1].keys}, ChildOut{w.cstart[L], w.pidx[L - 1]},
                  StartTotal{w.cstart[L]}, n_levels + L - 1, 0, w.partial, s);
  }
}

static int blocks_for(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 1 ? 1 : (b > kGrid ? kGrid : b));
}

template <class Key>
static void bind_check(const vx_voxels* levels, const int64_t* n_levels, int lo, int hi, const int64_t* rows,
                       const void* const* bound, int64_t* stats, hipStream_t s) {
  for (int L = lo; L <= hi; ++L)
    hipLaunchKernelGGL(k_fit_bind<Key>, dim3(blocks_for(rows[L - lo])), dim3(kBlock), 0, s,
                       (const Key*)levels[L].keys, n_levels + L, rows[L - lo],
                       bound ? (const Key*)bound[L - lo] : (const Key*)nullptr, stats);
}

vx_status fit_forward_run(const vx_grid* g, const vx_voxels* levels, const int64_t* n_levels, int lo, int hi,
                          const float* const* params, const int64_t* rows, const void* const* bound, const float* dirs,
                          int ndir, float* loss, int64_t* stats, void* ws, const int64_t* caps, hipStream_t s) {
  const bool key64 = g->log2_res > 10;
  FitWs w;
  fit_ws_layout(0, 0, 0, caps, hi, g->log2_res, ws, &w);
  launch_fill_i64(stats, VX_NSTAT, 0, s);
  if (key64) bind_check<uint64_t>(levels, n_levels, lo, hi, rows, bound, stats, s);
  else bind_check<uint32_t>(levels, n_levels, lo, hi, rows, bound, stats, s);
  child_starts(key64, levels, n_levels, hi, w, s);
  LossLevels ll;
  ll.count = 0;
  for (int L = lo; L <= hi; ++L) {
    VX_TIMED("fit_fwd", s);
    hipLaunchKernelGGL(k_fit_fwd, dim3(kGrid), dim3(kBlock), 0, s, levels[L], n_levels + L, rows[L - lo],
                       levels[L - 1], w.cstart[L], params[L - lo], dirs, ndir, w.loss_vox[L]);
    ll.p[ll.count] = w.loss_vox[L];
    ll.n[ll.count] = n_levels + L;
    ll.rows[ll.count] = rows[L - lo];
    ++ll.count;
  }
  VX_TIMED("fit_total", s);
  hipLaunchKernelGGL(k_fit_partial, dim3(kGrid), dim3(kBlock), 0, s, ll, w.part);
  hipLaunchKernelGGL(k_fit_total, dim3(1), dim3(1024), 0, s, w.part, loss);
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

// FP64 sums of levels 0..hi-1 from the re-emitted pairs (f.pa, emission order, left intact)
template <class Key>
static void level_sums64(const vx_grid* g, const vx_voxels* levels, const int64_t* n_levels, int hi,
                         const FitWs& w, const int64_t* caps, int64_t* stats, hipStream_t s) {
  VX_TIMED("fit_sums64", s);
  const int kb = int(sizeof(Key));
  hipLaunchKernelGGL(k_copy_pairs, dim3(kGrid), dim3(kBlock), 0, s, (const uint8_t*)w.f.pa.keys, w.f.pa.prim,
                     w.f.ctl, kb, (uint8_t*)w.pc.keys, w.pc.prim);
  const int res = radix_sort_pairs(kb == 8, 3 * g->log2_res, w.pc, w.pb, w.f.ctl + CTL_N_PAIRS, 0, w.hist,
                                   w.partial, s);
  const PairBufs P = res ? w.pb : w.pc;
  device_scan(HeadIn<Key, 0>{(const Key*)P.keys}, LeafSegOut{w.sstart, caps[0]},
              LeafSegTotal{w.sstart, caps[0], n_levels, stats}, w.f.ctl + CTL_N_PAIRS, 0, w.partial, s);
  const Lat lat = make_lat(g, 1, 0.0f);
  hipLaunchKernelGGL(k_fit_leaf64<Key>, dim3(kGrid), dim3(kBlock), 0, s, (const Key*)P.keys, P.prim, w.sstart,
                     w.f.rec, (const Key*)levels[0].keys, n_levels, caps[0], lat.Sb, g->log2_res, w.s64[0], stats);
  for (int L = 1; L < hi; ++L)
    hipLaunchKernelGGL(k_fit_up64, dim3(kGrid), dim3(kBlock), 0, s, w.cstart[L], n_levels + L, caps[L],
                       w.s64[L - 1], caps[L - 1], w.s64[L]);
}

vx_status fit_backward_run(const vx_grid* g, const float* pts, int64_t n_pts, const int64_t* offsets, int64_t n_fib,
                           float radius, int64_t max_cand, int64_t max_pairs, const vx_voxels* levels,
                           const int64_t* n_levels, int lo, int hi, const float* const* params, const int64_t* rows,
                           const void* const* bound, const float* dirs, int ndir, const float* dloss,
                           float* const* dparams, float* dpts, int64_t* stats, void* ws, const int64_t* caps,
                           hipStream_t s) {
  const bool key64 = g->log2_res > 10;
  FitWs w;
  fit_ws_layout(n_pts, max_cand, max_pairs, caps, hi, g->log2_res, ws, &w);
  for (int L = 0; L < hi; ++L)
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(7 * caps[L])), dim3(kBlock), 0, s, w.g[L], 7 * caps[L], 0.0);
  // re-emit the pairs in primitive order (this clears stats), then check the parameters' binding
  voxelize_front(1, g, pts, n_pts, offsets, n_fib, radius, max_cand, max_pairs, w.f, stats, s, nullptr);
  if (key64) bind_check<uint64_t>(levels, n_levels, lo, hi, rows, bound, stats, s);
  else bind_check<uint32_t>(levels, n_levels, lo, hi, rows, bound, stats, s);
  child_starts(key64, levels, n_levels, hi, w, s);
  // (no points: every level is empty and the FP64 sums, sized by the points, are not read)
  if (n_pts > 0) {
    if (key64) level_sums64<uint64_t>(g, levels, n_levels, hi, w, caps, stats, s);
    else level_sums64<uint32_t>(g, levels, n_levels, hi, w, caps, stats, s);
  }
  // lobe gradients and the children's (S, w) gradients, level by level
  for (int L = lo; L <= hi; ++L) {
    VX_TIMED("fit_bwd", s);
    if (ndir <= 128)
      hipLaunchKernelGGL(k_fit_bwd<8>, dim3(kGrid), dim3(kBlock), 0, s, levels[L], n_levels + L, rows[L - lo],
                         n_pts > 0 ? w.s64[L - 1] : nullptr, caps[L - 1], w.cstart[L], params[L - lo], dirs, ndir,
                         dloss, dparams[L - lo], w.g[L - 1], caps[L - 1]);
    else
      hipLaunchKernelGGL(k_fit_bwd<16>, dim3(kGrid), dim3(kBlock), 0, s, levels[L], n_levels + L, rows[L - lo],
                         n_pts > 0 ? w.s64[L - 1] : nullptr, caps[L - 1], w.cstart[L], params[L - lo], dirs, ndir,
                         dloss, dparams[L - lo], w.g[L - 1], caps[L - 1]);
  }
  // top-down accumulation to the leaf
  for (int L = hi - 2; L >= 0; --L) {
    VX_TIMED("fit_down", s);
    hipLaunchKernelGGL(k_fit_down, dim3(kGrid), dim3(kBlock), 0, s, w.pidx[L], n_levels + L, w.g[L], caps[L],
                       w.g[L + 1], caps[L + 1]);
  }
  // the chain rule per segment over its pairs (emission order) and per point
  const Lat lat = make_lat(g, 1, radius);
  const double vs = double(int64_t(1) << g->log2_res) / g->extent;
  const int64_t tiles = leaf_tiles(g->log2_res);
  if (tiles) {
    VX_TIMED("fit_tiles", s);
    launch_fill_i64(w.tfirst, tiles, 0, s);
    launch_fill_i64(w.tend, tiles, 0, s);
    if (key64)
      hipLaunchKernelGGL(k_tile_index<uint64_t>, dim3(kGrid), dim3(kBlock), 0, s, (const uint64_t*)levels[0].keys,
                         n_levels, w.tfirst, w.tend);
    else
      hipLaunchKernelGGL(k_tile_index<uint32_t>, dim3(kGrid), dim3(kBlock), 0, s, (const uint32_t*)levels[0].keys,
                         n_levels, w.tfirst, w.tend);
  }
  {
    VX_TIMED("fit_pairs", s);
    if (key64)
      hipLaunchKernelGGL(k_fit_pairs<uint64_t>, dim3(blocks_for(n_pts)), dim3(kBlock), 0, s, w.f.rec, w.f.cand_off,
                         n_pts, w.f.masks, w.f.wave_off, w.f.ctl, (const uint64_t*)w.f.pa.keys, levels[0], n_levels,
                         w.g[0], caps[0], lat.Sb, g->log2_res, vs, tiles ? w.tfirst : nullptr, w.tend, w.seg_grad);
    else
      hipLaunchKernelGGL(k_fit_pairs<uint32_t>, dim3(blocks_for(n_pts)), dim3(kBlock), 0, s, w.f.rec, w.f.cand_off,
                         n_pts, w.f.masks, w.f.wave_off, w.f.ctl, (const uint32_t*)w.f.pa.keys, levels[0], n_levels,
                         w.g[0], caps[0], lat.Sb, g->log2_res, vs, tiles ? w.tfirst : nullptr, w.tend, w.seg_grad);
  }
  {
    VX_TIMED("fit_points", s);
    hipLaunchKernelGGL(k_fit_points, dim3(blocks_for(n_pts)), dim3(kBlock), 0, s, w.seg_grad, n_pts, dpts);
  }
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

}  // namespace vx
