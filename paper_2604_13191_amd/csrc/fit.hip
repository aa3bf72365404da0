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

// children of parent key pk in the level below: [first, first + nc)
template <class Key>
__device__ __forceinline__ int child_range(const Key* ck, int64_t nch, uint64_t pk, int64_t& first) {
  first = key_lower_bound(ck, nch, pk << 3);
  int nc = 0;
  while (nc < kMaxChild && first + nc < nch && (uint64_t(ck[first + nc]) >> 3) == pk) ++nc;
  return nc;
}

// ---------------------------------------------------------------------------------------------
// forward: one wave per voxel, lanes over directions
// ---------------------------------------------------------------------------------------------
template <class Key>
__global__ void __launch_bounds__(kBlock) k_fit_fwd(vx_voxels par, const int64_t* n_par_p, vx_voxels ch,
                                                    const int64_t* n_ch_p, const float* __restrict__ Lp,
                                                    const float* __restrict__ dirs, int ndir,
                                                    float* __restrict__ loss_vox) {
  const int lane = lane_id();
  const int64_t n_par = *n_par_p, n_ch = *n_ch_p;
  const Key* pk = reinterpret_cast<const Key*>(par.keys);
  const Key* ck = reinterpret_cast<const Key*>(ch.keys);
  for (int64_t u = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6); u < n_par; u += int64_t(gridDim.x) * kWaves) {
    const float W = par.w[u];
    if (!(W > 0.f)) {
      if (lane == 0) loss_vox[u] = 0.f;
      continue;
    }
    int64_t first;
    const int nc = child_range(ck, n_ch, uint64_t(pk[u]), first);
    float cw[kMaxChild], cS[kMaxChild][6];
#pragma unroll
    for (int c = 0; c < kMaxChild; ++c) {
      cw[c] = c < nc ? ch.w[first + c] : 0.f;
#pragma unroll
      for (int t = 0; t < 6; ++t) cS[c][t] = c < nc ? ch.S[int64_t(t) * ch.cap + first + c] : 0.f;
    }
    float l[12];
    for (int t = 0; t < 12; ++t) l[t] = Lp[u * 12 + t];
    const float invW = 1.0f / W;
    float acc = 0.f;
    for (int k = lane; k < ndir; k += 64) {
      const float x = dirs[3 * k], y = dirs[3 * k + 1], z = dirs[3 * k + 2];
      float tau = 0.f;
#pragma unroll
      for (int c = 0; c < kMaxChild; ++c)
        if (c < nc && cw[c] > 0.f) tau += sqrtf(fmaxf(cw[c] * quadf(cS[c], x, y, z), 0.f));
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
    acc = wave_sum(acc);
    if (lane == 0) loss_vox[u] = acc / float(ndir);
  }
}

// deterministic sum of the per-voxel losses of all levels into loss[0] (one block)
struct LossLevels {
  const float* p[24];
  const int64_t* n[24];
  int count;
};

__global__ void __launch_bounds__(1024) k_fit_total(LossLevels lv, float* loss) {
  __shared__ float red[16];
  float acc = 0.f;
  for (int i = 0; i < lv.count; ++i) {
    const int64_t n = *lv.n[i];
    for (int64_t j = threadIdx.x; j < n; j += 1024) acc += lv.p[i][j];
  }
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
// gch: [7][gcap] (S components, then w) for the level below
// ---------------------------------------------------------------------------------------------
constexpr int kMaxDirPerLane = 4;     // up to 256 directions

__device__ __forceinline__ double quadd(const double* S, double x, double y, double z) {
  return S[0] * x * x + S[1] * y * y + S[2] * z * z + 2.0 * (S[3] * x * y + S[4] * x * z + S[5] * y * z);
}

template <class Key>
__global__ void __launch_bounds__(kBlock) k_fit_bwd(vx_voxels par, const int64_t* n_par_p, vx_voxels ch,
                                                    const int64_t* n_ch_p, const float* __restrict__ Lp,
                                                    const float* __restrict__ dirs, int ndir,
                                                    const float* __restrict__ dloss, float* __restrict__ dLp,
                                                    double* __restrict__ gch, int64_t gcap) {
  const int lane = lane_id();
  const int64_t n_par = *n_par_p, n_ch = *n_ch_p;
  const Key* pk = reinterpret_cast<const Key*>(par.keys);
  const Key* ck = reinterpret_cast<const Key*>(ch.keys);
  const double g0 = double(dloss[0]);
  for (int64_t u = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6); u < n_par; u += int64_t(gridDim.x) * kWaves) {
    const float Wf = par.w[u];
    if (!(Wf > 0.f)) {
      if (lane < 12) dLp[u * 12 + lane] = 0.f;
      continue;
    }
    int64_t first;
    const int nc = child_range(ck, n_ch, uint64_t(pk[u]), first);
    double l[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) l[t] = double(Lp[u * 12 + t]);
    const double invW = 1.0 / double(Wf);
    // pass 1 (lanes over directions): target, fit, residual; lobe gradients
    double dx[kMaxDirPerLane], dy[kMaxDirPerLane], dz[kMaxDirPerLane], dg[kMaxDirPerLane], dt[kMaxDirPerLane];
    double gl[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) gl[t] = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxDirPerLane; ++i) {
      const int k = lane + 64 * i;
      dg[i] = 0.0;
      dt[i] = 0.0;
      dx[i] = dy[i] = dz[i] = 0.0;
      if (k >= ndir) continue;
      const double x = dirs[3 * k], y = dirs[3 * k + 1], z = dirs[3 * k + 2];
      dx[i] = x;
      dy[i] = y;
      dz[i] = z;
      double tau = 0.0;
      for (int c = 0; c < nc; ++c) {
        const int64_t cc = first + c;
        const double wc = double(ch.w[cc]);
        if (!(wc > 0.0)) continue;
        double S[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) S[t] = double(ch.S[int64_t(t) * ch.cap + cc]);
        tau += sqrt(fmax(wc * quadd(S, x, y, z), 0.0));
      }
      tau *= invW;
      double f = 0.0, yv[2][3], ny[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double* lj = l + 6 * j;
        yv[j][0] = lj[0] * x + lj[1] * y + lj[3] * z;
        yv[j][1] = lj[2] * y + lj[4] * z;
        yv[j][2] = lj[5] * z;
        ny[j] = sqrt(yv[j][0] * yv[j][0] + yv[j][1] * yv[j][1] + yv[j][2] * yv[j][2]);
        f += ny[j];
      }
      const double g = 2.0 * (f - tau) / double(ndir) * g0;     // d loss / d f;  d loss / d tau = -g
      dg[i] = g;
      dt[i] = tau;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if (!(ny[j] > 0.0)) continue;
        const double s = g / ny[j];
        double* gj = gl + 6 * j;
        gj[0] += s * yv[j][0] * x;
        gj[1] += s * yv[j][0] * y;
        gj[2] += s * yv[j][1] * y;
        gj[3] += s * yv[j][0] * z;
        gj[4] += s * yv[j][1] * z;
        gj[5] += s * yv[j][2] * z;
      }
    }
#pragma unroll
    for (int t = 0; t < 12; ++t) {
      const double v = wave_sum(gl[t]);
      if (lane == t) dLp[u * 12 + t] = float(v);
    }
    // pass 2 (one child at a time): d loss / d (S_c, w_c)
    for (int c = 0; c < nc; ++c) {
      const int64_t cc = first + c;
      const double wc = double(ch.w[cc]);
      double S[6];
#pragma unroll
      for (int t = 0; t < 6; ++t) S[t] = double(ch.S[int64_t(t) * ch.cap + cc]);
      double acc[7] = {0, 0, 0, 0, 0, 0, 0};
      if (wc > 0.0) {
#pragma unroll
        for (int i = 0; i < kMaxDirPerLane; ++i) {
          if (lane + 64 * i >= ndir) continue;
          const double x = dx[i], y = dy[i], z = dz[i], g = dg[i];
          const double qs = quadd(S, x, y, z);
          const double q = sqrt(fmax(wc * qs, 0.0));
          double dw = -dt[i] * invW;
          if (q > 0.0) {
            const double k2 = -g * wc / (2.0 * q) * invW;      // d loss / d (w^T S_c w)
            acc[0] += k2 * x * x;
            acc[1] += k2 * y * y;
            acc[2] += k2 * z * z;
            acc[3] += k2 * 2.0 * x * y;
            acc[4] += k2 * 2.0 * x * z;
            acc[5] += k2 * 2.0 * y * z;
            dw += qs / (2.0 * q) * invW;
          }
          acc[6] += -g * dw;
        }
      }
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const double v = wave_sum(acc[t]);
        if (lane == t) gch[int64_t(t) * gcap + cc] = v;
      }
    }
  }
}

// top-down: every voxel of level L adds its parent's accumulated gradient (level L+1)
template <class Key>
__global__ void __launch_bounds__(kBlock) k_fit_down(vx_voxels lv, const int64_t* n_p, double* __restrict__ g,
                                                     int64_t gcap, vx_voxels up, const int64_t* n_up_p,
                                                     const double* __restrict__ gup, int64_t gupcap) {
  const int64_t n = *n_p, n_up = *n_up_p;
  const Key* k = reinterpret_cast<const Key*>(lv.keys);
  const Key* ku = reinterpret_cast<const Key*>(up.keys);
  for (int64_t c = int64_t(blockIdx.x) * kBlock + threadIdx.x; c < n; c += int64_t(gridDim.x) * kBlock) {
    const int64_t p = key_lower_bound(ku, n_up, uint64_t(k[c]) >> 3);
    if (p >= n_up) continue;
    for (int t = 0; t < 7; ++t) g[int64_t(t) * gcap + c] += gup[int64_t(t) * gupcap + p];
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
                                                      int log2R, double vs, float* __restrict__ seg_grad) {
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
        const int64_t v = key_lower_bound(lk, n_leaf, key);
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
      seg_grad[p * 6 + a] = float(gA[a] * vs);
      seg_grad[p * 6 + 3 + a] = float(gB[a] * vs);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_fit_points(const float* __restrict__ seg_grad, int64_t n,
                                                       float* __restrict__ dpts) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    for (int a = 0; a < 3; ++a)
      dpts[i * 3 + a] = seg_grad[i * 6 + a] + (i > 0 ? seg_grad[(i - 1) * 6 + 3 + a] : 0.f);
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------------------------
// orchestration
// ---------------------------------------------------------------------------------------------
struct FitWs {
  float* loss_vox[21];
  double* g[21];           // [7][cap_L] per level 0..hi-1
  float* seg_grad;         // [n_pts][6]
  FrontWs f;
};

static size_t fit_ws_layout(int64_t n_pts, int64_t max_cand, int64_t max_pairs, const int64_t* caps, int hi,
                            bool key64, void* base, FitWs* w) {
  Carver cv(base);
  FitWs x;
  for (int L = 0; L <= hi; ++L) x.loss_vox[L] = cv.take<float>(caps[L]);
  for (int L = 0; L < hi; ++L) x.g[L] = cv.take<double>(7 * caps[L]);
  x.seg_grad = cv.take<float>(6 * n_pts);
  front_ws_carve(cv, n_pts, max_cand, max_pairs, key64, &x.f);
  if (w) *w = x;
  return cv.off + 256;
}

size_t fit_ws_bytes(int64_t n_pts, int64_t max_cand, int64_t max_pairs, const int64_t* caps, int hi, bool key64) {
  return fit_ws_layout(n_pts, max_cand, max_pairs, caps, hi, key64, nullptr, nullptr);
}

static int blocks_for(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 1 ? 1 : (b > kGrid ? kGrid : b));
}

vx_status fit_forward_run(const vx_grid* g, const vx_voxels* levels, const int64_t* n_levels, int lo, int hi,
                          const float* const* params, const float* dirs, int ndir, float* loss, void* ws,
                          const int64_t* caps, hipStream_t s) {
  const bool key64 = g->log2_res > 10;
  FitWs w;
  fit_ws_layout(0, 0, 0, caps, hi, key64, ws, &w);
  LossLevels ll;
  ll.count = 0;
  for (int L = lo; L <= hi; ++L) {
    VX_TIMED("fit_fwd", s);
#define VX_FWD(K)                                                                                              \
  hipLaunchKernelGGL(k_fit_fwd<K>, dim3(kGrid), dim3(kBlock), 0, s, levels[L], n_levels + L, levels[L - 1],      \
                     n_levels + L - 1, params[L - lo], dirs, ndir, w.loss_vox[L])
    if (key64) VX_FWD(uint64_t); else VX_FWD(uint32_t);
#undef VX_FWD
    ll.p[ll.count] = w.loss_vox[L];
    ll.n[ll.count] = n_levels + L;
    ++ll.count;
  }
  VX_TIMED("fit_total", s);
  hipLaunchKernelGGL(k_fit_total, dim3(1), dim3(1024), 0, s, ll, loss);
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

vx_status fit_backward_run(const vx_grid* g, const float* pts, int64_t n_pts, const int64_t* offsets, int64_t n_fib,
                           float radius, int64_t max_cand, int64_t max_pairs, const vx_voxels* levels,
                           const int64_t* n_levels, int lo, int hi, const float* const* params, const float* dirs,
                           int ndir, const float* dloss, float* const* dparams, float* dpts, int64_t* stats,
                           void* ws, const int64_t* caps, hipStream_t s) {
  const bool key64 = g->log2_res > 10;
  FitWs w;
  fit_ws_layout(n_pts, max_cand, max_pairs, caps, hi, key64, ws, &w);
  for (int L = 0; L < hi; ++L)
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(7 * caps[L])), dim3(kBlock), 0, s, w.g[L], 7 * caps[L], 0.0);
  // lobe gradients and the children's (S, w) gradients, level by level
  for (int L = lo; L <= hi; ++L) {
    VX_TIMED("fit_bwd", s);
#define VX_BWD(K)                                                                                              \
  hipLaunchKernelGGL(k_fit_bwd<K>, dim3(kGrid), dim3(kBlock), 0, s, levels[L], n_levels + L, levels[L - 1],      \
                     n_levels + L - 1, params[L - lo], dirs, ndir, dloss, dparams[L - lo], w.g[L - 1], caps[L - 1])
    if (key64) VX_BWD(uint64_t); else VX_BWD(uint32_t);
#undef VX_BWD
  }
  // top-down accumulation to the leaf
  for (int L = hi - 2; L >= 0; --L) {
    VX_TIMED("fit_down", s);
    if (key64)
      hipLaunchKernelGGL(k_fit_down<uint64_t>, dim3(kGrid), dim3(kBlock), 0, s, levels[L], n_levels + L, w.g[L],
                         caps[L], levels[L + 1], n_levels + L + 1, w.g[L + 1], caps[L + 1]);
    else
      hipLaunchKernelGGL(k_fit_down<uint32_t>, dim3(kGrid), dim3(kBlock), 0, s, levels[L], n_levels + L, w.g[L],
                         caps[L], levels[L + 1], n_levels + L + 1, w.g[L + 1], caps[L + 1]);
  }
  // re-emit the pairs in primitive order, then the chain rule per segment and per point
  voxelize_front(1, g, pts, n_pts, offsets, n_fib, radius, max_cand, max_pairs, w.f, stats, s, nullptr);
  const Lat lat = make_lat(g, 1, radius);
  const double vs = double(int64_t(1) << g->log2_res) / g->extent;
  {
    VX_TIMED("fit_pairs", s);
    if (key64)
      hipLaunchKernelGGL(k_fit_pairs<uint64_t>, dim3(blocks_for(n_pts)), dim3(kBlock), 0, s, w.f.rec, w.f.cand_off,
                         n_pts, w.f.masks, w.f.wave_off, w.f.ctl, (const uint64_t*)w.f.pa.keys, levels[0], n_levels,
                         w.g[0], caps[0], lat.Sb, g->log2_res, vs, w.seg_grad);
    else
      hipLaunchKernelGGL(k_fit_pairs<uint32_t>, dim3(blocks_for(n_pts)), dim3(kBlock), 0, s, w.f.rec, w.f.cand_off,
                         n_pts, w.f.masks, w.f.wave_off, w.f.ctl, (const uint32_t*)w.f.pa.keys, levels[0], n_levels,
                         w.g[0], caps[0], lat.Sb, g->log2_res, vs, w.seg_grad);
  }
  {
    VX_TIMED("fit_points", s);
    hipLaunchKernelGGL(k_fit_points, dim3(blocks_for(n_pts)), dim3(kBlock), 0, s, w.seg_grad, n_pts, dpts);
  }
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

}  // namespace vx
