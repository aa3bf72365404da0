// compact.hip -- leaf eigen-fit and the 6-byte compact SGGX code, and its decoding.
//
// Per voxel with w > 0 the normalised SGGX M = S / w is diagonalised (Sec. 4.1: eigenvectors
// w_1..w_3, eigenvalues = the projected areas sigma(w_i)); the eigenvalues are floored at
// eps * lambda_1 so that a voxel of nearly one orientation still has a well-defined SGGX, and
// the matrix is rebuilt as (w_1 w_2 w_3) diag(lambda) (w_1 w_2 w_3)^T (Sec. 4.1, the SGGX
// from the fit).  The rebuilt matrix is scaled so that its largest diagonal entry is 1 and
// stored in Sec. 4.3's compact form: sigma_a = sqrt(S_aa) as rint(255 sigma), correlations
// r_ab = S_ab / sqrt(S_aa S_bb) as 128 + rint(127 r).  Voxels with w <= 0 get the isotropic
// SGGX.
//
// One thread per voxel, all arithmetic in FP64: cyclic Jacobi rotations on the 3x3 matrix
// (each zeroes one off-diagonal entry), until the off-diagonal part is below 2^-52 of the
// diagonal or after 12 sweeps.  Quotients and square roots use the hardware reciprocal and
// reciprocal-square-root estimates refined by Newton steps.  The kernel streams 28 bytes in and up to 82 bytes out per
// voxel, so it is bound by HBM once the rotations are cheap enough.
#include "vx_internal.hpp"

namespace vx {
namespace {

constexpr int kCBlock = 256;
constexpr int kCGrid = 4096;
constexpr int kMaxSweeps = 12;

// 1/x and 1/sqrt(x) from the hardware estimates plus Newton steps (a few ulp; the rotations and
// the code need no correctly rounded quotient)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x * r;
  return fma(r, fma(-h, r, 0.5), r);
}

// rotation in the (P, Q) plane that zeroes a[P][Q]; V accumulates the rotations by columns
template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(double (&a)[3][3], double (&V)[3][3], double skip) {
  constexpr int R = 3 - P - Q;
  const double apq = a[P][Q];
  if (!(fabs(apq) > skip)) return;        // already negligible against the diagonal
  // tangent of the rotation angle, the smaller root of t^2 + 2 theta t - 1 = 0 with
  // theta = d / (2 a_pq): t = 2 a_pq sgn(d) / (|d| + sqrt(d^2 + 4 a_pq^2)), one quotient
  const double d = a[Q][Q] - a[P][P];
  const double q = fma(d, d, 4.0 * apq * apq);
  const double t = (d < 0.0 ? -2.0 * apq : 2.0 * apq) * rcp_nr(fabs(d) + q * rsqrt_nr(q));
  const double c = rsqrt_nr(fma(t, t, 1.0));
  const double s = t * c;
  a[P][P] -= t * apq;
  a[Q][Q] += t * apq;
  a[P][Q] = a[Q][P] = 0.0;
  const double arp = a[R][P], arq = a[R][Q];
  a[R][P] = a[P][R] = c * arp - s * arq;
  a[R][Q] = a[Q][R] = s * arp + c * arq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vp = V[k][P], vq = V[k][Q];
    V[k][P] = c * vp - s * vq;
    V[k][Q] = s * vp + c * vq;
  }
}

template <int I, int J>
__device__ __forceinline__ void order_pair(double (&d)[3], double (&V)[3][3]) {
  if (d[J] > d[I]) {
    const double x = d[I];
    d[I] = d[J];
    d[J] = x;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double y = V[k][I];
      V[k][I] = V[k][J];
      V[k][J] = y;
    }
  }
}

template <int J>
__device__ __forceinline__ void fix_sign(double (&V)[3][3]) {
  int big = 0;
  if (fabs(V[1][J]) > fabs(V[big][J])) big = 1;
  if (fabs(V[2][J]) > fabs(V[big][J])) big = 2;
  const double v = big == 0 ? V[0][J] : (big == 1 ? V[1][J] : V[2][J]);
  if (v < 0.0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) V[k][J] = -V[k][J];
  }
}

__device__ __forceinline__ uint32_t sigma_code(double x) {   // x = S_aa / max diagonal, in (0, 1]
  const double q = x > 0.0 ? rint(255.0 * (x * rsqrt_nr(x))) : 0.0;
  return uint32_t(fmin(fmax(q, 0.0), 255.0));
}

__device__ __forceinline__ uint32_t corr_code(double sab, double saa, double sbb) {
  const double q = 128.0 + rint(127.0 * (sab * rsqrt_nr(saa * sbb)));
  return uint32_t(fmin(fmax(q, 1.0), 255.0));
}

__global__ void __launch_bounds__(kCBlock) k_sggx_compact(const float* __restrict__ w, const float* __restrict__ S,
                                                         const int64_t* __restrict__ n_dev, int64_t cap, double eps,
                                                         float* __restrict__ lam, float* __restrict__ vec,
                                                         uint16_t* __restrict__ code) {
  const int64_t n = min(*n_dev, cap);
  for (int64_t v = int64_t(blockIdx.x) * kCBlock + threadIdx.x; v < n; v += int64_t(gridDim.x) * kCBlock) {
    double a[3][3], V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
    double d[3] = {1.0, 1.0, 1.0};
    const double wv = w[v];
    bool iso = !(wv > 0.0);
    if (!iso) {
      const double rw = rcp_nr(wv);
      a[0][0] = double(S[v]) * rw;
      a[1][1] = double(S[cap + v]) * rw;
      a[2][2] = double(S[2 * cap + v]) * rw;
      a[0][1] = a[1][0] = double(S[3 * cap + v]) * rw;
      a[0][2] = a[2][0] = double(S[4 * cap + v]) * rw;
      a[1][2] = a[2][1] = double(S[5 * cap + v]) * rw;
      for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        const double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        const double diag = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]);
        if (!(off > 0x1p-52 * diag)) break;
        // entries below 2^-56 of the diagonal are left alone (their sum stays under the stop
        // level); the floor 2^-500 keeps 4 a_pq^2 a normal number, so every quotient of a
        // rotation is finite
        const double skip = fmax(0x1p-56 * diag, 0x1p-500);
        jacobi_rotate<0, 1>(a, V, skip);
        jacobi_rotate<0, 2>(a, V, skip);
        jacobi_rotate<1, 2>(a, V, skip);
      }
      d[0] = a[0][0];
      d[1] = a[1][1];
      d[2] = a[2][2];
      order_pair<0, 1>(d, V);
      order_pair<0, 2>(d, V);
      order_pair<1, 2>(d, V);
      if (d[0] > 0.0) {
        fix_sign<0>(V);
        fix_sign<1>(V);
        fix_sign<2>(V);
        const double fl = eps * d[0];
        d[1] = fmax(d[1], fl);
        d[2] = fmax(d[2], fl);
      } else {
        iso = true;
      }
    }
    if (iso) {
      d[0] = d[1] = d[2] = 1.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) V[k][i] = i == k ? 1.0 : 0.0;
    }
    // rebuilt matrix, entries xx yy zz xy xz yz
    double f[6];
    f[0] = d[0] * V[0][0] * V[0][0] + d[1] * V[0][1] * V[0][1] + d[2] * V[0][2] * V[0][2];
    f[1] = d[0] * V[1][0] * V[1][0] + d[1] * V[1][1] * V[1][1] + d[2] * V[1][2] * V[1][2];
    f[2] = d[0] * V[2][0] * V[2][0] + d[1] * V[2][1] * V[2][1] + d[2] * V[2][2] * V[2][2];
    f[3] = d[0] * V[0][0] * V[1][0] + d[1] * V[0][1] * V[1][1] + d[2] * V[0][2] * V[1][2];
    f[4] = d[0] * V[0][0] * V[2][0] + d[1] * V[0][1] * V[2][1] + d[2] * V[0][2] * V[2][2];
    f[5] = d[0] * V[1][0] * V[2][0] + d[1] * V[1][1] * V[2][1] + d[2] * V[1][2] * V[2][2];
    if (lam) {
#pragma unroll
      for (int i = 0; i < 3; ++i) lam[i * cap + v] = float(d[i]);
    }
    if (vec) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) vec[(3 * i + c) * cap + v] = float(V[c][i]);
    }
    const double mx = fmax(f[0], fmax(f[1], f[2]));
    const double rmx = rcp_nr(mx);
    const uint32_t b0 = sigma_code(f[0] * rmx), b1 = sigma_code(f[1] * rmx), b2 = sigma_code(f[2] * rmx);
    const uint32_t b3 = corr_code(f[3], f[0], f[1]), b4 = corr_code(f[4], f[0], f[2]), b5 = corr_code(f[5], f[1], f[2]);
    code[3 * v] = uint16_t(b0 | (b1 << 8));
    code[3 * v + 1] = uint16_t(b2 | (b3 << 8));
    code[3 * v + 2] = uint16_t(b4 | (b5 << 8));
  }
}

__global__ void __launch_bounds__(kCBlock) k_sggx_decode(const uint16_t* __restrict__ code,
                                                        const int64_t* __restrict__ n_dev, int64_t cap,
                                                        float* __restrict__ S) {
  static_assert(kCBlock == 256, "one table entry per thread");
  __shared__ double sig_t[256], cor_t[256];     // b / 255 and (b - 128) / 127, correctly rounded
  sig_t[threadIdx.x] = double(threadIdx.x) / 255.0;
  cor_t[threadIdx.x] = (double(threadIdx.x) - 128.0) / 127.0;
  __syncthreads();
  const int64_t n = min(*n_dev, cap);
  for (int64_t v = int64_t(blockIdx.x) * kCBlock + threadIdx.x; v < n; v += int64_t(gridDim.x) * kCBlock) {
    const uint32_t h0 = code[3 * v], h1 = code[3 * v + 1], h2 = code[3 * v + 2];
    const double sx = sig_t[h0 & 255u], sy = sig_t[h0 >> 8], sz = sig_t[h1 & 255u];
    const double rxy = cor_t[h1 >> 8], rxz = cor_t[h2 & 255u], ryz = cor_t[h2 >> 8];
    S[v] = float(sx * sx);
    S[cap + v] = float(sy * sy);
    S[2 * cap + v] = float(sz * sz);
    S[3 * cap + v] = float(rxy * sx * sy);
    S[4 * cap + v] = float(rxz * sx * sz);
    S[5 * cap + v] = float(ryz * sy * sz);
  }
}

int compact_grid(int64_t cap) {
  const int64_t b = (cap + kCBlock - 1) / kCBlock;
  return int(b < 1 ? 1 : (b > kCGrid ? kCGrid : b));
}

}  // namespace

void sggx_compact_run(const float* w, const float* S, const int64_t* n, int64_t cap, double eps, float* lam,
                      float* vec, uint8_t* code, hipStream_t s) {
  VX_TIMED("sggx_compact", s);
  hipLaunchKernelGGL(k_sggx_compact, dim3(compact_grid(cap)), dim3(kCBlock), 0, s, w, S, n, cap, eps, lam, vec,
                     reinterpret_cast<uint16_t*>(code));
}

void sggx_decode_run(const uint8_t* code, const int64_t* n, int64_t cap, float* S, hipStream_t s) {
  VX_TIMED("sggx_decode", s);
  hipLaunchKernelGGL(k_sggx_decode, dim3(compact_grid(cap)), dim3(kCBlock), 0, s,
                     reinterpret_cast<const uint16_t*>(code), n, cap, S);
}

}  // namespace vx
