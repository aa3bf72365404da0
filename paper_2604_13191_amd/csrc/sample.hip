// sample.hip -- the paper's sampling voxelizer (Sec. 3.2), a baseline for the exact path.
//
// Points are generated on the primitives from kernel indices (no random numbers) and each is
// stored in the voxel that contains it:
//   * fibers: the uniform Catmull-Rom span of every segment (control points i-1 .. i+2, the
//     fiber's end points repeated) cut at t = j / m into m chords, n samples per chord at
//     fractions (k + 1/2) / n, each weighing chord length / n along the chord's tangent;
//   * triangles: max(1, floor(N A / A_max)) samples per triangle (in proportion to its area
//     relative to the largest), sample k at ((k + 1/2) / n_T, radical inverse of k) mapped to
//     barycentric coordinates by Heitz's low-distortion triangle map, each weighing A / n_T.
// Per voxel: the number of samples, their weight and their moments (n n^T or I - t t^T), summed
// in sample order.  Positions are FP64 in grid units with the operation order fixed (no
// contraction, explicit fused multiply-adds), so every sample's voxel is reproducible; samples
// outside the grid get a key above every voxel's and are dropped after the sort.
#pragma clang fp contract(off)

#include "vx_internal.hpp"

namespace vx {
namespace {

enum { SC_TOTAL = 0, SC_SEGS = 1, SC_VOX = 2, SC_QMAX = 3, SC_INSIDE = 4, SC_OUTSIDE = 5 };

struct SampWs {
  int64_t* ctl;       // [8] (SC_*)
  int64_t* cnt;       // [n_prims + 1] samples per primitive, then their offsets
  double* q;          // triangles: [n] squared twice-area
  float4* dirs;       // fibers: [n_pts * m] chord tangent and length; triangles: [n] normal and area
  PairBufs a, b;      // samples (key, weight, chord or triangle id), ping-pong for the sort
  int32_t* hist;
  int64_t* partial;
  int64_t* start;     // [max_vox + 2] first sample of every key
};

size_t samp_ws_layout(int kind, int64_t n_prims, int64_t max_samples, int64_t max_vox, bool key64, int sub,
                      void* base, SampWs* w) {
  Carver cv(base);
  SampWs x;
  x.ctl = cv.take<int64_t>(8);
  x.cnt = cv.take<int64_t>(n_prims + 1);
  x.q = cv.take<double>(kind == 0 ? n_prims : 1);
  x.dirs = cv.take<float4>(kind == 0 ? n_prims : n_prims * int64_t(sub));
  const int kb = key64 ? 8 : 4;
  for (PairBufs* p : {&x.a, &x.b}) {
    p->keys = cv.take<uint8_t>(max_samples * kb);
    p->w = cv.take<float>(max_samples);
    p->prim = cv.take<uint32_t>(max_samples);
  }
  x.hist = cv.take<int32_t>(int64_t(kRadixBuckets) * kGrid);
  x.partial = cv.take<int64_t>(kGrid + 1);
  x.start = cv.take<int64_t>(max_vox + 2);
  if (w) *w = x;
  return cv.off + 256;
}

struct Grid64 {
  double bmin[3];
  double vs;       // grid units per world unit, R / extent
  int64_t R;
};

__device__ __forceinline__ void to_grid(const float* p, const Grid64& G, double g[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) g[a] = (double(p[a]) - G.bmin[a]) * G.vs;
}

// the key of grid point X, or `outside` when X lies outside [0, R)^3
template <class Key>
__device__ __forceinline__ Key sample_key(const double X[3], const Grid64& G, Key outside) {
  uint32_t v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = floor(X[a]);
    if (!(f >= 0.0 && f < double(G.R))) return outside;
    v[a] = uint32_t(f);
  }
  return Key(morton3(v[0], v[1], v[2]));
}

__device__ __forceinline__ bool finite3(const float* p) {
  return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]);
}
__device__ __forceinline__ void flag_input(int64_t* stats) {
  atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_INPUT);
}
// samples that fell outside the grid, one atomic per wave
__device__ __forceinline__ void add_outside(int64_t n, int64_t* ctl) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if (lane_id() == 0 && n) atomicAdd(reinterpret_cast<unsigned long long*>(ctl + SC_OUTSIDE), (unsigned long long)n);
}

// offsets: 0 first, non-decreasing, n_pts last
__global__ void k_samp_offsets(const int64_t* __restrict__ off, int64_t F, int64_t n_pts, int64_t* stats) {
  for (int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; f <= F; f += int64_t(gridDim.x) * blockDim.x) {
    bool bad = f == 0 ? off[0] != 0 : off[f] < off[f - 1];
    if (f == F) bad = bad || off[F] != n_pts;
    if (bad)
      atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_OFFSETS);
  }
}

// the Catmull-Rom span of segment (i, i+1) of a fiber [a, b): polynomial coefficients
__device__ __forceinline__ void span_coeffs(const float* __restrict__ pts, int64_t i, int64_t a, int64_t b,
                                            const Grid64& G, double c[4][3]) {
  double P[4][3];
  to_grid(pts + 3 * (i > a ? i - 1 : i), G, P[0]);
  to_grid(pts + 3 * i, G, P[1]);
  to_grid(pts + 3 * (i + 1), G, P[2]);
  to_grid(pts + 3 * (i + 2 < b ? i + 2 : i + 1), G, P[3]);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    c[0][x] = P[1][x];
    c[1][x] = 0.5 * (P[2][x] - P[0][x]);
    c[2][x] = ((P[0][x] - 2.5 * P[1][x]) + 2.0 * P[2][x]) - 0.5 * P[3][x];
    c[3][x] = 0.5 * (P[3][x] - P[0][x]) + 1.5 * (P[1][x] - P[2][x]);
  }
}

__device__ __forceinline__ void span_point(const double c[4][3], double t, double out[3]) {
#pragma unroll
  for (int x = 0; x < 3; ++x) out[x] = fma(fma(fma(c[3][x], t, c[2][x]), t, c[1][x]), t, c[0][x]);
}

// fiber [a, b) holding point i (offsets non-decreasing): the last f with offsets[f] <= i
__device__ __forceinline__ int64_t fiber_of(const int64_t* __restrict__ off, int64_t F, int64_t i) {
  int64_t lo = 0, hi = F;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// per point: the samples of its segment (m * n, or 0 when the point ends its fiber) and the
// chords' tangents and lengths
__global__ void __launch_bounds__(kBlock) k_samp_fib_count(const float* __restrict__ pts, int64_t n_pts,
                                                           const int64_t* __restrict__ off, int64_t F, int sub,
                                                           int per, Grid64 G, int64_t* __restrict__ cnt,
                                                           float4* __restrict__ dirs, int64_t* stats) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_pts; i += int64_t(gridDim.x) * kBlock) {
    const int64_t f = fiber_of(off, F, i);
    const int64_t a = off[f], b = off[f + 1];
    const bool seg = a >= 0 && i >= a && i + 1 < b && b <= n_pts;   // in bounds whatever the offsets hold
    cnt[i] = seg ? int64_t(sub) * per : 0;
    if (!seg) continue;
    if (!finite3(pts + 3 * i) || !finite3(pts + 3 * (i + 1))) flag_input(stats);
    double c[4][3];
    span_coeffs(pts, i, a, b, G, c);
    for (int j = 0; j < sub; ++j) {
      double A[3], B[3];
      span_point(c, double(j) / double(sub), A);
      span_point(c, double(j + 1) / double(sub), B);
      const double d0 = B[0] - A[0], d1 = B[1] - A[1], d2 = B[2] - A[2];
      const double len = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double il = len > 0.0 ? 1.0 / len : 0.0;
      dirs[i * sub + j] = make_float4(float(d0 * il), float(d1 * il), float(d2 * il), float(len));
    }
  }
}

template <class Key>
__global__ void __launch_bounds__(kBlock) k_samp_fib_emit(const float* __restrict__ pts, int64_t n_pts,
                                                          const int64_t* __restrict__ off, int64_t F, int sub,
                                                          int per, Grid64 G, const int64_t* __restrict__ soff,
                                                          int64_t* __restrict__ ctl, int64_t cap, Key outside,
                                                          Key* __restrict__ keys, float* __restrict__ wts,
                                                          uint32_t* __restrict__ ids) {
  if (ctl[SC_TOTAL] > cap) return;                  // over capacity: nothing is written
  int64_t outs = 0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_pts; i += int64_t(gridDim.x) * kBlock) {
    if (soff[i + 1] == soff[i]) continue;
    const int64_t f = fiber_of(off, F, i);
    const int64_t a = off[f], b = off[f + 1];
    double c[4][3];
    span_coeffs(pts, i, a, b, G, c);
    int64_t o = soff[i];
    for (int j = 0; j < sub; ++j) {
      double A[3], B[3], d[3];
      span_point(c, double(j) / double(sub), A);
      span_point(c, double(j + 1) / double(sub), B);
#pragma unroll
      for (int x = 0; x < 3; ++x) d[x] = B[x] - A[x];
      const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      const float wk = float(len / double(per));
      const uint32_t id = uint32_t(i * sub + j);
      for (int k = 0; k < per; ++k) {
        const double fr = (double(k) + 0.5) / double(per);
        double X[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) X[x] = fma(fr, d[x], A[x]);
        const Key key = sample_key<Key>(X, G, outside);
        outs += key == outside;
        keys[o] = key;
        wts[o] = wk;
        ids[o] = id;
        ++o;
      }
    }
  }
  add_outside(outs, ctl);
}

__device__ __forceinline__ void tri_grid(const float* __restrict__ tris, int64_t t, const Grid64& G, double g[3][3],
                                         double c[3]) {
#pragma unroll
  for (int v = 0; v < 3; ++v) to_grid(tris + 9 * t + 3 * v, G, g[v]);
  double e0[3], e1[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    e0[x] = g[1][x] - g[0][x];
    e1[x] = g[2][x] - g[0][x];
  }
  c[0] = e0[1] * e1[2] - e0[2] * e1[1];
  c[1] = e0[2] * e1[0] - e0[0] * e1[2];
  c[2] = e0[0] * e1[1] - e0[1] * e1[0];
}

// squared twice-areas and their maximum (non-negative doubles order like their bits)
__global__ void __launch_bounds__(kBlock) k_samp_tri_q(const float* __restrict__ tris, int64_t n, Grid64 G,
                                                       double* __restrict__ q, int64_t* __restrict__ ctl,
                                                       int64_t* stats) {
  __shared__ uint64_t red[kWaves];
  uint64_t best = 0;
  for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t < n; t += int64_t(gridDim.x) * kBlock) {
    double g[3][3], c[3];
    tri_grid(tris, t, G, g, c);
    double qq = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    if (!finite3(tris + 9 * t) || !finite3(tris + 9 * t + 3) || !finite3(tris + 9 * t + 6) || !isfinite(qq)) {
      flag_input(stats);
      qq = 0.0;
    }
    q[t] = qq;
    const uint64_t b = qq > 0.0 ? uint64_t(__double_as_longlong(qq)) : 0ull;
    best = b > best ? b : best;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t u = uint64_t(__shfl_xor((unsigned long long)best, o, 64));
    best = u > best ? u : best;
  }
  if (lane_id() == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t m = 0;
    for (int i = 0; i < kWaves; ++i) m = red[i] > m ? red[i] : m;
    atomicMax(reinterpret_cast<unsigned long long*>(ctl + SC_QMAX), (unsigned long long)m);
  }
}

// max(1, floor(N sqrt(q / qmax))): the guess from the square root, settled on products
__device__ __forceinline__ int64_t tri_samples(double q, double qmax, int N) {
  if (!(qmax > 0.0)) return 1;
  const double nn = double(N) * double(N) * q;
  int64_t k = int64_t(floor(double(N) * sqrt(q / qmax)));
  if (k < 0) k = 0;
  while (double(k + 1) * double(k + 1) * qmax <= nn) ++k;
  while (k > 0 && double(k) * double(k) * qmax > nn) --k;
  return k > 1 ? k : 1;
}

__global__ void __launch_bounds__(kBlock) k_samp_tri_count(const float* __restrict__ tris, int64_t n, Grid64 G, int N,
                                                           const double* __restrict__ q,
                                                           const int64_t* __restrict__ ctl,
                                                           int64_t* __restrict__ cnt, float4* __restrict__ dirs) {
  const double qmax = __longlong_as_double((long long)ctl[SC_QMAX]);
  for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t < n; t += int64_t(gridDim.x) * kBlock) {
    cnt[t] = tri_samples(q[t], qmax, N);
    double g[3][3], c[3];
    tri_grid(tris, t, G, g, c);
    const double a2 = sqrt(q[t]);
    const double ia = a2 > 0.0 ? 1.0 / a2 : 0.0;
    dirs[t] = make_float4(float(c[0] * ia), float(c[1] * ia), float(c[2] * ia), float(0.5 * a2));
  }
}

__device__ __forceinline__ double radical_inverse2(uint32_t k) { return double(__brev(k)) * 0x1p-32; }

template <class Key>
__global__ void __launch_bounds__(kBlock) k_samp_tri_emit(const float* __restrict__ tris, int64_t n, Grid64 G,
                                                          const double* __restrict__ q,
                                                          const int64_t* __restrict__ soff,
                                                          int64_t* __restrict__ ctl, int64_t cap, Key outside,
                                                          Key* __restrict__ keys, float* __restrict__ wts,
                                                          uint32_t* __restrict__ ids) {
  if (ctl[SC_TOTAL] > cap) return;
  int64_t outs = 0;
  for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t < n; t += int64_t(gridDim.x) * kBlock) {
    const int64_t o0 = soff[t], nt = soff[t + 1] - o0;
    double g[3][3], c[3];
    tri_grid(tris, t, G, g, c);
    double d0[3], d1[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      d0[x] = g[0][x] - g[2][x];
      d1[x] = g[1][x] - g[2][x];
    }
    const float wk = float(0.5 * sqrt(q[t]) / double(nt));
    for (int64_t k = 0; k < nt; ++k) {
      const double u1 = (double(k) + 0.5) / double(nt);
      const double u2 = radical_inverse2(uint32_t(k));
      // Heitz's map, both halves by selects
      const bool up = u2 > u1;
      const double h1 = 0.5 * u1, h2 = 0.5 * u2;
      const double b0 = up ? h1 : u1 - h2;
      const double b1 = up ? u2 - h1 : h2;
      double X[3];
#pragma unroll
      for (int x = 0; x < 3; ++x) X[x] = fma(b0, d0[x], fma(b1, d1[x], g[2][x]));
      const Key key = sample_key<Key>(X, G, outside);
      outs += key == outside;
      keys[o0 + k] = key;
      wts[o0 + k] = wk;
      ids[o0 + k] = uint32_t(t);
    }
  }
  add_outside(outs, ctl);
}

struct SampTotal {
  int64_t* ctl;
  int64_t* stats;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    ctl[SC_TOTAL] = total;
    stats[VX_STAT_CAND] = total;
    if (total > cap) {
      atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_PAIR_CAPACITY);
    }
    (void)n;
  }
};
struct CntOut {
  int64_t* o;
  __device__ void operator()(int64_t i, int64_t ex, int64_t) const { o[i] = ex; }
};
struct CntIn {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};
// the sort's element count: the samples, or none when they did not fit
__global__ void k_samp_n(int64_t* ctl, int64_t cap) {
  if (threadIdx.x == 0) ctl[SC_INSIDE] = ctl[SC_TOTAL] <= cap ? ctl[SC_TOTAL] : 0;
}
struct SegOut {
  int64_t* start;
  int64_t cap;   // entries of start: the voxels' cap + 2
  __device__ void operator()(int64_t i, int64_t ex, int64_t v) const {
    if (v && ex < cap) start[ex] = i;
  }
};
struct SegTotal {
  int64_t* start;
  int64_t* ctl;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    if (total < cap) start[total] = n;
    ctl[SC_SEGS] = total;
  }
};

// voxels = key segments, less the trailing one of samples outside the grid
__global__ void k_samp_finish(int64_t* ctl, int64_t* stats, int64_t vcap) {
  if (threadIdx.x != 0) return;
  const int64_t out = ctl[SC_OUTSIDE];
  const int64_t nv = ctl[SC_SEGS] - (out > 0);
  stats[VX_STAT_PAIRS] = ctl[SC_INSIDE] - out;
  stats[VX_STAT_VOXELS] = nv;
  if (nv > vcap)
    atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)VX_FLAG_VOXEL_CAPACITY);
  ctl[SC_VOX] = nv <= vcap ? nv : 0;
}

template <int KIND, class Key>
__global__ void __launch_bounds__(kBlock) k_samp_reduce(const Key* __restrict__ keys, const float* __restrict__ wts,
                                                        const uint32_t* __restrict__ ids,
                                                        const int64_t* __restrict__ start,
                                                        const float4* __restrict__ dirs,
                                                        const int64_t* __restrict__ ctl, vx_voxels out) {
  const int64_t nv = ctl[SC_VOX];
  for (int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x; v < nv; v += int64_t(gridDim.x) * kBlock) {
    const int64_t a = start[v], b = start[v + 1];
    Moment m{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t j = a; j < b; ++j) accum_pair<KIND>(m, wts[j], dirs[ids[j]]);
    static_cast<Key*>(out.keys)[v] = keys[a];
    out.count[v] = uint32_t(b - a);
    out.w[v] = m.W;
    out.S[v] = m.xx;
    out.S[out.cap + v] = m.yy;
    out.S[2 * out.cap + v] = m.zz;
    out.S[3 * out.cap + v] = m.xy;
    out.S[4 * out.cap + v] = m.xz;
    out.S[5 * out.cap + v] = m.yz;
  }
}

int blocks_for(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 1 ? 1 : (b > 4 * kGrid ? 4 * kGrid : b));
}

template <class Key>
void samp_back(int kind, const vx_grid* g, int64_t max_samples, const SampWs& w, const vx_voxels* out,
               int64_t* stats, hipStream_t s) {
  const int key_bits = 3 * g->log2_res + 1;     // one bit above the voxels' keys: the outside key
  hipLaunchKernelGGL(k_samp_n, dim3(1), dim3(64), 0, s, w.ctl, max_samples);
  const int res = radix_sort_pairs(sizeof(Key) == 8, key_bits, w.a, w.b, w.ctl + SC_INSIDE, max_samples, w.hist,
                                   w.partial, s);
  const PairBufs P = res ? w.b : w.a;
  {
    VX_TIMED("sample_heads", s);
    device_scan(HeadIn<Key, 0>{(const Key*)P.keys}, SegOut{w.start, out->cap + 2},
                SegTotal{w.start, w.ctl, out->cap + 2}, w.ctl + SC_INSIDE, 0, w.partial, s);
    hipLaunchKernelGGL(k_samp_finish, dim3(1), dim3(64), 0, s, w.ctl, stats, out->cap);
  }
  VX_TIMED("sample_reduce", s);
  if (kind == 0)
    hipLaunchKernelGGL((k_samp_reduce<0, Key>), dim3(kGrid), dim3(kBlock), 0, s, (const Key*)P.keys, P.w, P.prim,
                       w.start, w.dirs, w.ctl, *out);
  else
    hipLaunchKernelGGL((k_samp_reduce<1, Key>), dim3(kGrid), dim3(kBlock), 0, s, (const Key*)P.keys, P.w, P.prim,
                       w.start, w.dirs, w.ctl, *out);
}

}  // namespace

size_t sample_ws_bytes(int kind, int64_t n_prims, int64_t max_samples, int64_t max_vox, int log2R, int sub) {
  return samp_ws_layout(kind, n_prims, max_samples, max_vox, log2R > 10, sub, nullptr, nullptr);
}

vx_status sample_voxelize(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                          int64_t n_fib, const vx_sampling* sp, int64_t max_samples, void* ws, const vx_voxels* out,
                          int64_t* stats, hipStream_t s) {
  const bool key64 = g->log2_res > 10;
  SampWs w;
  samp_ws_layout(kind, n_prims, max_samples, out->cap, key64, sp->chords_per_segment, ws, &w);
  Grid64 G;
  for (int a = 0; a < 3; ++a) G.bmin[a] = g->bmin[a];
  G.vs = ldexp(1.0, g->log2_res) / g->extent;
  G.R = int64_t(1) << g->log2_res;
  launch_fill_i64(w.ctl, 8, 0, s);
  launch_fill_i64(stats, VX_NSTAT, 0, s);
  launch_fill_i64(w.cnt + n_prims, 1, 0, s);      // the scan's last element: the total
  {
    VX_TIMED(kind == 0 ? "sample_tri_count" : "sample_fib_count", s);
    if (kind == 0) {
      hipLaunchKernelGGL(k_samp_tri_q, dim3(blocks_for(n_prims)), dim3(kBlock), 0, s, data, n_prims, G, w.q, w.ctl,
                         stats);
      hipLaunchKernelGGL(k_samp_tri_count, dim3(blocks_for(n_prims)), dim3(kBlock), 0, s, data, n_prims, G,
                         sp->max_triangle_samples, w.q, w.ctl, w.cnt, w.dirs);
    } else {
      hipLaunchKernelGGL(k_samp_offsets, dim3(blocks_for(n_fib + 1)), dim3(kBlock), 0, s, offsets, n_fib, n_prims,
                         stats);
      hipLaunchKernelGGL(k_samp_fib_count, dim3(blocks_for(n_prims)), dim3(kBlock), 0, s, data, n_prims, offsets,
                         n_fib, sp->chords_per_segment, sp->samples_per_chord, G, w.cnt, w.dirs, stats);
    }
    device_scan(CntIn{w.cnt}, CntOut{w.cnt}, SampTotal{w.ctl, stats, max_samples}, nullptr, n_prims + 1, w.partial,
                s);
  }
  {
    VX_TIMED(kind == 0 ? "sample_tri_emit" : "sample_fib_emit", s);
    const uint64_t out64 = uint64_t(1) << (3 * g->log2_res);
#define VX_SAMP_EMIT(K)                                                                                              \
  if (kind == 0)                                                                                                     \
    hipLaunchKernelGGL(k_samp_tri_emit<K>, dim3(blocks_for(n_prims)), dim3(kBlock), 0, s, data, n_prims, G, w.q,    \
                       w.cnt, w.ctl, max_samples, K(out64), (K*)w.a.keys, w.a.w, w.a.prim);                          \
  else                                                                                                               \
    hipLaunchKernelGGL(k_samp_fib_emit<K>, dim3(blocks_for(n_prims)), dim3(kBlock), 0, s, data, n_prims, offsets,   \
                       n_fib, sp->chords_per_segment, sp->samples_per_chord, G, w.cnt, w.ctl, max_samples, K(out64), \
                       (K*)w.a.keys, w.a.w, w.a.prim)
    if (key64) { VX_SAMP_EMIT(uint64_t); } else { VX_SAMP_EMIT(uint32_t); }
#undef VX_SAMP_EMIT
  }
  if (key64)
    samp_back<uint64_t>(kind, g, max_samples, w, out, stats, s);
  else
    samp_back<uint32_t>(kind, g, max_samples, w, out, stats, s);
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

}  // namespace vx
