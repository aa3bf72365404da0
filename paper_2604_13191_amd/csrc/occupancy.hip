// occupancy.hip -- sub-voxel occupancy and projected densities (Sec. 3.5 occupancy equation and
// XY / XZ / YZ projections; Sec. 4.2 the same projections for the coarser levels).
//
// Every voxel of every level holds 8^3 sub-cells.  At the leaf a sub-cell is hit when a primitive
// touches its closed box (the voxel level's exact predicate on the same lattice, with boxes of
// s / 8 lattice units).  The pairs (primitive, voxel) come from the candidate pipeline; for each
// pair the sub-cells are found by descending the voxel's octree three times (halves, quarters,
// eighths), testing only the children of touched boxes, and the pair's 512-bit mask is OR-ed into
// its voxel's mask.  OR is order-free, so the result does not depend on the order of the atomics.
// A coarser voxel's sub-cell is the union of 2 x 2 x 2 sub-cells of one child, so its mask is its
// children's masks with every byte OR-reduced to one bit.
//
// Mask layout: sub-cell (i, j, k) in [0, 8)^3 has the Morton index m (x bits at 0, 3, 6); word
// m >> 6, bit m & 63.  Word c therefore covers the octant c of the voxel, byte b of it the octant
// b of that octant, and bit b' of the byte the sub-cell b' of that.
#include "geom.hpp"
#include "vx_internal.hpp"

namespace vx {
namespace {

__device__ __forceinline__ void occ_flag(int64_t* stats, int64_t bit) {
  atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)bit);
}

// ---------------------------------------------------------------------------------------------
// triangles: the sub-box test with the triangle's figures computed once per pair
// ---------------------------------------------------------------------------------------------
// All coordinates are lattice units relative to the voxel's corner.  The edge-axis projections
// and every box bound are integers below 2^53 (see tri_touch), so FP64 holds them exactly; the
// plane test uses the same error bound and exact fallback as tri_touch.
struct TriSub {
  double c0[3];              // vertex 0
  double e[3][3];            // edges
  double pmin[9], pmax[9];   // the triangle's projections on the nine edge x axis directions
  double amin[3], amax[3];   // its bounding box
  double n[3];               // plane normal
  double base;               // -n . c0
  double mag0;               // sum |n_a c0_a|
};

__device__ __forceinline__ void tri_sub_setup(const int32_t* q, const int64_t v[3], int Sb, TriSub& T) {
  double c[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) c[i][a] = double(q[3 * i + a] - (int32_t(v[a]) << Sb));
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T.c0[a] = c[0][a];
    T.e[0][a] = c[1][a] - c[0][a];
    T.e[1][a] = c[2][a] - c[1][a];
    T.e[2][a] = c[0][a] - c[2][a];
    T.amin[a] = fmin(fmin(c[0][a], c[1][a]), c[2][a]);
    T.amax[a] = fmax(fmax(c[0][a], c[1][a]), c[2][a]);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int u = (k + 1) % 3, w = (k + 2) % 3;
      const double au = -T.e[j][w], aw = T.e[j][u];
      const double p0 = fma(au, c[j][u], aw * c[j][w]);
      const double p2 = fma(au, c[(j + 2) % 3][u], aw * c[(j + 2) % 3][w]);
      T.pmin[3 * j + k] = fmin(p0, p2);
      T.pmax[3 * j + k] = fmax(p0, p2);
    }
  }
  T.n[0] = fma(T.e[0][2], T.e[2][1], -(T.e[0][1] * T.e[2][2]));
  T.n[1] = fma(T.e[0][0], T.e[2][2], -(T.e[0][2] * T.e[2][0]));
  T.n[2] = fma(T.e[0][1], T.e[2][0], -(T.e[0][0] * T.e[2][1]));
  T.base = -(T.n[0] * c[0][0] + T.n[1] * c[0][1] + T.n[2] * c[0][2]);
  T.mag0 = fabs(T.n[0] * c[0][0]) + fabs(T.n[1] * c[0][1]) + fabs(T.n[2] * c[0][2]);
}

// does the triangle meet the closed box [o, o + sl]^3?
__device__ __forceinline__ bool tri_sub_touch(const TriSub& T, double o0, double o1, double o2, double sl) {
  const double o[3] = {o0, o1, o2};
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (o[a] > T.amax[a] || o[a] + sl < T.amin[a]) return false;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int u = (k + 1) % 3, w = (k + 2) % 3;
      const double au = -T.e[j][w], aw = T.e[j][u];
      const double ao = fma(au, o[u], aw * o[w]);
      const double blo = ao + (fmin(au, 0.0) + fmin(aw, 0.0)) * sl;
      const double bhi = ao + (fmax(au, 0.0) + fmax(aw, 0.0)) * sl;
      if (T.pmax[3 * j + k] < blo || T.pmin[3 * j + k] > bhi) return false;
    }
  }
  // plane: n . (corner - c0) over the box's corners must not keep one strict sign
  const double no = T.n[0] * o[0] + T.n[1] * o[1] + T.n[2] * o[2];
  const double b = T.base + no;
  double lo = b, hi = b;
  double mag = T.mag0 + fabs(T.n[0] * o[0]) + fabs(T.n[1] * o[1]) + fabs(T.n[2] * o[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double t = T.n[a] * sl;
    if (T.n[a] > 0) hi += t; else lo += t;
    mag += fabs(t);
  }
  const double err = mag * 0x1p-48;
  if (lo > err || hi < -err) return false;
  if (lo < -err && hi > err) return true;
  return plane_exact(int64_t(T.n[0]), int64_t(T.n[1]), int64_t(T.n[2]), int64_t(o[0] - T.c0[0]),
                     int64_t(o[1] - T.c0[1]), int64_t(o[2] - T.c0[2]), int64_t(sl));
}

// ---------------------------------------------------------------------------------------------
// capsules: the voxel level's test on the sub-boxes (absolute sub-box indices), plus a
// conservative containment test that settles whole subtrees
// ---------------------------------------------------------------------------------------------
// Is the closed box (index u, size 2^Sb) inside the capsule?  Its farthest point from the
// segment is within dist(centre, segment) + h sqrt(3); a true answer is certain (the margins
// cover every rounding), a false one only means "not known".
__device__ __forceinline__ bool cap_contains(const int32_t* r, const int64_t u[3], int64_t s, int Sb, int64_t rho,
                                             double inv_dd) {
  CapIn q;
  cap_setup(r, u, s, Sb, q);
  const double h = 0.5 * double(s);
  double wx = h - q.c[0], wy = h - q.c[1], wz = h - q.c[2];
  double tc = (wx * q.d[0] + wy * q.d[1] + wz * q.d[2]) * inv_dd;
  tc = fmin(fmax(tc, 0.0), 1.0);
  wx = fma(-tc, q.d[0], wx);
  wy = fma(-tc, q.d[1], wy);
  wz = fma(-tc, q.d[2], wz);
  const double dc = sqrt(wx * wx + wy * wy + wz * wz + q.err);
  return (dc + h * 1.7320508075688772 * (1.0 + 0x1p-40)) * (1.0 + 0x1p-40) <= double(rho);
}

// ---------------------------------------------------------------------------------------------
// per pair: find the voxel in the leaf, descend, OR the words in
// ---------------------------------------------------------------------------------------------
template <class Key>
__device__ __forceinline__ int64_t find_key(const Key* __restrict__ keys, int64_t n, Key k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo < n && keys[lo] == k ? lo : -1;
}

template <int KIND, class Key>
__global__ void __launch_bounds__(kBlock) k_occ_pairs(const int32_t* __restrict__ rec, const Key* __restrict__ pkeys,
                                                      const uint32_t* __restrict__ prim,
                                                      const int64_t* __restrict__ ctl, Lat L,
                                                      const Key* __restrict__ leaf_keys,
                                                      const int64_t* __restrict__ n_leaf, int64_t leaf_cap,
                                                      unsigned long long* __restrict__ mask, int64_t cap,
                                                      int64_t* stats) {
  const int64_t n = ctl[CTL_N_PAIRS];
  // a leaf over either capacity is flagged by k_occ_check; searching a clamped prefix keeps every
  // access in bounds
  const int64_t nl = imin(imin(*n_leaf, leaf_cap), cap);
  const int Sb = L.Sb;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    const Key key = pkeys[i];
    const int64_t idx = find_key<Key>(leaf_keys, nl, key);
    if (idx < 0) {                     // the leaf given is not this voxelization's
      occ_flag(stats, VX_FLAG_OCC_LEAF);
      continue;
    }
    const int64_t v[3] = {int64_t(compact3(uint64_t(key))), int64_t(compact3(uint64_t(key) >> 1)),
                          int64_t(compact3(uint64_t(key) >> 2))};
    const int32_t* r = rec + int64_t(prim[i]) * kRec;
    if (KIND == 0) {
      TriSub T;
      tri_sub_setup(r, v, Sb, T);
      const double s1 = double(int64_t(1) << (Sb - 1)), s2 = 0.5 * s1, s3 = 0.25 * s1;
      for (int c1 = 0; c1 < 8; ++c1) {
        const double a0 = (c1 & 1) * s1, a1 = ((c1 >> 1) & 1) * s1, a2 = (c1 >> 2) * s1;
        if (!tri_sub_touch(T, a0, a1, a2, s1)) continue;
        uint64_t word = 0;
        for (int c2 = 0; c2 < 8; ++c2) {
          const double b0 = a0 + (c2 & 1) * s2, b1 = a1 + ((c2 >> 1) & 1) * s2, b2 = a2 + (c2 >> 2) * s2;
          if (!tri_sub_touch(T, b0, b1, b2, s2)) continue;
          uint32_t bits = 0;
          for (int c3 = 0; c3 < 8; ++c3)
            if (tri_sub_touch(T, b0 + (c3 & 1) * s3, b1 + ((c3 >> 1) & 1) * s3, b2 + (c3 >> 2) * s3, s3))
              bits |= 1u << c3;
          word |= uint64_t(bits) << (8 * c2);
        }
        if (word) atomicOr(mask + int64_t(c1) * cap + idx, (unsigned long long)word);
      }
    } else {
      const double inv_dd = cap_inv_len2(r);
      const int64_t rho = L.rho;
      for (int c1 = 0; c1 < 8; ++c1) {
        const int64_t u1[3] = {2 * v[0] + (c1 & 1), 2 * v[1] + ((c1 >> 1) & 1), 2 * v[2] + (c1 >> 2)};
        const int64_t s1 = int64_t(1) << (Sb - 1);
        if (!cap_touch(r, u1, s1, Sb - 1, rho)) continue;
        uint64_t word = ~0ull;
        if (!cap_contains(r, u1, s1, Sb - 1, rho, inv_dd)) {
          word = 0;
          for (int c2 = 0; c2 < 8; ++c2) {
            const int64_t u2[3] = {2 * u1[0] + (c2 & 1), 2 * u1[1] + ((c2 >> 1) & 1), 2 * u1[2] + (c2 >> 2)};
            const int64_t s2 = s1 >> 1;
            if (!cap_touch(r, u2, s2, Sb - 2, rho)) continue;
            uint32_t bits = 0xffu;
            if (!cap_contains(r, u2, s2, Sb - 2, rho, inv_dd)) {
              bits = 0;
              for (int c3 = 0; c3 < 8; ++c3) {
                const int64_t u3[3] = {2 * u2[0] + (c3 & 1), 2 * u2[1] + ((c3 >> 1) & 1), 2 * u2[2] + (c3 >> 2)};
                if (cap_touch(r, u3, s2 >> 1, Sb - 3, rho)) bits |= 1u << c3;
              }
            }
            word |= uint64_t(bits) << (8 * c2);
          }
        }
        if (word) atomicOr(mask + int64_t(c1) * cap + idx, (unsigned long long)word);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// counts and the coarser levels
// ---------------------------------------------------------------------------------------------
// hits and the cells of the XY, XZ and YZ planes whose column holds a hit
__device__ __forceinline__ void occ_counts(const uint64_t m[8], uint16_t out[4]) {
  int h = 0, xy = 0, xz = 0, yz = 0;
#pragma unroll
  for (int w = 0; w < 8; ++w) h += __popcll(m[w]);
  // along z: the word's z bit is 4, in-word z bits are 2 and 5
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint64_t x = m[w] | m[w + 4];
    x |= x >> 32;
    x |= x >> 4;
    xy += __popcll(x & 0x0f0f0f0full);
  }
  // along y: word bit 2, in-word bits 1 and 4
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int w = (t & 1) | ((t & 2) << 1);
    uint64_t x = m[w] | m[w + 2];
    x |= x >> 16;
    x |= x >> 2;
    xz += __popcll(x & 0x0000333300003333ull);
  }
  // along x: word bit 1, in-word bits 0 and 3
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int w = 2 * t;
    uint64_t x = m[w] | m[w + 1];
    x |= x >> 8;
    x |= x >> 1;
    yz += __popcll(x & 0x0055005500550055ull);
  }
  out[0] = uint16_t(h);
  out[1] = uint16_t(xy);
  out[2] = uint16_t(xz);
  out[3] = uint16_t(yz);
}

__global__ void __launch_bounds__(kBlock) k_occ_zero(unsigned long long* __restrict__ mask, int64_t cap,
                                                     const int64_t* __restrict__ n_ptr) {
  const int64_t n = *n_ptr < cap ? *n_ptr : cap;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
#pragma unroll
    for (int w = 0; w < 8; ++w) mask[w * cap + i] = 0ull;
}

__global__ void __launch_bounds__(kBlock) k_occ_leaf_counts(const unsigned long long* __restrict__ mask, int64_t cap,
                                                            const int64_t* __restrict__ n_ptr,
                                                            uint16_t* __restrict__ hits) {
  const int64_t n = *n_ptr < cap ? *n_ptr : cap;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    uint64_t m[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) m[w] = mask[w * cap + i];
    uint16_t c[4];
    occ_counts(m, c);
#pragma unroll
    for (int t = 0; t < 4; ++t) hits[t * cap + i] = c[t];
  }
}

// the byte-wise OR of one 64-bit word, byte b -> bit b
__device__ __forceinline__ uint32_t byte_any(uint64_t x) {
  x |= x >> 4;
  x |= x >> 2;
  x |= x >> 1;
  x &= 0x0101010101010101ull;
  return uint32_t((x * 0x0102040810204080ull) >> 56);
}

// Parent p's children are the voxels of the level below with key >> 3 == key_p, contiguous in
// key order: found by a search for key_p << 3.
// cstride / pstride: the occupancy capacities (mask and count strides); cmax / pmax: the most
// voxels both the level and its occupancy hold
template <class Key>
__global__ void __launch_bounds__(kBlock) k_occ_up(const Key* __restrict__ ckeys, const int64_t* __restrict__ n_child,
                                                   const unsigned long long* __restrict__ cmask, int64_t cstride,
                                                   int64_t cmax, const Key* __restrict__ pkeys,
                                                   const int64_t* __restrict__ n_par,
                                                   unsigned long long* __restrict__ pmask, uint16_t* __restrict__ hits,
                                                   int64_t pstride, int64_t pmax, int64_t* stats) {
  const int64_t np = *n_par, nc = *n_child;
  if (np > pmax || nc > cmax) {
    if (blockIdx.x == 0 && threadIdx.x == 0) occ_flag(stats, VX_FLAG_VOXEL_CAPACITY);
    return;
  }
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < np; p += int64_t(gridDim.x) * kBlock) {
    const Key pk = pkeys[p];
    const Key first = Key(pk << 3);
    int64_t lo = 0, hi = nc;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ckeys[mid] < first) lo = mid + 1; else hi = mid;
    }
    uint64_t m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t c = lo; c < nc && Key(ckeys[c] >> 3) == pk; ++c) {
      const int oct = int(ckeys[c] & 7);
      uint64_t word = 0;
#pragma unroll
      for (int w = 0; w < 8; ++w) word |= uint64_t(byte_any(cmask[w * cstride + c])) << (8 * w);
#pragma unroll
      for (int w = 0; w < 8; ++w)
        if (w == oct) m[w] = word;
    }
#pragma unroll
    for (int w = 0; w < 8; ++w) pmask[w * pstride + p] = m[w];
    uint16_t cnt[4];
    occ_counts(m, cnt);
#pragma unroll
    for (int t = 0; t < 4; ++t) hits[t * pstride + p] = cnt[t];
  }
}

// the leaf's count against its occupancy capacity
__global__ void k_occ_check(const int64_t* __restrict__ n_leaf, int64_t vcap, int64_t ocap, int64_t* stats) {
  if (threadIdx.x == 0 && (*n_leaf > vcap || *n_leaf > ocap)) occ_flag(stats, VX_FLAG_VOXEL_CAPACITY);
}

int occ_blocks(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 1 ? 1 : (b > 4 * kGrid ? 4 * kGrid : b));
}

}  // namespace

size_t occupancy_ws_bytes(int64_t n_prims, int64_t max_cand, int64_t max_pairs, bool key64) {
  Carver cv(nullptr);
  front_ws_carve(cv, n_prims, max_cand, max_pairs, key64, nullptr);
  return cv.off + 256;
}

vx_status occupancy_run(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                        int64_t n_fib, float radius, const vx_voxels* leaf, const vx_voxels* out,
                        const int64_t* n_levels, int levels, int64_t max_cand, int64_t max_pairs,
                        const vx_occupancy* occ, void* ws, int64_t* stats, hipStream_t s) {
  const bool key64 = g->log2_res > 10;
  Carver cv(ws);
  FrontWs w;
  front_ws_carve(cv, n_prims, max_cand, max_pairs, key64, &w);
  voxelize_front(kind, g, data, n_prims, offsets, n_fib, radius, max_cand, max_pairs, w, stats, s, nullptr);
  const Lat L = make_lat(g, kind, radius);
  hipLaunchKernelGGL(k_occ_check, dim3(1), dim3(64), 0, s, n_levels, leaf->cap, occ[0].cap, stats);
  hipLaunchKernelGGL(k_occ_zero, dim3(occ_blocks(occ[0].cap)), dim3(kBlock), 0, s,
                     reinterpret_cast<unsigned long long*>(occ[0].mask), occ[0].cap, n_levels);
  {
    VX_TIMED(kind == 0 ? "occ_pairs_tri" : "occ_pairs_fib", s);
#define VX_OCC(KD, K)                                                                                           \
  hipLaunchKernelGGL((k_occ_pairs<KD, K>), dim3(kGrid * 4), dim3(kBlock), 0, s, w.rec, (const K*)w.pa.keys,   \
                     w.pa.prim, w.ctl, L, (const K*)leaf->keys, n_levels, leaf->cap,                            \
                     reinterpret_cast<unsigned long long*>(occ[0].mask), occ[0].cap, stats)
    if (kind == 0) {
      if (key64) VX_OCC(0, uint64_t); else VX_OCC(0, uint32_t);
    } else {
      if (key64) VX_OCC(1, uint64_t); else VX_OCC(1, uint32_t);
    }
#undef VX_OCC
  }
  VX_TIMED("occ_levels", s);
  hipLaunchKernelGGL(k_occ_leaf_counts, dim3(occ_blocks(occ[0].cap)), dim3(kBlock), 0, s,
                     reinterpret_cast<const unsigned long long*>(occ[0].mask), occ[0].cap, n_levels, occ[0].hits);
  for (int l = 1; l < levels; ++l) {
    const vx_voxels& C = l == 1 ? *leaf : out[l - 2];
    const vx_voxels& P = out[l - 1];
    const int64_t pmax = imin(P.cap, occ[l].cap), cmax = imin(C.cap, occ[l - 1].cap);
#define VX_UP(K)                                                                                                  \
  hipLaunchKernelGGL(k_occ_up<K>, dim3(occ_blocks(pmax)), dim3(kBlock), 0, s, (const K*)C.keys, n_levels + l - 1, \
                     reinterpret_cast<const unsigned long long*>(occ[l - 1].mask), occ[l - 1].cap, cmax,        \
                     (const K*)P.keys, n_levels + l, reinterpret_cast<unsigned long long*>(occ[l].mask),        \
                     occ[l].hits, occ[l].cap, pmax, stats)
    if (key64) VX_UP(uint64_t); else VX_UP(uint32_t);
#undef VX_UP
  }
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

}  // namespace vx
