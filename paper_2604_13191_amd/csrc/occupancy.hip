// occupancy.hip -- sub-voxel occupancy and projected densities (Sec. 3.5 occupancy equation and
// XY / XZ / YZ projections; Sec. 4.2 the same projections for the coarser levels).
//
// Every voxel of every level holds 8^3 sub-cells.  At the leaf a sub-cell is hit when a primitive
// touches its closed box (the voxel level's exact predicate on the same lattice, with boxes of
// s / 8 lattice units).  The pairs (primitive, voxel) come from the candidate pipeline; for each
// pair the sub-cells inside the primitive's bounding box are tested (triangles through their three
// axis projections and the plane, capsules by the distance from each sub-cell's centre), and the
// pair's 512-bit mask is OR-ed into its voxel's mask.  OR is order-free, so the result does not
// depend on the order of the atomics.
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
// triangles
// ---------------------------------------------------------------------------------------------
// The closed-box test is the separating-axis test on the box axes, the plane normal and the nine
// edge x box-axis directions.  The three edge directions perpendicular to axis k and the two box
// axes other than k are the separating-axis test of the triangle and the box projected along k, so
// a sub-cell (i, j, k) is touched exactly when
//     P_z(i, j)  and  P_y(i, k)  and  P_x(j, k)  and  the plane meets the box,
// with P_z, P_y, P_x the 8 x 8 masks of the squares the projected triangle meets (each 64 bits,
// first coordinate * 8 + second).  Coordinates are lattice units from the voxel's corner.  The
// projections and every box bound of the edge tests are integers below 2^53 (see tri_touch), so
// FP64 holds them exactly; the plane test takes tri_touch's error bound and exact fallback.
struct TriOcc {
  double c0[3];
  double e[3][3];
  double pmin[9], pmax[9];   // the triangle on the nine edge x axis directions (edge j, axis k: 3j + k)
  double n[3], nlo, nhi;     // plane normal, sums of its negative and positive parts
  double base;               // -n . c0
  double err;                // bound on the rounding of every plane evaluation in this voxel
  int lo[3], hi[3];          // sub-cells the bounding box meets, per axis
};

__device__ __forceinline__ void tri_occ_setup(const int32_t* q, const int64_t v[3], int Sb, TriOcc& T) {
  double c[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) c[i][a] = double(q[3 * i + a] - (int32_t(v[a]) << Sb));
  const double sl = double(int64_t(1) << (Sb - 3)), isl = 1.0 / sl;    // exact: powers of two
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T.c0[a] = c[0][a];
    T.e[0][a] = c[1][a] - c[0][a];
    T.e[1][a] = c[2][a] - c[1][a];
    T.e[2][a] = c[0][a] - c[2][a];
    const double mn = fmin(fmin(c[0][a], c[1][a]), c[2][a]), mx = fmax(fmax(c[0][a], c[1][a]), c[2][a]);
    // box [i sl, (i+1) sl] meets [mn, mx] for ceil(mn / sl) - 1 <= i <= floor(mx / sl)
    T.lo[a] = int(fmax(ceil(mn * isl) - 1.0, 0.0));
    T.hi[a] = int(fmin(floor(mx * isl), 7.0));
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
  T.nlo = (fmin(T.n[0], 0.0) + fmin(T.n[1], 0.0) + fmin(T.n[2], 0.0)) * sl;
  T.nhi = (fmax(T.n[0], 0.0) + fmax(T.n[1], 0.0) + fmax(T.n[2], 0.0)) * sl;
  T.base = -(T.n[0] * c[0][0] + T.n[1] * c[0][1] + T.n[2] * c[0][2]);
  const double mag0 = fabs(T.n[0] * c[0][0]) + fabs(T.n[1] * c[0][1]) + fabs(T.n[2] * c[0][2]);
  // every sub-box corner offset is at most 8 sl per axis, and its bounds add sl more
  T.err = (mag0 + 9.0 * sl * (fabs(T.n[0]) + fabs(T.n[1]) + fabs(T.n[2]))) * 0x1p-48;
}

// the squares (a, b) of the plane perpendicular to axis k (a along (k+1) % 3, b along (k+2) % 3)
// that the projected triangle meets: bit a * 8 + b
__device__ __forceinline__ uint64_t tri_occ_proj(const TriOcc& T, int k, double sl) {
  const int u = (k + 1) % 3, w = (k + 2) % 3;
  uint64_t m = 0;
  for (int a = T.lo[u]; a <= T.hi[u]; ++a) {
    for (int b = T.lo[w]; b <= T.hi[w]; ++b) {
      const double ou = a * sl, ow = b * sl;
      bool in = true;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double au = -T.e[j][w], aw = T.e[j][u];
        const double ao = fma(au, ou, aw * ow);
        const double blo = ao + (fmin(au, 0.0) + fmin(aw, 0.0)) * sl;
        const double bhi = ao + (fmax(au, 0.0) + fmax(aw, 0.0)) * sl;
        in = in && !(T.pmax[3 * j + k] < blo || T.pmin[3 * j + k] > bhi);
      }
      if (in) m |= 1ull << (a * 8 + b);
    }
  }
  return m;
}

// does the plane meet the closed box at sub-cell (i, j, k)?
__device__ __forceinline__ bool tri_occ_plane(const TriOcc& T, int i, int j, int k, double sl) {
  const double o0 = i * sl, o1 = j * sl, o2 = k * sl;
  const double b = T.base + (T.n[0] * o0 + T.n[1] * o1 + T.n[2] * o2);
  const double lo = b + T.nlo, hi = b + T.nhi;
  if (lo > T.err || hi < -T.err) return false;
  if (lo < -T.err && hi > T.err) return true;
  return plane_exact(int64_t(T.n[0]), int64_t(T.n[1]), int64_t(T.n[2]), int64_t(o0 - T.c0[0]), int64_t(o1 - T.c0[1]),
                     int64_t(o2 - T.c0[2]), int64_t(sl));
}

// ---------------------------------------------------------------------------------------------
// capsules: per sub-cell the distance from its centre to the segment decides (the box holds the
// ball of radius h around its centre and lies in the one of radius h sqrt(3)); the rest take the
// exact voxel-level test on the sub-box.
// ---------------------------------------------------------------------------------------------
struct CapOcc {
  double c[3], d[3];         // segment start from the voxel's corner, direction (lattice units)
  double inv_dd;             // 1 / |d|^2 (0 for a point)
  double err;                // rounding bound of a squared distance, as in cap_ball
  double rin2, rout2;        // touch below (h + rho)^2, none above (h sqrt 3 + rho)^2
  int lo[3], hi[3];
};

__device__ __forceinline__ void cap_occ_setup(const int32_t* r, const int64_t v[3], int Sb, int64_t rho, CapOcc& C) {
  const double s = double(int64_t(1) << Sb), sl = 0.125 * s, isl = 1.0 / sl;
  double M = s;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t ci = r[a] - (int32_t(v[a]) << Sb);
    const int32_t di = r[3 + a] - r[a];
    C.c[a] = double(ci);
    C.d[a] = double(di);
    M = fmax(M, fabs(C.c[a]) + fabs(C.d[a]) + s);
    const double mn = fmin(C.c[a], C.c[a] + C.d[a]) - double(rho), mx = fmax(C.c[a], C.c[a] + C.d[a]) + double(rho);
    C.lo[a] = int(fmax(ceil(mn * isl) - 1.0, 0.0));
    C.hi[a] = int(fmin(floor(mx * isl), 7.0));
  }
  C.inv_dd = cap_inv_len2(r);
  C.err = M * M * 0x1p-44;
  const double h = 0.5 * sl, rh = double(rho);
  C.rin2 = (h + rh) * (h + rh);
  C.rout2 = (h * 1.7320508075688772 + rh) * (h * 1.7320508075688772 + rh) * (1.0 + 0x1p-40);
}

__device__ __attribute__((noinline)) bool cap_occ_exact(const int32_t* r, int64_t u0, int64_t u1, int64_t u2,
                                                        int64_t sl, int Sbl, int64_t rho) {
  const int64_t u[3] = {u0, u1, u2};
  return cap_touch(r, u, sl, Sbl, rho);
}

// A sub-cell whose centre lies between the two balls.  P, the segment's point nearest the centre
// X, and u = (X - P) / |X - P|: the segment projects onto u at or below u . P (P is its nearest
// point to X) and the box at or above u . X - h (|u_x| + |u_y| + |u_z|), so the box lies farther
// than |X - P| - h sum |u_a| from the segment; and the box lies within the distance from P to the
// box.  Either settles most; the margins (2 err on squared lengths) cover every rounding.  The
// rest take the exact test.
__device__ __forceinline__ bool cap_occ_band(const CapOcc& C, const int32_t* r, const int64_t v[3], int a, int b,
                                             int c, double sl, int Sb, int64_t rho) {
  const double h = 0.5 * sl, rh = double(rho);
  const double o[3] = {a * sl, b * sl, c * sl};
  double w[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) w[x] = (o[x] + h) - C.c[x];
  double tc = (w[0] * C.d[0] + w[1] * C.d[1] + w[2] * C.d[2]) * C.inv_dd;
  tc = fmin(fmax(tc, 0.0), 1.0);
  double dc2 = 0.0, s1 = 0.0, f = 0.0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const double wx = fma(-tc, C.d[x], w[x]);
    dc2 = fma(wx, wx, dc2);
    s1 += fabs(wx);
    const double p = fma(tc, C.d[x], C.c[x]) - o[x];          // P from the box's corner
    const double e = p < 0 ? p : (p > sl ? p - sl : 0.0);
    f = fma(e, e, f);
  }
  if (f + C.err <= rh * rh) return true;
  const double lhs = dc2 - h * s1 - 2.0 * C.err;
  if (lhs > 0.0 && lhs > rh * sqrt(dc2 + C.err) * (1.0 + 0x1p-40)) return false;
  return cap_occ_exact(r, 8 * v[0] + a, 8 * v[1] + b, 8 * v[2] + c, int64_t(sl), Sb - 3, rho);
}

// ---------------------------------------------------------------------------------------------
// per pair: find the voxel in the leaf, build each octant's word, OR it in
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

// Morton bit of sub-cell (i, j, k) inside its octant's word: the low bits of the coordinates
__device__ __forceinline__ int oct_bit(int i, int j, int k) {
  return (i & 1) | ((j & 1) << 1) | ((k & 1) << 2) | ((i & 2) << 2) | ((j & 2) << 3) | ((k & 2) << 4);
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
  const double sl = double(int64_t(1) << (Sb - 3));
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
      TriOcc T;
      tri_occ_setup(r, v, Sb, T);
      const uint64_t pz = tri_occ_proj(T, 2, sl);     // (x, y)
      const uint64_t py = tri_occ_proj(T, 1, sl);     // (z, x)
      const uint64_t px = tri_occ_proj(T, 0, sl);     // (y, z)
      for (int oct = 0; oct < 8; ++oct) {
        const int i0 = (oct & 1) * 4, j0 = ((oct >> 1) & 1) * 4, k0 = (oct >> 2) * 4;
        const int ia = max(T.lo[0], i0), ib = min(T.hi[0], i0 + 3);
        const int ja = max(T.lo[1], j0), jb = min(T.hi[1], j0 + 3);
        const int ka = max(T.lo[2], k0), kb = min(T.hi[2], k0 + 3);
        uint64_t word = 0;
        for (int a = ia; a <= ib; ++a)
          for (int b = ja; b <= jb; ++b) {
            if (!((pz >> (a * 8 + b)) & 1)) continue;
            for (int c = ka; c <= kb; ++c)
              if (((py >> (c * 8 + a)) & 1) && ((px >> (b * 8 + c)) & 1) && tri_occ_plane(T, a, b, c, sl))
                word |= 1ull << oct_bit(a, b, c);
          }
        if (word) atomicOr(mask + int64_t(oct) * cap + idx, (unsigned long long)word);
      }
    } else {
      CapOcc C;
      cap_occ_setup(r, v, Sb, L.rho, C);
      const double h = 0.5 * sl;
      for (int oct = 0; oct < 8; ++oct) {
        const int i0 = (oct & 1) * 4, j0 = ((oct >> 1) & 1) * 4, k0 = (oct >> 2) * 4;
        const int ia = max(C.lo[0], i0), ib = min(C.hi[0], i0 + 3);
        const int ja = max(C.lo[1], j0), jb = min(C.hi[1], j0 + 3);
        const int ka = max(C.lo[2], k0), kb = min(C.hi[2], k0 + 3);
        // the centre test decides most sub-cells; the few near the capsule's surface wait for the
        // exact test until the octant's loop is done, so that one lane's slow path does not stall
        // the wave at every step
        uint64_t word = 0, band = 0;
        for (int a = ia; a <= ib; ++a)
          for (int b = ja; b <= jb; ++b)
            for (int c = ka; c <= kb; ++c) {
              double wx = fma(a, sl, h) - C.c[0], wy = fma(b, sl, h) - C.c[1], wz = fma(c, sl, h) - C.c[2];
              double tc = (wx * C.d[0] + wy * C.d[1] + wz * C.d[2]) * C.inv_dd;
              tc = fmin(fmax(tc, 0.0), 1.0);
              wx = fma(-tc, C.d[0], wx);
              wy = fma(-tc, C.d[1], wy);
              wz = fma(-tc, C.d[2], wz);
              const double dc2 = wx * wx + wy * wy + wz * wz;
              const uint64_t bit = 1ull << oct_bit(a, b, c);
              if (dc2 + C.err <= C.rin2) word |= bit;
              else if (!(dc2 - C.err > C.rout2)) band |= bit;
            }
        while (band) {
          const int t = __builtin_ctzll(band);
          band &= band - 1;
          const int a = i0 + ((t & 1) | ((t >> 2) & 2)), b = j0 + (((t >> 1) & 1) | ((t >> 3) & 2)),
                    c = k0 + (((t >> 2) & 1) | ((t >> 4) & 2));
          if (cap_occ_band(C, r, v, a, b, c, sl, Sb, L.rho)) word |= 1ull << t;
        }
        if (word) atomicOr(mask + int64_t(oct) * cap + idx, (unsigned long long)word);
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
  voxelize_front(kind, g, data, n_prims, offsets, n_fib, radius, max_cand, max_pairs, w, stats, s, nullptr, false);
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
