// tiles.hip -- the leaf pass by spatial tiles (Sec. 3.2-3.4 on a tiled grid).
//
// Space is cut into aligned tiles of 2^tb voxels per axis (tb = 4: 16^3 voxels, one Morton
// range each).  Every primitive is listed once per tile its candidate box overlaps; the list is
// sorted by tile (a small radix sort over primitive-tile records, not over pairs).  Tiles whose
// candidate count exceeds what a work unit holds are split into octants, recursively, down to
// single voxels.  One block then takes a unit: it tests the unit's candidates, keeps the
// surviving (voxel, weight, primitive) triples in LDS, groups them by voxel and sums every
// voxel's pairs in primitive order -- the order of the pair list of the global path, so the
// sums are bit-identical -- and writes the unit's voxels.  No pair list goes through HBM.
#include "geom.hpp"
#include "vx_internal.hpp"

namespace vx {

namespace {

__device__ __forceinline__ void flag_set(int64_t* stats, int64_t bit) {
  atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)bit);
}


// a block-wide sum (all threads get it); tmp: kWaves + 1 entries
template <class T>
__device__ __forceinline__ T block_sum(T v, T* tmp) {
  T tot;
  (void)block_exclusive_scan(v, tmp, tot);
  return tot;
}

// candidates of primitive record r inside the box [o, o + sz): per-axis first voxel and extent
__device__ __forceinline__ int64_t clip_box(const int32_t* r, const int32_t o[3], const int32_t sz[3], int32_t lo[3],
                                            int32_t n[3]) {
  int64_t c = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t l = r[9 + a] > o[a] ? r[9 + a] : o[a];
    const int32_t h0 = r[9 + a] + r[12 + a] - 1, h1 = o[a] + sz[a] - 1;
    const int32_t h = h0 < h1 ? h0 : h1;
    lo[a] = l;
    n[a] = h >= l ? h - l + 1 : 0;
    c *= n[a];
  }
  return c;
}

// the same from a packed box
__device__ __forceinline__ int64_t clip_packed(const ulonglong2& b, const int32_t o[3], const int32_t sz[3]) {
  int32_t bl[3], bh[3];
  unpack_box(b, bl, bh);
  int64_t c = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t l = bl[a] > o[a] ? bl[a] : o[a];
    const int32_t h1 = o[a] + sz[a] - 1;
    const int32_t h = bh[a] < h1 ? bh[a] : h1;
    c *= h >= l ? h - l + 1 : 0;
  }
  return c;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// primitive-tile records
// ---------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_rec_count(const ulonglong2* __restrict__ box,
                                                      const int64_t* __restrict__ cand_cnt, int64_t n_prims, int tb,
                                                      int64_t* __restrict__ rcnt) {
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < n_prims; p += int64_t(gridDim.x) * kBlock) {
    int64_t c = 0;
    if (cand_cnt[p] > 0) {
      int32_t lo[3], hi[3];
      unpack_box(box[p], lo, hi);
      c = 1;
#pragma unroll
      for (int a = 0; a < 3; ++a) c *= int64_t((hi[a] >> tb) - (lo[a] >> tb) + 1);
    }
    rcnt[p] = c;
  }
}

struct RecTotal {
  int64_t* off;
  int64_t* ctl;
  int64_t* stats;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    off[n] = total;
    stats[VX_STAT_RECORDS] = total;
    const bool over = total > cap;
    if (over) flag_set(stats, VX_FLAG_RECORD_CAPACITY);
    ctl[CTL_N_REC] = over ? 0 : total;
  }
};

// record (tile key, primitive) for every tile a primitive's candidate box overlaps; the tile key
// is the Morton code of the tile coordinates (batched: with the patch id above it).  roff: the
// scanned record counts (n_prims + 1 entries); a primitive without candidates has none.
template <class Key>
__global__ void __launch_bounds__(kBlock) k_rec_emit(const int32_t* __restrict__ rec,
                                                     const ulonglong2* __restrict__ box,
                                                     const int64_t* __restrict__ roff, int64_t n_prims,
                                                     const int64_t* __restrict__ ctl, int tb, int batch,
                                                     Key* __restrict__ rkeys, uint32_t* __restrict__ rprim) {
  if (ctl[CTL_N_REC] == 0) return;
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < n_prims; p += int64_t(gridDim.x) * kBlock) {
    if (roff[p + 1] == roff[p]) continue;
    int32_t t0[3], t1[3];
    unpack_box(box[p], t0, t1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      t0[a] >>= tb;
      t1[a] >>= tb;
    }
    const Key hi = batch ? Key(uint64_t(uint32_t(rec[p * kRec + 15])) << (kPatchShift - 3 * tb)) : Key(0);
    int64_t o = roff[p];
    for (int32_t z = t0[2]; z <= t1[2]; ++z)
      for (int32_t y = t0[1]; y <= t1[1]; ++y)
        for (int32_t x = t0[0]; x <= t1[0]; ++x) {
          rkeys[o] = hi | Key(morton3(uint32_t(x), uint32_t(y), uint32_t(z)));
          rprim[o] = uint32_t(p);
          ++o;
        }
  }
}

struct TileTotal {
  int64_t* start;
  int64_t* ctl;
  __device__ void operator()(int64_t total, int64_t n) const {
    start[total] = n;
    ctl[CTL_N_TILES] = total;
  }
};

// ---------------------------------------------------------------------------------------------
// work units: a tile, or an octant of one, whose candidates fit a block's LDS
// ---------------------------------------------------------------------------------------------
struct Unit {
  int64_t tile;       // index into the tile list
  int64_t cand;       // candidates inside the unit
  int32_t o[3];       // first voxel
  int16_t lev;        // cells of 2^lev voxels per axis
  int16_t ncell;      // 1, 2 or 4 sibling cells, consecutive in Morton order (one box)
};

// box of a unit: ncell aligned siblings of 2^lev cells; 2 spans x, 4 spans x and y
__device__ __forceinline__ void unit_box(int lev, int ncell, int32_t sz[3]) {
  sz[0] = (ncell >= 2 ? 2 : 1) << lev;
  sz[1] = (ncell >= 4 ? 2 : 1) << lev;
  sz[2] = 1 << lev;
}

// Per tile (one block each): walk the octant tree depth first in Morton order and count (PASS 0)
// or write (PASS 1) the units.  A cell whose candidates exceed the unit budget is split; among its
// eight children, aligned groups of four or two siblings whose candidates fit together become
// one unit, the others single-cell units or further splits.  A single voxel is always a unit
// (summed in streaming order when it holds more than the budget).
namespace {
enum { kEntUnit = 0, kEntSplit = 1 };
struct PlanEntry {
  int32_t o[3];
  int16_t lev, ncell, kind, pad;
  int64_t cand;
};
}  // namespace

template <int PASS, class Key>
__global__ void __launch_bounds__(kBlock) k_unit_plan(const ulonglong2* __restrict__ box,
                                                      const Key* __restrict__ rkeys,
                                                      const uint32_t* __restrict__ rprim,
                                                      const int64_t* __restrict__ tstart,
                                                      const int64_t* __restrict__ ctl, int tb, int batch,
                                                      int64_t budget, int64_t* __restrict__ ucnt,
                                                      const int64_t* __restrict__ uoff, Unit* __restrict__ units) {
  __shared__ PlanEntry stk[48];
  __shared__ PlanEntry g[8];                         // one split's groups, before they are pushed
  __shared__ int64_t csum[8];
  __shared__ int64_t tmp[kWaves + 1];
  __shared__ int32_t s_top;
  const int64_t n_tiles = ctl[CTL_N_TILES];
  if (PASS == 1 && ctl[CTL_N_UNITS] == 0) return;
  // tile coordinates: the Morton bits below the patch id (batched) or the whole key
  const uint64_t lowmask = batch ? (uint64_t(1) << (kPatchShift - 3 * tb)) - 1 : ~uint64_t(0);
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t s = tstart[t], e = tstart[t + 1];
    const uint64_t tk = uint64_t(rkeys[s]) & lowmask;
    const int32_t to[3] = {int32_t(compact3(tk)) << tb, int32_t(compact3(tk >> 1)) << tb,
                           int32_t(compact3(tk >> 2)) << tb};
    if (PASS == 1) {
      // a tile that is one unit as a whole: its candidate count came with the count pass
      const int64_t wc = ucnt[t] >> 32;
      if (wc > 0) {
        if (threadIdx.x == 0 && wc > 1) {
          Unit u;
          u.tile = t;
          u.cand = wc - 1;
          u.o[0] = to[0];
          u.o[1] = to[1];
          u.o[2] = to[2];
          u.lev = int16_t(tb);
          u.ncell = 1;
          units[uoff[t]] = u;
        }
        continue;
      }
    }
    // the whole tile
    int64_t c = 0;
    for (int64_t j = s + threadIdx.x; j < e; j += kBlock) {
      const int32_t sz[3] = {1 << tb, 1 << tb, 1 << tb};
      c += clip_packed(box[rprim[j]], to, sz);
    }
    c = block_sum(c, tmp);
    if (threadIdx.x == 0) {
      PlanEntry r;
      r.o[0] = to[0];
      r.o[1] = to[1];
      r.o[2] = to[2];
      r.lev = int16_t(tb);
      r.ncell = 1;
      r.kind = (c <= budget || tb == 0) ? kEntUnit : kEntSplit;
      r.cand = c;
      stk[0] = r;
      s_top = 1;
    }
    __syncthreads();
    int64_t nu = 0;
    int64_t out = PASS == 1 ? uoff[t] : 0;
    while (s_top > 0) {
      const PlanEntry E = stk[s_top - 1];
      __syncthreads();                               // everyone has read the top before it changes
      if (E.kind == kEntUnit) {
        if (threadIdx.x == 0) {
          s_top = s_top - 1;
          if (PASS == 1 && E.cand > 0) {
            Unit u;
            u.tile = t;
            u.cand = E.cand;
            u.o[0] = E.o[0];
            u.o[1] = E.o[1];
            u.o[2] = E.o[2];
            u.lev = E.lev;
            u.ncell = E.ncell;
            units[out] = u;
          }
        }
        if (E.cand > 0) {
          ++nu;
          ++out;
        }
        __syncthreads();
        continue;
      }
      // split: candidates of the eight children in one pass (halves per axis)
      const int32_t h = 1 << (E.lev - 1);
      if (threadIdx.x < 8) csum[threadIdx.x] = 0;
      __syncthreads();
      int64_t cc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int64_t j = s + threadIdx.x; j < e; j += kBlock) {
        int32_t bl[3], bh[3];
        unpack_box(box[rprim[j]], bl, bh);
        int64_t nh[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int32_t l = bl[a], hh = bh[a];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int32_t c0 = E.o[a] + q * h, c1 = c0 + h - 1;
            const int32_t lo = l > c0 ? l : c0, hi = hh < c1 ? hh : c1;
            nh[a][q] = hi >= lo ? hi - lo + 1 : 0;
          }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) cc[k] += nh[0][k & 1] * nh[1][(k >> 1) & 1] * nh[2][k >> 2];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int64_t v = wave_sum(cc[k]);
        if (lane_id() == 0) atomicAdd(reinterpret_cast<unsigned long long*>(&csum[k]), (unsigned long long)v);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int top = s_top - 1;                          // pop the split entry
        // groups in Morton order, pushed in reverse so that they pop in order
        int ng = 0;
        auto child = [&](int k, int ncell, int64_t cnt, int kind) {
          PlanEntry r;
          r.o[0] = E.o[0] + ((k & 1) ? h : 0);
          r.o[1] = E.o[1] + ((k & 2) ? h : 0);
          r.o[2] = E.o[2] + ((k & 4) ? h : 0);
          r.lev = int16_t(E.lev - 1);
          r.ncell = int16_t(ncell);
          r.kind = int16_t(kind);
          r.cand = cnt;
          g[ng++] = r;
        };
        for (int q = 0; q < 8; q += 4) {
          const int64_t s4 = csum[q] + csum[q + 1] + csum[q + 2] + csum[q + 3];
          if (s4 <= budget) {
            child(q, 4, s4, kEntUnit);
            continue;
          }
          for (int pp = q; pp < q + 4; pp += 2) {
            const int64_t s2 = csum[pp] + csum[pp + 1];
            if (s2 <= budget) {
              child(pp, 2, s2, kEntUnit);
              continue;
            }
            for (int k = pp; k < pp + 2; ++k)
              child(k, 1, csum[k], (csum[k] <= budget || E.lev - 1 == 0) ? kEntUnit : kEntSplit);
          }
        }
        for (int i = ng - 1; i >= 0; --i) stk[top++] = g[i];
        s_top = top;
      }
      __syncthreads();
    }
    // units per tile (low half); a tile that is one unit as a whole also keeps its candidate
    // count plus one (high half), so that the writing pass skips it
    if (PASS == 0 && threadIdx.x == 0)
      ucnt[t] = nu | ((c <= budget || tb == 0) && c < (int64_t(1) << 30) ? (c + 1) << 32 : 0);
    __syncthreads();
  }
}

struct UnitTotal {
  int64_t* off;
  int64_t* ctl;
  int64_t* stats;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    off[n] = total;
    stats[VX_STAT_UNITS] = total;
    const bool over = total > cap;
    if (over) flag_set(stats, VX_FLAG_UNIT_CAPACITY);
    ctl[CTL_N_UNITS] = over ? 0 : total;
  }
};

// ---------------------------------------------------------------------------------------------
// the unit kernel: test, weigh, group by voxel and sum in LDS
// ---------------------------------------------------------------------------------------------
struct UnitLds {
  uint32_t* start;    // [budget]   after the batches: the voxels' keys and range ends (2 x u16)
  uint16_t* key;      // [budget]   unit-local Morton code of each pair
  uint16_t* idx;      // [budget]   grouped order -> pair
  float* w;           // [budget]   (before the weights: the queue of undecided candidates)
  uint32_t* prim;     // [budget]  
  uint16_t* ckey;     // [budget]   per candidate of the batch: kTouch | its unit-local key,
                      // kUndecided, or 0 for a miss (after the batches: each pair's arrival
                      // slot among its voxel's pairs)
  uint64_t* sbm;      // [64] batch: bit c set where a slot's first candidate is c
  uint32_t* spre;     // [64] slot starts below each word
  int32_t* bprim;     // [kBlock] the current record batch
  int32_t* blo;       // [3][kBlock]
  int32_t* bn;        // [3][kBlock]
  int32_t* boff;      // [kBlock] candidate offsets within the batch
  int32_t* brec;      // [kBlock][9] the slot's primitive vertices (record words 0..8; after
                      // the batches: the per-key counters, then starts)
  int32_t* bpatch;    // [kBlock] the slot's patch (batched)
  double* binv;       // [kBlock] fibers: the slot's 1 / |B - A|^2 (lattice units); triangles:
                      // twice the slot's area (voxel^2)
  int32_t* tmp32;     // [kWaves + 1]
  int32_t* misc;      // [8]
};

// above this many pairs per voxel (unit mean) the grouping places stably instead of sorting
// (triangles: a surface voxel holds a handful of pairs, sorted per voxel in parallel faster than
// one wave places them in order; fibers: dense patches hold hundreds per voxel)
template <int KIND>
constexpr int32_t stable_mean() { return KIND == 0 ? 24 : 4; }
// keys of a unit's range: at most one 16^3 tile
constexpr int32_t kUnitKeys = 4096;
static_assert(kBlock * 9 * 4 >= kUnitKeys * 2, "per-key counters live in the record batch's space");
static_assert(kBlock * 16 == kUnitKeys, "each thread owns 16 keys in the scan of the counters");

// a candidate's outcome and key in one 16-bit word (keys below 4096)
constexpr uint16_t kTouch = 0x8000, kUndecided = 0x4000;
static_assert(kUnitKeys <= kUndecided, "keys fit below the flags");

// LDS of a unit with a budget of CAND candidates; the budgets and the unit kernel's waves per
// SIMD that the LDS then allows (160 KB per CU: 2 blocks at 3072 and 2048, 3 at 1536, 4 at 1024)
template <int CAND>
constexpr size_t unit_lds_bytes() {
  return size_t(CAND) * (4 + 2 + 2 + 4 + 4 + 2) + 64 * 8 + 64 * 4 + kBlock * 4 * (8 + 9 + 1) + kBlock * 8 +
         (kWaves + 1) * 4 + 8 * 4 + 256;
}
constexpr int unit_waves(int cand) { return cand <= 1024 ? 4 : (cand <= 1536 ? 3 : 2); }
static_assert(2 * unit_lds_bytes<3072>() <= 160 * 1024, "two units per CU at the largest budget");
static_assert(3 * unit_lds_bytes<1536>() <= 160 * 1024, "three units per CU at 1536");
static_assert(4 * unit_lds_bytes<1024>() <= 160 * 1024, "four units per CU at 1024");

template <int CAND>
__device__ __forceinline__ UnitLds carve_unit_lds(char* base) {
  UnitLds L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off += (bytes + 7) & ~size_t(7);
    return p;
  };
  L.sbm = reinterpret_cast<uint64_t*>(take(64 * 8));
  L.start = reinterpret_cast<uint32_t*>(take(CAND * 4));
  L.w = reinterpret_cast<float*>(take(CAND * 4));
  L.prim = reinterpret_cast<uint32_t*>(take(CAND * 4));
  L.key = reinterpret_cast<uint16_t*>(take(CAND * 2));
  L.idx = reinterpret_cast<uint16_t*>(take(CAND * 2));
  L.ckey = reinterpret_cast<uint16_t*>(take(CAND * 2));
  L.spre = reinterpret_cast<uint32_t*>(take(64 * 4));
  L.bprim = reinterpret_cast<int32_t*>(take(kBlock * 4));
  L.blo = reinterpret_cast<int32_t*>(take(3 * kBlock * 4));
  L.bn = reinterpret_cast<int32_t*>(take(3 * kBlock * 4));
  L.boff = reinterpret_cast<int32_t*>(take(kBlock * 4));
  L.brec = reinterpret_cast<int32_t*>(take(kBlock * 9 * 4));
  L.bpatch = reinterpret_cast<int32_t*>(take(kBlock * 4));
  L.binv = reinterpret_cast<double*>(take(kBlock * 8));
  L.tmp32 = reinterpret_cast<int32_t*>(take((kWaves + 1) * 4));
  L.misc = reinterpret_cast<int32_t*>(take(8 * 4));
  return L;
}

// Load records [j0, j0 + kBlock) of the tile clipped to the unit box, keeping those with
// candidates in it (compacted, in record order, with a copy of their vertices); returns the
// batch's candidate total and the number of slots kept.  Contains __syncthreads().
template <int KIND>
__device__ __forceinline__ int32_t load_batch(const UnitLds& S, const int32_t* __restrict__ rec,
                                              const uint32_t* __restrict__ rprim, const float4* __restrict__ dirs,
                                              int64_t j0, int64_t e,
                                              const int32_t o[3], const int32_t sz[3], int& nslot) {
  const int64_t j = j0 + threadIdx.x;
  int32_t c = 0, lo[3], n[3];
  uint32_t p = 0;
  // the whole record (and the triangle's doubled area) in registers at once: one round of loads
  // after the primitive id, none after the scan below
  int32_t r[kRec];
  float a2 = 0.f;
  if (threadIdx.x < 64) S.sbm[threadIdx.x] = 0;
  if (j < e) {
    p = rprim[j];
    const int4* r4 = reinterpret_cast<const int4*>(rec + int64_t(p) * kRec);
#pragma unroll
    for (int k = 0; k < kRec / 4; ++k) {
      const int4 v = r4[k];
      r[4 * k] = v.x;
      r[4 * k + 1] = v.y;
      r[4 * k + 2] = v.z;
      r[4 * k + 3] = v.w;
    }
    if (KIND == 0) a2 = dirs[p].w;
    c = int32_t(clip_box(r, o, sz, lo, n));
  }
  // candidates (below 2^21 per batch) and kept slots (bits 21 and up) in one scan
  int32_t tot;
  const int32_t ex = block_exclusive_scan(c | (c > 0 ? (1 << 21) : 0), S.tmp32, tot);
  if (c > 0) {
    const int q = ex >> 21;
    const int32_t off = ex & ((1 << 21) - 1);
    S.bprim[q] = int32_t(p);
    S.boff[q] = off;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      S.blo[a * kBlock + q] = lo[a];
      S.bn[a * kBlock + q] = n[a];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) S.brec[q * 9 + k] = r[k];
    S.bpatch[q] = r[15];
    if (KIND == 1) S.binv[q] = cap_inv_len2(r);
    else S.binv[q] = double(a2);
    atomicOr(reinterpret_cast<unsigned long long*>(&S.sbm[off >> 6]), 1ull << (off & 63));
  }
  nslot = tot >> 21;
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t cnt = uint32_t(__popcll(S.sbm[threadIdx.x]));
    const uint32_t inc = wave_inclusive_scan(cnt);
    S.spre[threadIdx.x] = inc - cnt;
  }
  __syncthreads();
  return tot & ((1 << 21) - 1);
}

// voxel of candidate li (x fastest) of the record in batch slot `slot`.  li < 16^3 and extents
// <= 16: the quotients by float reciprocal are exact (the rounding error, below 1e-3, stays
// under the 1/32 margin of (li + 1/2) / n to the next integer)
__device__ __forceinline__ void slot_voxel(const UnitLds& S, int slot, int32_t li, int64_t v[3]) {
  const int32_t nx = S.bn[slot], ny = S.bn[kBlock + slot];
  const int32_t t = int32_t((float(li) + 0.5f) * __builtin_amdgcn_rcpf(float(nx)));
  const int32_t iz = int32_t((float(t) + 0.5f) * __builtin_amdgcn_rcpf(float(ny)));
  v[0] = S.blo[slot] + (li - t * nx);
  v[1] = S.blo[kBlock + slot] + (t - iz * ny);
  v[2] = S.blo[2 * kBlock + slot] + iz;
}

// candidate c (< 4096) of the batch -> its record slot: the slot starts at or below c, less one
__device__ __forceinline__ int find_slot(const UnitLds& S, int32_t c) {
  const int wd = c >> 6;
  return int(S.spre[wd] + uint32_t(__popcll(S.sbm[wd] & ((2ull << (c & 63)) - 1)))) - 1;
}

template <int KIND>
__device__ __forceinline__ bool unit_test(const int32_t* r, const int64_t v[3], const LatQ& Lp) {
  if (KIND == 0) return tri_touch(r, v, Lp.s, Lp.Sb);
  return cap_touch(r, v, Lp.s, Lp.Sb, Lp.rho);
}

template <int KIND>
__device__ __forceinline__ float unit_weight(const int32_t* r, const int64_t v[3], const LatQ& Lp, float len) {
  if (KIND == 0) return tri_area(r, v, Lp.Sb, len);
  return seg_length(r, v, Lp.Sb, len);
}
// the same, out of line: the rare streaming path keeps no second copy of the weight code
template <int KIND>
__device__ __attribute__((noinline)) float unit_weight_call(const int32_t* r, int64_t v0, int64_t v1, int64_t v2,
                                                            int Sb, float len) {
  const int64_t v[3] = {v0, v1, v2};
  if (KIND == 0) return tri_area(r, v, Sb, len);
  return seg_length(r, v, Sb, len);
}

// Staging of a unit's voxels (SoA, capacity cap); units claim contiguous ranges in any order.
struct Stage {
  void* key;          // u64, or u32 where the leaf's keys are 32-bit
  int key64;
  uint32_t* count;
  float* w;
  float* S;           // [6][cap]
  int64_t cap;
};

template <int KIND>
__device__ __forceinline__ void write_voxel(const Stage& st, int64_t i, uint64_t key, uint32_t cnt, const Moment& m) {
  if (st.key64) static_cast<uint64_t*>(st.key)[i] = key;
  else static_cast<uint32_t*>(st.key)[i] = uint32_t(key);
  st.count[i] = cnt;
  st.w[i] = m.W;
  st.S[i] = m.xx;
  st.S[st.cap + i] = m.yy;
  st.S[2 * st.cap + i] = m.zz;
  st.S[3 * st.cap + i] = m.xy;
  st.S[4 * st.cap + i] = m.xz;
  st.S[5 * st.cap + i] = m.yz;
}

template <int KIND, int CAND>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(unit_waves(CAND)))) k_unit(const int32_t* __restrict__ rec, const float4* __restrict__ dirs,
                                                 const uint32_t* __restrict__ rprim,
                                                 const int64_t* __restrict__ tstart, const Unit* __restrict__ units,
                                                 const int64_t* __restrict__ ctl, Lat L, const Lat* __restrict__ lats,
                                                 int64_t* __restrict__ unv, int64_t* __restrict__ unp,
                                                 int64_t* __restrict__ usoff, Stage st, int64_t* stage_ctr,
                                                 int64_t* stats) {
  extern __shared__ double lds_dyn[];
  static_assert(CAND <= 0xffff, "pair positions are 16-bit");
  static_assert(CAND % (kWaves * 64) == 0, "each wave's queue holds all of its candidates");
  const UnitLds S = carve_unit_lds<CAND>(reinterpret_cast<char*>(lds_dyn));
  const int64_t n_units = ctl[CTL_N_UNITS];
  const int tid = threadIdx.x;
  for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
    const Unit U = units[u];
    const int64_t s = tstart[U.tile], e = tstart[U.tile + 1];
    int32_t usz[3];
    unit_box(U.lev, U.ncell, usz);
    const uint64_t m0 = morton3(uint32_t(U.o[0]), uint32_t(U.o[1]), uint32_t(U.o[2]));   // the unit's first key
    const bool stream = U.cand > CAND;          // a single voxel holding too many candidates
    int32_t np = 0;                                   // pairs so far (uniform)
    Moment acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};   // streaming sums (thread 0)
    uint32_t acc_n = 0;
    for (int64_t j0 = s; j0 < e; j0 += kBlock) {
      int nb;
      const int32_t cb = load_batch<KIND>(S, rec, rprim, dirs, j0, e, U.o, usz, nb);
      (void)nb;
      if (stream) {
        for (int32_t c0 = 0; c0 < cb; c0 += kBlock) {
          const int32_t c = c0 + tid;
          bool hit = false;
          float wgt = 0.f;
          uint32_t p = 0;
          if (c < cb) {
            const int slot = find_slot(S, c);
            int64_t v[3];
            slot_voxel(S, slot, c - S.boff[slot], v);
            p = uint32_t(S.bprim[slot]);
            const int32_t* r = S.brec + slot * 9;
            const LatQ Lp = lat_q(lats, S.bpatch[slot], L);
            hit = unit_test<KIND>(r, v, Lp);
            if (hit) wgt = unit_weight_call<KIND>(r, v[0], v[1], v[2], Lp.Sb, dirs[p].w);
          }
          int32_t tot;
          const int32_t pos = block_exclusive_scan(int32_t(hit), S.tmp32, tot);
          // one voxel: sum this chunk's hits in order (thread 0), chunk by chunk
          if (hit) {
            S.w[pos] = wgt;
            S.prim[pos] = p;
          }
          __syncthreads();
          if (tid == 0) {
            for (int32_t i = 0; i < tot; ++i) accum_pair<KIND>(acc, S.w[i], dirs[S.prim[i]]);
            acc_n += uint32_t(tot);
          }
          np += tot;
          __syncthreads();
        }
        continue;
      }
      // Test in two rounds so that lanes stay busy: a cheap filter decides most candidates and
      // queues the rest (fibers: the centre-ball filter), then the queue gets the full test.
      // Each wave works on its own candidates and drains its own queue (a quarter of the queue
      // space: a wave holds at most a quarter of a unit's candidates); every candidate records
      // its outcome in place, and the touching ones are then compacted in candidate order,
      // which is primitive order.
      const int wv = tid >> 6, lane = tid & 63;
      const uint64_t lt = (uint64_t(1) << lane) - 1;
      uint32_t* wq = reinterpret_cast<uint32_t*>(S.w) + wv * (CAND / kWaves);
      int32_t nq = 0;                                  // this wave's queue (uniform)
      for (int32_t c0 = wv * 64; c0 < cb; c0 += kBlock) {
        const int32_t c = c0 + lane;
        int res = 0;                                   // 0 miss, 1 touch, 2 undecided
        if (c < cb) {
          const int slot = find_slot(S, c);
          int64_t v[3];
          slot_voxel(S, slot, c - S.boff[slot], v);
          const int32_t* r = S.brec + slot * 9;
          const LatQ Lp = lat_q(lats, S.bpatch[slot], L);
          if (KIND == 0) {
            res = tri_touch(r, v, Lp.s, Lp.Sb) ? 1 : 0;
          } else {
            const int b = cap_ball(r, v, Lp.s, Lp.Sb, Lp.rho, S.binv[slot]);
            res = b < 0 ? 2 : b;
          }
          S.ckey[c] = res == 1 ? uint16_t(kTouch | (morton3(uint32_t(v[0]), uint32_t(v[1]), uint32_t(v[2])) - m0))
                               : (res == 2 ? kUndecided : uint16_t(0));
        }
        const uint64_t mb = __ballot(res == 2);
        if (res == 2) wq[nq + int32_t(__popcll(mb & lt))] = uint32_t(c);
        nq += int32_t(__popcll(mb));
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      for (int32_t q = lane; KIND == 1 && q < nq; q += 64) {
        const int32_t c = int32_t(wq[q]);
        const int slot = find_slot(S, c);
        int64_t v[3];
        slot_voxel(S, slot, c - S.boff[slot], v);
        const int32_t* r = S.brec + slot * 9;
        const LatQ Lp = lat_q(lats, S.bpatch[slot], L);
        const bool hit = cap_bracket(r, v, Lp.s, Lp.Sb, Lp.rho);
        S.ckey[c] = hit ? uint16_t(kTouch | (morton3(uint32_t(v[0]), uint32_t(v[1]), uint32_t(v[2])) - m0)) : uint16_t(0);
      }
      __syncthreads();
      // ordered compaction: wave w takes candidates [w span, (w + 1) span)
      {
        const int32_t span = ((cb + kWaves * 64 - 1) / (kWaves * 64)) * 64;
        const int32_t w0 = wv * span, w1 = w0 + span < cb ? w0 + span : cb;
        int32_t cnt = 0;
        for (int32_t c0 = w0; c0 < w1; c0 += 64) {
          const int32_t c = c0 + lane;
          cnt += int32_t(__popcll(__ballot(c < w1 && (S.ckey[c] & kTouch) != 0)));
        }
        if (lane == 0) S.tmp32[wv] = cnt;
        __syncthreads();
        int32_t base = np, tot = 0;
        for (int i = 0; i < kWaves; ++i) {
          if (i < wv) base += S.tmp32[i];
          tot += S.tmp32[i];
        }
        for (int32_t c0 = w0; c0 < w1; c0 += 64) {
          const int32_t c = c0 + lane;
          const bool hit = c < w1 && (S.ckey[c] & kTouch) != 0;
          const uint64_t mh = __ballot(hit);
          if (hit) {
            const int32_t q = base + int32_t(__popcll(mh & lt));
            if (q < CAND) {
              const int sl = find_slot(S, c);
              S.key[q] = uint16_t(S.ckey[c] & (kTouch - 1));
              S.prim[q] = uint32_t(S.bprim[sl]);
              if (KIND == 0) S.idx[q] = uint16_t(sl);
            } else {
              flag_set(stats, VX_FLAG_UNIT_CAPACITY);   // planning and test disagree: never expected
            }
          }
          base += int32_t(__popcll(mh));
        }
        // triangles: the batch's pairs are weighed now, from the records still in LDS
        if (KIND == 0) {
          __syncthreads();
          const int32_t q1 = np + tot < CAND ? np + tot : CAND;
          for (int32_t q = np + tid; q < q1; q += kBlock) {
            const int sl = S.idx[q];
            const uint64_t m = m0 + S.key[q];
            const int64_t v[3] = {int64_t(compact3(m)), int64_t(compact3(m >> 1)), int64_t(compact3(m >> 2))};
            const LatQ Lp = lat_q(lats, S.bpatch[sl], L);
            S.w[q] = unit_weight<KIND>(S.brec + sl * 9, v, Lp, float(S.binv[sl]));
          }
        }
        np += tot;
        __syncthreads();
      }
    }
    if (stream) {
      if (tid == 0) {
        const int64_t nv = acc_n > 0 ? 1 : 0;
        int64_t b = 0;
        if (nv) {
          b = int64_t(atomicAdd(reinterpret_cast<unsigned long long*>(stage_ctr), 1ull));
          const uint64_t key = morton3(uint32_t(U.o[0]), uint32_t(U.o[1]), uint32_t(U.o[2])) |
                               (lats ? uint64_t(uint32_t(rec[int64_t(rprim[s]) * kRec + 15])) << kPatchShift : 0ull);
          if (b < st.cap) write_voxel<KIND>(st, b, key, acc_n, acc);
          else flag_set(stats, VX_FLAG_VOXEL_CAPACITY);
        }
        unv[u] = nv;
        unp[u] = np;
        usoff[u] = b;
      }
      __syncthreads();
      continue;
    }
    const int32_t npairs = np < CAND ? np : CAND;
    // Group the pairs by voxel with one counter per key of the unit's range (at most 4096 keys;
    // 16-bit counts packed two to a word, in the record batch's space, dead now); the fibers'
    // weights are computed in the same pass.  Each pair keeps its arrival slot among its voxel's
    // pairs.
    uint32_t* kcw = reinterpret_cast<uint32_t*>(S.brec);                 // [2048] packed counts
    uint16_t* kst = reinterpret_cast<uint16_t*>(S.brec);                 // [4096] then starts
    uint16_t* slot = S.ckey;                                              // [npairs]
    uint16_t* vkey = reinterpret_cast<uint16_t*>(S.start);               // [nv] key of voxel v
    uint16_t* vend = reinterpret_cast<uint16_t*>(S.start) + CAND;   // [nv] end of its pairs
    for (int32_t j = tid; j < kUnitKeys / 2; j += kBlock) kcw[j] = 0u;
    __syncthreads();
    for (int32_t i = tid; i < npairs; i += kBlock) {
      const uint32_t p = S.prim[i], k = S.key[i];
      const uint32_t sh = 16u * (k & 1u);
      slot[i] = uint16_t(atomicAdd(&kcw[k >> 1], 1u << sh) >> sh);
      if (KIND == 1) {                            // (triangles were weighed batch by batch)
        const int32_t* r = rec + int64_t(p) * kRec;
        const LatQ Lp = lat_q(lats, r[15], L);
        const uint64_t m = m0 + k;
        const int64_t v[3] = {int64_t(compact3(m)), int64_t(compact3(m >> 1)), int64_t(compact3(m >> 2))};
        S.w[i] = unit_weight<KIND>(r, v, Lp, dirs[p].w);
      }
    }
    __syncthreads();
    // starts and the voxel list: thread t owns keys [16 t, 16 t + 16); one block scan of the
    // (pairs, voxels) counts packed in one word (at most 3072 pairs and 4096 voxels)
    int32_t nv;
    {
      uint32_t c[16];
      uint32_t sp = 0, sv = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint32_t w2 = kcw[tid * 8 + j];
        c[2 * j] = w2 & 0xffffu;
        c[2 * j + 1] = w2 >> 16;
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        sp += c[k];
        sv += c[k] != 0u ? 1u : 0u;
      }
      int32_t tot;
      const uint32_t pre = uint32_t(block_exclusive_scan(int32_t(sp | (sv << 16)), S.tmp32, tot));
      nv = tot >> 16;
      uint32_t rp = pre & 0xffffu, rv = pre >> 16;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t key = uint32_t(tid) * 16u + uint32_t(k);
        kst[key] = uint16_t(rp);
        if (c[k] != 0u) {
          vkey[rv] = uint16_t(key);
          vend[rv] = uint16_t(rp + c[k]);
          ++rv;
        }
        rp += c[k];
      }
    }
    if (tid == 0) {
      // claim the staging range now; the claim's round trip overlaps the placement below
      const int64_t b = nv ? int64_t(atomicAdd(reinterpret_cast<unsigned long long*>(stage_ctr),
                                               (unsigned long long)nv))
                           : 0;
      S.misc[1] = int32_t(b & 0xffffffff);
      S.misc[2] = int32_t(b >> 32);
      if (b + nv > st.cap) flag_set(stats, VX_FLAG_VOXEL_CAPACITY);
      unv[u] = nv;
      unp[u] = np;
      usoff[u] = b;
    }
    __syncthreads();
    // Place the pairs by voxel.  Sparse units (few pairs per voxel) place by arrival slot and
    // restore primitive order per voxel by insertion sort below; dense ones place stably: one
    // wave walks the list (primitive order) and lanes holding the same key find each other by
    // ballots over the 12 key bits.
    const bool stable = npairs > stable_mean<KIND>() * nv;
    if (!stable) {
      for (int32_t i = tid; i < npairs; i += kBlock) S.idx[kst[S.key[i]] + slot[i]] = uint16_t(i);
    } else if (tid < 64) {
      const uint64_t lt = (uint64_t(1) << tid) - 1;
      for (int32_t i0 = 0; i0 < npairs; i0 += 64) {
        const int32_t i = i0 + tid;
        const bool ok = i < npairs;
        const uint32_t k = ok ? uint32_t(S.key[i]) : 0u;
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 12; ++bit) {
          const uint64_t m = __ballot((k >> bit) & 1);
          peers &= ((k >> bit) & 1) ? m : ~m;
        }
        uint32_t q = 0;
        if (ok) q = uint32_t(kst[k]) + uint32_t(__popcll(peers & lt));
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (ok) {
          S.idx[q] = uint16_t(i);
          if ((peers & lt) == 0) kst[k] = uint16_t(kst[k] + uint32_t(__popcll(peers)));   // the group's first lane
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
    }
    __syncthreads();
    const int64_t b = int64_t(uint32_t(S.misc[1])) | (int64_t(S.misc[2]) << 32);
    const uint64_t hi = lats ? uint64_t(uint32_t(rec[int64_t(rprim[s]) * kRec + 15])) << kPatchShift : 0ull;
    if (b + nv <= st.cap) {
      for (int32_t v = tid; v < nv; v += kBlock) {
        const uint32_t a = v ? uint32_t(vend[v - 1]) : 0u, z = vend[v];
        // the voxel's pairs in list order, which is primitive order (insertion sort)
        for (uint32_t i = a + 1; !stable && i < z; ++i) {
          const uint16_t x = S.idx[i];
          uint32_t j = i;
          while (j > a && S.idx[j - 1] > x) {
            S.idx[j] = S.idx[j - 1];
            --j;
          }
          S.idx[j] = x;
        }
        Moment m{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (uint32_t i0 = a; i0 < z; i0 += 8) {
          // the loads of a group do not wait for each other, the sums stay in order
          float4 t[8];
          float wv[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            if (i0 + k < z) {
              const uint16_t x = S.idx[i0 + k];
              t[k] = dirs[S.prim[x]];
              wv[k] = S.w[x];
            }
          }
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (i0 + k < z) accum_pair<KIND>(m, wv[k], t[k]);
        }
        write_voxel<KIND>(st, b + v, hi | (m0 + vkey[v]), z - a, m);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------------
// totals and the final, dense leaf
// ---------------------------------------------------------------------------------------------
struct VoxTotal {
  int64_t* pos;
  int64_t* ctl;
  int64_t* stats;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    pos[n] = total;
    stats[VX_STAT_VOXELS] = total;
    const bool over = total > cap;
    if (over) flag_set(stats, VX_FLAG_VOXEL_CAPACITY);
    ctl[CTL_N_VOX] = over ? 0 : total;
  }
};
struct SumTotal {
  int64_t* dst;
  __device__ void operator()(int64_t total, int64_t) const { *dst = total; }
};
struct NoOut {
  __device__ void operator()(int64_t, int64_t, int64_t) const {}
};
struct UnitCand {
  const Unit* u;
  __device__ int64_t operator()(int64_t i) const { return u[i].cand; }
};

// The three unit-level sums after the unit kernel in one two-kernel scan: totals of the pairs and
// of the candidates (statistics) and the exclusive scan of the voxels per unit (leaf positions).
// Same chunking as device_scan; partial holds 3 values per block.
__global__ void __launch_bounds__(kBlock) k_unit_sums_partial(const int64_t* __restrict__ unp,
                                                              const Unit* __restrict__ units,
                                                              const int64_t* __restrict__ unv,
                                                              const int64_t* __restrict__ ctl,
                                                              int64_t* __restrict__ partial) {
  __shared__ int64_t red[3][kWaves];
  const int64_t n = ctl[CTL_N_UNITS];
  const int64_t chunk = scan_chunk(n);
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  int64_t ap = 0, ac = 0, av = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
    ap += unp[i];
    ac += units[i].cand;
    av += unv[i];
  }
  ap = wave_sum(ap);
  ac = wave_sum(ac);
  av = wave_sum(av);
  if (lane_id() == 0) {
    red[0][threadIdx.x >> 6] = ap;
    red[1][threadIdx.x >> 6] = ac;
    red[2][threadIdx.x >> 6] = av;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    int64_t t = 0;
    for (int i = 0; i < kWaves; ++i) t += red[threadIdx.x][i];
    partial[3 * blockIdx.x + threadIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock) k_unit_sums_apply(const int64_t* __restrict__ unv,
                                                            int64_t* __restrict__ ctl,
                                                            const int64_t* __restrict__ partial,
                                                            int64_t* __restrict__ upos, int64_t* __restrict__ stats,
                                                            int64_t cap) {
  __shared__ int64_t tmp[kWaves + 1];
  const int64_t n = ctl[CTL_N_UNITS];
  const int64_t chunk = scan_chunk(n);
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  int64_t pre = 0, tp = 0, tc = 0, tv = 0;
  for (int i = threadIdx.x; i < kGrid; i += kBlock) {
    const int64_t v = partial[3 * i + 2];
    if (i < int(blockIdx.x)) pre += v;
    if (blockIdx.x == 0) {
      tp += partial[3 * i];
      tc += partial[3 * i + 1];
      tv += v;
    }
  }
  int64_t base;
  (void)block_exclusive_scan(pre, tmp, base);
  if (blockIdx.x == 0) {
    int64_t t;
    (void)block_exclusive_scan(tp, tmp, t);
    if (threadIdx.x == 0) stats[VX_STAT_PAIRS] = t;
    (void)block_exclusive_scan(tc, tmp, t);
    if (threadIdx.x == 0) stats[VX_STAT_CAND] = t;
    (void)block_exclusive_scan(tv, tmp, t);
    if (threadIdx.x == 0) VoxTotal{upos, ctl, stats, cap}(t, n);
  }
  if (b0 >= b1) return;
  for (int64_t t0 = b0; t0 < b1; t0 += kBlock) {
    const int64_t i = t0 + threadIdx.x;
    const int64_t v = i < b1 ? unv[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, tmp, tot);
    if (i < b1) upos[i] = base + ex;
    base += tot;
  }
}

// one block per unit: copy its staged voxels to their place in the leaf
template <class Key>
__global__ void __launch_bounds__(kBlock) k_unit_compact(const int64_t* __restrict__ unv,
                                                         const int64_t* __restrict__ usoff,
                                                         const int64_t* __restrict__ upos,
                                                         const int64_t* __restrict__ ctl, Stage st, vx_voxels out) {
  const int64_t n_units = ctl[CTL_N_UNITS];
  if (ctl[CTL_N_VOX] == 0) return;
  Key* okeys = reinterpret_cast<Key*>(out.keys);
  for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
    const int64_t n = unv[u], src = usoff[u], dst = upos[u];
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
      okeys[dst + i] = static_cast<const Key*>(st.key)[src + i];
      out.count[dst + i] = st.count[src + i];
      out.w[dst + i] = st.w[src + i];
#pragma unroll
      for (int c = 0; c < 6; ++c) out.S[c * out.cap + dst + i] = st.S[c * st.cap + src + i];
    }
  }
}

// ---------------------------------------------------------------------------------------------
// orchestration
// ---------------------------------------------------------------------------------------------
struct TileWs {
  int64_t* ctl;
  int32_t* rec;
  float4* dirs;
  int64_t* cand_cnt;
  int64_t* roff;          // [n_prims + 1]
  ulonglong2* box;        // [n_prims] packed candidate boxes
  PairBufs ra, rb;        // records (tile key, primitive; no weight), ping-pong
  int32_t* hist;
  int64_t* partial;
  int64_t* tstart;        // [max_records + 1]
  int64_t* ucnt;          // [max_records + 1] units per tile, then their offsets
  int64_t* uoff;
  Unit* units;            // [max_units]
  int64_t* unv;           // [max_units + 1]
  int64_t* unp;
  int64_t* usoff;
  int64_t* upos;          // [max_units + 1]
  int64_t* stage_ctr;
  Stage st;
};

static size_t tile_ws_layout(int64_t n_prims, int64_t max_rec, int64_t max_units, int64_t max_vox, bool key64,
                             void* base, TileWs* w) {
  Carver cv(base);
  TileWs x;
  const int kb = key64 ? 8 : 4;
  x.ctl = cv.take<int64_t>(CTL_SIZE);
  x.rec = cv.take<int32_t>(n_prims * kRec);
  x.dirs = cv.take<float4>(n_prims);
  x.cand_cnt = cv.take<int64_t>(n_prims);
  x.roff = cv.take<int64_t>(n_prims + 1);
  x.box = cv.take<ulonglong2>(n_prims);
  x.ra.keys = cv.take<uint8_t>(max_rec * kb);
  x.ra.w = nullptr;
  x.ra.prim = cv.take<uint32_t>(max_rec);
  x.rb.keys = cv.take<uint8_t>(max_rec * kb);
  x.rb.w = nullptr;
  x.rb.prim = cv.take<uint32_t>(max_rec);
  x.hist = cv.take<int32_t>(int64_t(kRadixBuckets) * kGrid);
  x.partial = cv.take<int64_t>(3 * kGrid + 1);     // 3 values per block for the unit sums
  x.tstart = cv.take<int64_t>(max_rec + 1);
  x.ucnt = cv.take<int64_t>(max_rec + 1);
  x.uoff = cv.take<int64_t>(max_rec + 1);
  x.units = cv.take<Unit>(max_units);
  x.unv = cv.take<int64_t>(max_units + 1);
  x.unp = cv.take<int64_t>(max_units + 1);
  x.usoff = cv.take<int64_t>(max_units + 1);
  x.upos = cv.take<int64_t>(max_units + 1);
  x.stage_ctr = cv.take<int64_t>(1);
  x.st.key = cv.take<uint8_t>(max_vox * kb);
  x.st.key64 = key64 ? 1 : 0;
  x.st.count = cv.take<uint32_t>(max_vox);
  x.st.w = cv.take<float>(max_vox);
  x.st.S = cv.take<float>(6 * max_vox);
  x.st.cap = max_vox;
  if (w) *w = x;
  return cv.off + 256;
}

size_t tile_ws_bytes(int64_t n_prims, int64_t max_rec, int64_t max_units, int64_t max_vox, bool key64) {
  return tile_ws_layout(n_prims, max_rec, max_units, max_vox, key64, nullptr, nullptr);
}

struct ArrIn64 {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};
struct UnitCountIn {                 // units per tile: the low half of the planner's count word
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i] & 0xffffffff; }
};
struct ArrOut64 {
  int64_t* o;
  __device__ void operator()(int64_t i, int64_t ex, int64_t) const { o[i] = ex; }
};

vx_status tile_voxelize(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                        int64_t n_fib, float radius, int64_t max_rec, int64_t max_units, void* ws_ptr,
                        const vx_voxels* out, int64_t* stats, hipStream_t s, const BatchLattice* batch, int tb,
                        const Tuning& tu) {
  const bool key64 = batch || g->log2_res > 10;
  TileWs w;
  tile_ws_layout(n_prims, max_rec, max_units, out->cap, key64, ws_ptr, &w);
  // prep (snap, candidate boxes) is shared with the pair path
  FrontWs f{};
  f.ctl = w.ctl;
  f.rec = w.rec;
  f.dirs = w.dirs;
  f.cand_cnt = w.cand_cnt;
  f.partial = w.partial;
  f.fstart = reinterpret_cast<uint8_t*>(w.roff);       // free until the record counts
  if (kind == 0) {                                      // triangles: the prep counts the records
    f.rcnt = w.roff;
    f.tb = tb;
  }
  f.box = w.box;
  prep_prims(kind, g, data, n_prims, offsets, n_fib, radius, f, stats, s, batch, w.stage_ctr, 1);
  const int pgrid = int(n_prims / kBlock + 1 < kPrimGrid ? n_prims / kBlock + 1 : kPrimGrid);
  {
    VX_TIMED("tile_records", s);
    // fibers: their fiber-start bytes share the counts' space, so the count is a pass of its own
    if (kind != 0)
      hipLaunchKernelGGL(k_rec_count, dim3(pgrid), dim3(kBlock), 0, s, w.box, w.cand_cnt, n_prims, tb, w.roff);
    device_scan(ArrIn64{w.roff}, ArrOut64{w.roff}, RecTotal{w.roff, w.ctl, stats, max_rec}, nullptr, n_prims,
                w.partial, s);
    if (key64)
      hipLaunchKernelGGL(k_rec_emit<uint64_t>, dim3(pgrid), dim3(kBlock), 0, s, w.rec, w.box, w.roff, n_prims, w.ctl, tb,
                         batch ? 1 : 0, (uint64_t*)w.ra.keys, w.ra.prim);
    else
      hipLaunchKernelGGL(k_rec_emit<uint32_t>, dim3(pgrid), dim3(kBlock), 0, s, w.rec, w.box, w.roff, n_prims, w.ctl, tb, 0,
                         (uint32_t*)w.ra.keys, w.ra.prim);
  }
  int key_bits = 3 * (g->log2_res - tb);
  if (batch) {
    int pb = 1;
    while ((1 << pb) < batch->n_patches) ++pb;
    key_bits = kPatchShift - 3 * tb + pb;
  }
  // the records carry no weight: the sort moves keys and primitive ids only
  const int res = radix_sort_pairs(key64, key_bits, w.ra, w.rb, w.ctl + CTL_N_REC, max_rec, w.hist, w.partial, s);
  const PairBufs R = res ? w.rb : w.ra;
  {
    VX_TIMED("tile_heads", s);
    if (key64)
      device_scan(HeadIn<uint64_t, 0>{(const uint64_t*)R.keys}, HeadOut{w.tstart}, TileTotal{w.tstart, w.ctl},
                  w.ctl + CTL_N_REC, 0, w.partial, s);
    else
      device_scan(HeadIn<uint32_t, 0>{(const uint32_t*)R.keys}, HeadOut{w.tstart}, TileTotal{w.tstart, w.ctl},
                  w.ctl + CTL_N_REC, 0, w.partial, s);
  }
  {
    VX_TIMED("unit_plan", s);
    const int grid = tu.grids[kTunePlan];
    const int64_t budget = tu.unit_budget;
#define VX_PLAN(P, K)                                                                                        \
  hipLaunchKernelGGL((k_unit_plan<P, K>), dim3(grid), dim3(kBlock), 0, s, w.box, (const K*)R.keys, R.prim, w.tstart, \
                     w.ctl, tb, batch ? 1 : 0, budget, w.ucnt, w.uoff, w.units)
    if (key64) VX_PLAN(0, uint64_t); else VX_PLAN(0, uint32_t);
    device_scan(UnitCountIn{w.ucnt}, ArrOut64{w.uoff}, UnitTotal{w.uoff, w.ctl, stats, max_units}, w.ctl + CTL_N_TILES,
                0, w.partial, s);
    if (key64) VX_PLAN(1, uint64_t); else VX_PLAN(1, uint32_t);
#undef VX_PLAN
  }
  {
    VX_TIMED(kind == 0 ? "unit_tri" : "unit_fib", s);
    const Lat L = make_lat(g, kind, radius);
    const Lat* lats = batch ? batch->lats : nullptr;
    const int ugrid = tu.grids[kTuneUnit];
#define VX_UNIT(KD, C)                                                                                           \
  do {                                                                                                          \
    static bool attr_ = false;                                                                                  \
    if (!attr_) {                                                                                               \
      (void)hipFuncSetAttribute((const void*)k_unit<KD, C>, hipFuncAttributeMaxDynamicSharedMemorySize,        \
                                int(unit_lds_bytes<C>()));                                                      \
      attr_ = true;                                                                                             \
    }                                                                                                           \
    hipLaunchKernelGGL((k_unit<KD, C>), dim3(ugrid), dim3(kBlock), unit_lds_bytes<C>(), s, w.rec, w.dirs, R.prim, \
                       w.tstart, w.units, w.ctl, L, lats, w.unv, w.unp, w.usoff, w.st, w.stage_ctr, stats);    \
  } while (0)
#define VX_UNIT_KIND(KD)                                        \
  switch (tu.unit_budget) {                                     \
    case 1024: VX_UNIT(KD, 1024); break;                        \
    case 1536: VX_UNIT(KD, 1536); break;                        \
    case 2048: VX_UNIT(KD, 2048); break;                        \
    default: VX_UNIT(KD, 3072); break;                          \
  }
    if (kind == 0) {
      VX_UNIT_KIND(0);
    } else {
      VX_UNIT_KIND(1);
    }
#undef VX_UNIT_KIND
#undef VX_UNIT
  }
  {
    VX_TIMED("unit_compact", s);
    hipLaunchKernelGGL(k_unit_sums_partial, dim3(kGrid), dim3(kBlock), 0, s, w.unp, w.units, w.unv, w.ctl,
                       w.partial);
    hipLaunchKernelGGL(k_unit_sums_apply, dim3(kGrid), dim3(kBlock), 0, s, w.unv, w.ctl, w.partial, w.upos, stats,
                       out->cap);
    if (key64)
      hipLaunchKernelGGL(k_unit_compact<uint64_t>, dim3(tu.grids[kTuneCompact]), dim3(kBlock), 0, s, w.unv,
                         w.usoff, w.upos, w.ctl, w.st, *out);
    else
      hipLaunchKernelGGL(k_unit_compact<uint32_t>, dim3(tu.grids[kTuneCompact]), dim3(kBlock), 0, s, w.unv,
                         w.usoff, w.upos, w.ctl, w.st, *out);
  }
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

}  // namespace vx
