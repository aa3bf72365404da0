// prims.hip -- per-primitive work of the voxelizer on gfx950:
//   prep  : Sec. 3.1 grid transform snapped to the lattice, candidate voxel ranges;
//   test  : exact closed-box touch test per candidate, wave ballot -> 64-bit survivor masks;
//   emit  : weight (clipped area / length) and Morton key per survivor, written at offsets
//           from a scan of the mask popcounts (deterministic order, no atomics).
// The paper generates point samples per primitive and bins them (Sec. 3.2-3.3); here every
// (primitive, voxel) overlap is found exactly and carries its exact measure instead.
#include "geom.hpp"
#include "vx_internal.hpp"

namespace vx {

__device__ __forceinline__ void flag_or(int64_t* stats, int64_t bit) {
  atomicOr(reinterpret_cast<unsigned long long*>(stats + VX_STAT_FLAGS), (unsigned long long)bit);
}

// ---------------------------------------------------------------------------------------------
// prep
// ---------------------------------------------------------------------------------------------
// a record (16 x int32, 64-byte aligned) as four 16-byte stores
__device__ __forceinline__ void store_record(int32_t* __restrict__ dst, const int32_t (&r)[kRec]) {
  int4* d = reinterpret_cast<int4*>(dst);
#pragma unroll
  for (int k = 0; k < kRec / 4; ++k) d[k] = make_int4(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]);
}

// rcnt (optional): the number of aligned tiles of 2^tb voxels per axis that the candidate box
// overlaps (0 without candidates), for the tiled path's primitive-tile records
__global__ void __launch_bounds__(kBlock) k_prep_tri(const float* __restrict__ tris, int64_t n, Lat L,
                                                     int32_t* __restrict__ rec, float4* __restrict__ dirs,
                                                     int64_t* __restrict__ cand_cnt, int64_t* __restrict__ rcnt,
                                                     int tb, ulonglong2* __restrict__ box, int64_t* stats) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    bool ok;
    int32_t r[kRec];                                 // built in registers, stored as 4 x 16 bytes
    const int64_t cc = prep_triangle(tris + i * 9, L, r, dirs + i, ok);
    if (!rcnt) cand_cnt[i] = cc;                   // (the tiled path reads only the record counts)
    store_record(rec + i * kRec, r);
    if (box) box[i] = pack_box(r);
    if (rcnt) {
      int64_t c = 0;
      if (cc > 0) {
        c = 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) c *= int64_t(((r[9 + a] + r[12 + a] - 1) >> tb) - (r[9 + a] >> tb) + 1);
      }
      rcnt[i] = c;
    }
    if (!ok) flag_or(stats, VX_FLAG_INPUT);
  }
}

// One thread per point: point i starts segment (i, i+1) when both belong to the same fiber.
__global__ void __launch_bounds__(kBlock) k_prep_fib(const float* __restrict__ pts, int64_t n_pts,
                                                     const uint8_t* __restrict__ fstart, Lat L,
                                                     int32_t* __restrict__ rec, float4* __restrict__ dirs,
                                                     int64_t* __restrict__ cand_cnt, ulonglong2* __restrict__ box,
                                                     int64_t* stats) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_pts; i += int64_t(gridDim.x) * kBlock) {
    // point i and the next make a segment unless the next starts a fiber (offsets are
    // non-decreasing, so a later point of the same fiber starts none)
    const bool seg = (i + 1 < n_pts) && !fstart[i + 1];
    bool ok;
    int32_t r[kRec];
    cand_cnt[i] = prep_segment(pts + i * 3, seg ? pts + (i + 1) * 3 : nullptr, L, r, dirs + i, ok);
    store_record(rec + i * kRec, r);
    if (box) box[i] = pack_box(r);
    if (!ok) flag_or(stats, VX_FLAG_INPUT);
  }
}

// Batched fibers: patch p owns points [pt_begin[p], pt_begin[p+1]) and is snapped to its own
// lattice; the record keeps the patch id in its last slot.
__global__ void __launch_bounds__(kBlock) k_prep_fib_batch(const float* __restrict__ pts, int64_t n_pts,
                                                           const uint8_t* __restrict__ fstart,
                                                           const Lat* __restrict__ lats,
                                                           const int64_t* __restrict__ pt_begin, int n_patches,
                                                           int32_t* __restrict__ rec, float4* __restrict__ dirs,
                                                           int64_t* __restrict__ cand_cnt,
                                                           ulonglong2* __restrict__ box, int64_t* stats) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_pts; i += int64_t(gridDim.x) * kBlock) {
    int lo = 0, hi = n_patches;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pt_begin[mid] <= i) lo = mid; else hi = mid;
    }
    const int patch = lo;
    const bool seg = (i + 1 < n_pts) && !fstart[i + 1] && (i + 1 < pt_begin[patch + 1]);
    bool ok;
    int32_t r[kRec];
    cand_cnt[i] = prep_segment(pts + i * 3, seg ? pts + (i + 1) * 3 : nullptr, lats[patch], r, dirs + i, ok);
    r[15] = patch;
    store_record(rec + i * kRec, r);
    if (box) box[i] = pack_box(r);
    if (!ok) flag_or(stats, VX_FLAG_INPUT);
  }
}

// also marks the first point of every fiber (fstart cleared beforehand)
__global__ void k_check_offsets(const int64_t* __restrict__ offsets, int64_t n_fib, int64_t n_pts,
                                uint8_t* __restrict__ fstart, int64_t* stats) {
  for (int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; f <= n_fib; f += int64_t(gridDim.x) * blockDim.x) {
    if (f < n_fib) {
      const int64_t o = offsets[f];
      if (o >= 0 && o < n_pts) fstart[o] = 1;
    }
    bool bad = false;
    if (f == 0) bad = offsets[0] != 0;
    else bad = offsets[f] < offsets[f - 1];
    if (f == n_fib) bad = bad || offsets[n_fib] != n_pts;
    if (bad) flag_or(stats, VX_FLAG_OFFSETS);
  }
}


// ---------------------------------------------------------------------------------------------
// test: one wave per 64 candidates
// ---------------------------------------------------------------------------------------------
// chunk_prim[ch]: the primitive holding candidate 64 ch, one bisection per chunk (independent
// threads, so the dependent loads of many chunks overlap)
__global__ void __launch_bounds__(kBlock) k_chunk_start(const int64_t* __restrict__ cand_off, int64_t n_prims,
                                                        const int64_t* __restrict__ ctl,
                                                        int64_t* __restrict__ chunk_prim) {
  const int64_t n_chunks = ctl[CTL_N_CHUNKS];
  for (int64_t ch = int64_t(blockIdx.x) * kBlock + threadIdx.x; ch < n_chunks; ch += int64_t(gridDim.x) * kBlock)
    chunk_prim[ch] = find_prim_bisect(cand_off, n_prims, ch * 64);
}

// Primitive of candidate ci for every lane of a wave whose chunk starts in primitive p0 (all 64
// lanes call it): the starts of the next 64 primitives are loaded once, coalesced, and each lane
// counts those at or below its candidate with a 6-step search across lanes; a lane past all of
// them (more than 63 primitives begin inside the chunk) continues by galloping.
__device__ __forceinline__ int64_t wave_find_prim(const int64_t* __restrict__ cand_off, int64_t p0, int64_t n_prims,
                                                  int64_t ci) {
  const int64_t j = p0 + 1 + lane_id();
  const int64_t b = j < n_prims ? cand_off[j] : INT64_MAX;
  int k = 0;
#pragma unroll
  for (int step = 32; step > 0; step >>= 1) {
    const int64_t bk = __shfl(b, k + step - 1, 64);
    if (bk <= ci) k += step;
  }
  const int64_t b63 = __shfl(b, 63, 64);
  if (k == 63 && b63 <= ci) return find_prim(cand_off, p0 + 64, n_prims, ci);
  return p0 + k;
}

// ---------------------------------------------------------------------------------------------
// test: one wave per 64 candidates
// ---------------------------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_test(const int32_t* __restrict__ rec, const int64_t* __restrict__ cand_off,
                                                 int64_t n_prims, const int64_t* __restrict__ ctl, Lat L,
                                                 const Lat* __restrict__ lats, uint64_t* __restrict__ masks,
                                                 const int64_t* __restrict__ chunk_prim) {
  const int64_t n_cand = ctl[CTL_N_CAND];
  const int64_t n_chunks = ctl[CTL_N_CHUNKS];
  const int64_t w0 = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  const int64_t ws = int64_t(gridDim.x) * kWaves;
  for (int64_t ch = w0; ch < n_chunks; ch += ws) {
    const int64_t ci = ch * 64 + lane_id();
    const int64_t p = wave_find_prim(cand_off, chunk_prim[ch], n_prims, ci);
    bool hit = false;
    if (ci < n_cand) {
      const int32_t* r = rec + p * kRec;
      int64_t v[3];
      candidate_voxel(r, ci - cand_off[p], v);
      const LatQ Lp = lat_q(lats, r[15], L);          // batched patches: the primitive's own lattice
      if (KIND == 0) hit = tri_touch(r, v, Lp.s, Lp.Sb);
      else hit = cap_touch(r, v, Lp.s, Lp.Sb, Lp.rho);
    }
    const uint64_t m = __ballot(hit);
    if (lane_id() == 0) masks[ch] = m;
  }
}

// ---------------------------------------------------------------------------------------------
// emit: survivors write (key, weight, primitive) at scan offsets
// ---------------------------------------------------------------------------------------------
template <int KIND, class Key>
__global__ void __launch_bounds__(kBlock) k_emit(const int32_t* __restrict__ rec, const float4* __restrict__ dirs,
                                                 const int64_t* __restrict__ cand_off, int64_t n_prims,
                                                 const int64_t* __restrict__ ctl, Lat L, const Lat* __restrict__ lats,
                                                 const uint64_t* __restrict__ masks,
                                                 const int64_t* __restrict__ chunk_prim,
                                                 const int64_t* __restrict__ wave_off, Key* __restrict__ keys,
                                                 float* __restrict__ wts, uint32_t* __restrict__ prim, bool weights) {
  const int64_t n_chunks = ctl[CTL_N_CHUNKS];
  const int lane = lane_id();
  const int64_t w0 = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  const int64_t ws = int64_t(gridDim.x) * kWaves;
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  for (int64_t ch = w0; ch < n_chunks; ch += ws) {
    const uint64_t m = masks[ch];
    if (m == 0) continue;
    const int64_t ci = ch * 64 + lane;
    const int64_t p = wave_find_prim(cand_off, chunk_prim[ch], n_prims, ci);
    if (!((m >> lane) & 1)) continue;
    const int64_t pos = wave_off[ch] + __popcll(m & lt);
    const int32_t* r = rec + p * kRec;
    int64_t v[3];
    candidate_voxel(r, ci - cand_off[p], v);
    float wgt = 0.0f;
    const int Sb = lats ? lats[r[15]].Sb : L.Sb;
    if (weights) {
      if (KIND == 0) wgt = tri_area(r, v, Sb, dirs[p].w);
      else wgt = seg_length(r, v, Sb, dirs[p].w);
    }
    Key key = Key(morton3(uint32_t(v[0]), uint32_t(v[1]), uint32_t(v[2])));
    if (lats) key |= Key(uint64_t(uint32_t(r[15])) << kPatchShift);
    keys[pos] = key;
    wts[pos] = wgt;
    prim[pos] = uint32_t(p);
  }
}

// ---------------------------------------------------------------------------------------------
// scans: candidate offsets, survivor offsets
// ---------------------------------------------------------------------------------------------
struct ArrIn {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};
struct ArrOut {
  int64_t* o;
  __device__ void operator()(int64_t i, int64_t ex, int64_t) const { o[i] = ex; }
};
struct CandTotal {
  int64_t* cand_off;
  int64_t* ctl;
  int64_t* stats;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    cand_off[n] = total;
    stats[VX_STAT_CAND] = total;
    const bool over = total > cap;
    if (over) flag_or(stats, VX_FLAG_CAND_CAPACITY);
    const int64_t eff = over ? 0 : total;
    ctl[CTL_N_CAND] = eff;
    ctl[CTL_N_CHUNKS] = (eff + 63) / 64;
  }
};
struct PopIn {
  const uint64_t* m;
  __device__ int64_t operator()(int64_t i) const { return __popcll(m[i]); }
};
struct PairTotal {
  int64_t* wave_off;
  int64_t* ctl;
  int64_t* stats;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    wave_off[n] = total;
    stats[VX_STAT_PAIRS] = total;
    const bool over = total > cap;
    if (over) {
      flag_or(stats, VX_FLAG_PAIR_CAPACITY);
      ctl[CTL_N_CHUNKS] = 0;          // emit nothing
    }
    ctl[CTL_N_PAIRS] = over ? 0 : total;
  }
};

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

void launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
  int blocks = int((n + 255) / 256);
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(k_fill_i64, dim3(blocks), dim3(256), 0, s, p, n, v);
}

// up to four ranges cleared by one launch (ranges with n = 0 are skipped)
struct ZeroSet {
  int64_t* p[4];
  int64_t n[4];
};

__global__ void k_zero_multi(ZeroSet z) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    for (int64_t i = t; i < z.n[r]; i += stride) z.p[r][i] = 0;
}

static void launch_zero_multi(const ZeroSet& z, hipStream_t s) {
  int64_t m = 1;
  for (int r = 0; r < 4; ++r) m = z.n[r] > m ? z.n[r] : m;
  int blocks = int((m + 255) / 256);
  blocks = blocks > 1024 ? 1024 : blocks;
  hipLaunchKernelGGL(k_zero_multi, dim3(blocks), dim3(256), 0, s, z);
}

// ---------------------------------------------------------------------------------------------
// the whole voxelize pass
// ---------------------------------------------------------------------------------------------
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

void front_ws_carve(Carver& cv, int64_t n_prims, int64_t max_cand, int64_t max_pairs, bool key64, FrontWs* f) {
  const int64_t n_chunks = cdiv(max_cand, 64);
  FrontWs x;
  x.ctl = cv.take<int64_t>(CTL_SIZE);
  x.rec = cv.take<int32_t>(n_prims * kRec);
  x.dirs = cv.take<float4>(n_prims);
  x.cand_cnt = cv.take<int64_t>(n_prims);
  x.cand_off = cv.take<int64_t>(n_prims + 1);
  x.fstart = reinterpret_cast<uint8_t*>(x.cand_off);    // free until the candidate scan
  x.masks = cv.take<uint64_t>(n_chunks);
  x.chunk_prim = cv.take<int64_t>(n_chunks);
  x.wave_off = cv.take<int64_t>(n_chunks + 1);
  x.pa.keys = cv.take<uint8_t>(max_pairs * (key64 ? 8 : 4));
  x.pa.w = cv.take<float>(max_pairs);
  x.pa.prim = cv.take<uint32_t>(max_pairs);
  x.partial = cv.take<int64_t>(kGrid + 1);
  if (f) *f = x;
}

void prep_prims(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                int64_t n_fib, float radius, const FrontWs& w, int64_t* stats, hipStream_t s,
                const BatchLattice* batch, int64_t* zero_extra, int64_t zero_extra_n) {
  const Lat L = make_lat(g, kind, radius);
  // one launch clears the stats, the control block, the fiber-start bytes and the caller's range
  ZeroSet z{{stats, w.ctl, kind == 1 ? reinterpret_cast<int64_t*>(w.fstart) : nullptr, zero_extra},
            {VX_NSTAT, CTL_SIZE, kind == 1 ? (n_prims + 8) / 8 : 0, zero_extra ? zero_extra_n : 0}};
  launch_zero_multi(z, s);
  const int pgrid = int(n_prims / kBlock + 1 < kPrimGrid ? n_prims / kBlock + 1 : kPrimGrid);
  if (kind == 0) {
    VX_TIMED("prep_tri", s);
    hipLaunchKernelGGL(k_prep_tri, dim3(pgrid), dim3(kBlock), 0, s, data, n_prims, L, w.rec, w.dirs, w.cand_cnt,
                       w.rcnt, w.tb, w.box, stats);
  } else {
    {
      VX_TIMED("check_offsets", s);
      hipLaunchKernelGGL(k_check_offsets, dim3(int(n_fib / 256 + 1 < 256 ? n_fib / 256 + 1 : 256)), dim3(256), 0,
                         s, offsets, n_fib, n_prims, w.fstart, stats);
    }
    VX_TIMED("prep_fib", s);
    if (batch)
      hipLaunchKernelGGL(k_prep_fib_batch, dim3(pgrid), dim3(kBlock), 0, s, data, n_prims, w.fstart, batch->lats,
                         batch->pt_begin, batch->n_patches, w.rec, w.dirs, w.cand_cnt, w.box, stats);
    else
      hipLaunchKernelGGL(k_prep_fib, dim3(pgrid), dim3(kBlock), 0, s, data, n_prims, w.fstart, L, w.rec, w.dirs,
                         w.cand_cnt, w.box, stats);
  }
}

// prep -> candidate scan -> exact test -> pair scan -> emit: pairs in emission order in f.pa
void voxelize_front(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                    int64_t n_fib, float radius, int64_t max_cand, int64_t max_pairs, const FrontWs& w,
                    int64_t* stats, hipStream_t s, const BatchLattice* batch, bool weights) {
  const bool key64 = batch || g->log2_res > 10;
  const Lat L = make_lat(g, kind, radius);
  const Lat* lats = batch ? batch->lats : nullptr;
  prep_prims(kind, g, data, n_prims, offsets, n_fib, radius, w, stats, s, batch);
  {
    VX_TIMED("scan_cand", s);
    device_scan(ArrIn{w.cand_cnt}, ArrOut{w.cand_off}, CandTotal{w.cand_off, w.ctl, stats, max_cand}, nullptr,
                n_prims, w.partial, s);
  }
  {
    VX_TIMED("chunk_start", s);
    hipLaunchKernelGGL(k_chunk_start, dim3(kGrid), dim3(kBlock), 0, s, w.cand_off, n_prims, w.ctl, w.chunk_prim);
  }
  {
    VX_TIMED(kind == 0 ? "test_tri" : "test_fib", s);
    if (kind == 0)
      hipLaunchKernelGGL(k_test<0>, dim3(kGrid), dim3(kBlock), 0, s, w.rec, w.cand_off, n_prims,
                         w.ctl, L, lats, w.masks, w.chunk_prim);
    else
      hipLaunchKernelGGL(k_test<1>, dim3(kGrid), dim3(kBlock), 0, s, w.rec, w.cand_off, n_prims,
                         w.ctl, L, lats, w.masks, w.chunk_prim);
  }
  {
    VX_TIMED("scan_pairs", s);
    device_scan(PopIn{w.masks}, ArrOut{w.wave_off}, PairTotal{w.wave_off, w.ctl, stats, max_pairs},
                w.ctl + CTL_N_CHUNKS, 0, w.partial, s);
  }
  VX_TIMED(kind == 0 ? "emit_tri" : "emit_fib", s);
#define VX_EMIT(KD, K)                                                                                        \
  hipLaunchKernelGGL((k_emit<KD, K>), dim3(kGrid), dim3(kBlock), 0, s, w.rec, w.dirs, w.cand_off, \
                     n_prims, w.ctl, L, lats, w.masks, w.chunk_prim, w.wave_off, (K*)w.pa.keys, w.pa.w, w.pa.prim, \
                     weights)
  if (kind == 0) {
    if (key64) VX_EMIT(0, uint64_t); else VX_EMIT(0, uint32_t);
  } else {
    if (key64) VX_EMIT(1, uint64_t); else VX_EMIT(1, uint32_t);
  }
#undef VX_EMIT
}

}  // namespace vx
