// sortreduce.hip -- ordering keyed records and the parent levels of the pyramid.
//   radix sort  : Sec. 3.3 orders the samples by voxel id so that each voxel's samples are
//                 contiguous; here a stable LSD radix sort (9-bit digits) with wave-level
//                 ranking in LDS, fixed grid, no atomics on global memory -- applied to the
//                 primitive-tile records, which group the work by tile.
//   LoD level   : Sec. 4.3 aggregates 2x2x2 children into a coarser voxel; children of a parent
//                 are contiguous in Morton order, so this is a segmented sum over key >> 3.
#include "vx_internal.hpp"

namespace vx {

__device__ __forceinline__ void flag_or_s(int64_t* p, int64_t bit) {
  atomicOr(reinterpret_cast<unsigned long long*>(p), (unsigned long long)bit);
}

// ---------------------------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------------------------
constexpr int kDigitBits = 9;                 // 18-bit tile keys (1024^3 grids) sort in two passes
constexpr int kBuckets = 1 << kDigitBits;
static_assert(kBuckets == kRadixBuckets, "histogram workspace");
// blocks of the sort kernels: four per CU, all resident at once with the scatter's LDS (the digit
// histograms, kBuckets per block, and their scan stay small)
constexpr int kSortGrid = 1024;
static_assert(kSortGrid <= kGrid, "histogram workspace");

__device__ __forceinline__ int64_t sort_chunk(int64_t n) {
  const int64_t c = (n + kSortGrid - 1) / kSortGrid;
  return (c + kBlock - 1) / kBlock * kBlock;
}

template <class Key>
__global__ void __launch_bounds__(kBlock) k_radix_hist(const Key* __restrict__ keys, const int64_t* n_ptr, int shift,
                                                       int32_t* __restrict__ hist) {
  __shared__ int32_t h[kBuckets];
  for (int d = threadIdx.x; d < kBuckets; d += kBlock) h[d] = 0;
  __syncthreads();
  const int64_t n = *n_ptr;
  const int64_t chunk = sort_chunk(n);
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  // Four rows of 256 keys per step, loaded together.  Lanes of a wave holding the same digit find
  // each other by ballots over its bits and the first of them adds the group's count: one LDS
  // atomic per distinct digit and wave (runs of equal digits are common in the record lists).
  constexpr int kRows = 4;
  const int lane = lane_id();
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  for (int64_t t0 = b0; t0 < b1; t0 += int64_t(kRows) * kBlock) {
    int dg[kRows];
    bool ok[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int64_t i = t0 + j * kBlock + threadIdx.x;
      ok[j] = i < b1;
      dg[j] = ok[j] ? int((keys[i] >> shift) & (kBuckets - 1)) : 0;
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      uint64_t peers = __ballot(ok[j]);
#pragma unroll
      for (int b = 0; b < kDigitBits; ++b) {
        const uint64_t m = __ballot((dg[j] >> b) & 1);
        peers &= ((dg[j] >> b) & 1) ? m : ~m;
      }
      if (ok[j] && (peers & lt) == 0) atomicAdd(&h[dg[j]], int32_t(__popcll(peers)));
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kBuckets; d += kBlock) hist[int64_t(d) * kSortGrid + blockIdx.x] = h[d];
}

struct I32In {
  const int32_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};
struct I32Out {
  int32_t* o;
  __device__ void operator()(int64_t i, int64_t ex, int64_t) const { o[i] = int32_t(ex); }
};
struct NoTotal {
  __device__ void operator()(int64_t, int64_t) const {}
};

// One pass of the stable scatter.  A block takes its chunk in tiles of kTileN elements; a tile
// is ranked by digit (wave ballots within each row of 256, counts per row and wave, one scan over
// the digits), placed digit by digit in LDS, and written out in that order, so each digit's run
// of the tile lands contiguously (coalesced) at the digit's next position.  Order within a digit
// is row, wave, lane = input order: the sort is stable.  w may be null (not carried).
constexpr int kTileE = 4;                      // rows of 256 elements per tile (38 KB of LDS per block)
constexpr int kTileN = kBlock * kTileE;
static_assert(kBuckets == 2 * kBlock, "the digit scan takes two digits per thread");
static_assert(kTileN <= 32767, "16-bit tile positions");

template <class Key>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const Key* __restrict__ kin, const float* __restrict__ win,
                                                          const uint32_t* __restrict__ pin, Key* __restrict__ kout,
                                                          float* __restrict__ wout, uint32_t* __restrict__ pout,
                                                          const int64_t* n_ptr, int shift,
                                                          const int32_t* __restrict__ hist_off) {
  __shared__ int32_t run[kBuckets];                    // next output position of each digit
  __shared__ int16_t cnt[kTileE][kWaves][kBuckets];    // per row and wave; then their prefixes (< kTileN)
  __shared__ int32_t toff[kBuckets];                   // each digit's first slot in the sorted tile
  __shared__ int32_t ttot[kBuckets];
  __shared__ Key sk[kTileN];
  __shared__ float sw[kTileN];
  __shared__ uint32_t sp[kTileN];
  __shared__ int32_t stmp[kWaves + 1];
  const int t = threadIdx.x, w = t >> 6, lane = lane_id();
  const bool has_w = win != nullptr;
  for (int d = t; d < kBuckets; d += kBlock) run[d] = hist_off[int64_t(d) * kSortGrid + blockIdx.x];
  const int64_t n = *n_ptr;
  const int64_t chunk = sort_chunk(n);
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  for (int64_t t0 = b0; t0 < b1; t0 += kTileN) {
    const int ntile = int(b1 - t0 < kTileN ? b1 - t0 : kTileN);
    for (int q = t; q < kTileE * kWaves * kBuckets; q += kBlock) (&cnt[0][0][0])[q] = 0;
    Key k[kTileE];
    float wv[kTileE];
    uint32_t pv[kTileE];
    int dg[kTileE], rk[kTileE];
#pragma unroll
    for (int j = 0; j < kTileE; ++j) {
      const int64_t i = t0 + j * kBlock + t;
      const bool valid = i < b1;
      k[j] = valid ? kin[i] : Key(0);
      wv[j] = valid && has_w ? win[i] : 0.f;
      pv[j] = valid ? pin[i] : 0u;
      dg[j] = int((k[j] >> shift) & (kBuckets - 1));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTileE; ++j) {
      const bool valid = t0 + j * kBlock + t < b1;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kDigitBits; ++b) {
        const uint64_t m = __ballot((dg[j] >> b) & 1);
        peers &= ((dg[j] >> b) & 1) ? m : ~m;
      }
      rk[j] = valid ? __popcll(peers & lt) : -1;
      if (valid && rk[j] == 0) cnt[j][w][dg[j]] = int16_t(__popcll(peers));
    }
    __syncthreads();
    // per digit: prefixes over (row, wave) in input order, and the tile's count
    int32_t dsum = 0;
    for (int d = t; d < kBuckets; d += kBlock) {
      int32_t acc = 0;
#pragma unroll
      for (int j = 0; j < kTileE; ++j)
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
          const int32_t c = cnt[j][ww][d];
          cnt[j][ww][d] = int16_t(acc);
          acc += c;
        }
      ttot[d] = acc;
    }
    __syncthreads();
    // tile offsets of the digits: thread t scans digits 2t and 2t + 1
    {
      const int32_t a = ttot[2 * t], b = ttot[2 * t + 1];
      int32_t total;
      const int32_t ex = block_exclusive_scan<int32_t>(a + b, stmp, total);
      toff[2 * t] = ex;
      toff[2 * t + 1] = ex + a;
      (void)dsum;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kTileE; ++j) {
      if (rk[j] >= 0) {
        const int slot = toff[dg[j]] + cnt[j][w][dg[j]] + rk[j];
        sk[slot] = k[j];
        sw[slot] = wv[j];
        sp[slot] = pv[j];
      }
    }
    __syncthreads();
    for (int q = t; q < ntile; q += kBlock) {
      const Key kk = sk[q];
      const int d = int((kk >> shift) & (kBuckets - 1));
      const int32_t pos = run[d] + (q - toff[d]);
      kout[pos] = kk;
      if (has_w) wout[pos] = sw[q];
      pout[pos] = sp[q];
    }
    __syncthreads();
    for (int d = t; d < kBuckets; d += kBlock) run[d] += ttot[d];
    __syncthreads();
  }
}

int radix_sort_pairs(bool key64, int key_bits, PairBufs a, PairBufs b, const int64_t* n_dev, int64_t cap,
                     int32_t* hist, int64_t* partial, hipStream_t s) {
  (void)cap;
  const int passes = (key_bits + kDigitBits - 1) / kDigitBits;
  PairBufs src = a, dst = b;
  for (int p = 0; p < passes; ++p) {
    const int shift = kDigitBits * p;
    {
      VX_TIMED("radix_hist", s);
      if (key64)
        hipLaunchKernelGGL(k_radix_hist<uint64_t>, dim3(kSortGrid), dim3(kBlock), 0, s, (const uint64_t*)src.keys, n_dev,
                           shift, hist);
      else
        hipLaunchKernelGGL(k_radix_hist<uint32_t>, dim3(kSortGrid), dim3(kBlock), 0, s, (const uint32_t*)src.keys, n_dev,
                           shift, hist);
    }
    {
      VX_TIMED("radix_scan", s);
      device_scan(I32In{hist}, I32Out{hist}, NoTotal{}, nullptr, int64_t(kBuckets) * kSortGrid, partial, s);
    }
    {
      VX_TIMED("radix_scatter", s);
      if (key64)
        hipLaunchKernelGGL(k_radix_scatter<uint64_t>, dim3(kSortGrid), dim3(kBlock), 0, s, (const uint64_t*)src.keys,
                           src.w, src.prim, (uint64_t*)dst.keys, dst.w, dst.prim, n_dev, shift, hist);
      else
        hipLaunchKernelGGL(k_radix_scatter<uint32_t>, dim3(kSortGrid), dim3(kBlock), 0, s, (const uint32_t*)src.keys,
                           src.w, src.prim, (uint32_t*)dst.keys, dst.w, dst.prim, n_dev, shift, hist);
    }
    PairBufs tmp = src;
    src = dst;
    dst = tmp;
  }
  return passes & 1;
}

// ---------------------------------------------------------------------------------------------
// LoD: parent = sum of its (<= 8, contiguous) children
// ---------------------------------------------------------------------------------------------
// sum of the children [a, b) of one parent (in Morton order, so the sums are sequential and fixed)
template <class Key, bool BATCH>
__device__ __forceinline__ void lod_parent(const vx_voxels& in, const Key* ikeys, int64_t a, int64_t b,
                                           const vx_voxels& out, int64_t p) {
  const int64_t ci = in.cap, co = out.cap;
  uint32_t c = 0, mask = 0;
  float W = 0.f, S[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int64_t j = a; j < b; ++j) {
    c += in.count[j];
    mask |= 1u << uint32_t(ikeys[j] & 7);
    W += in.w[j];
#pragma unroll
    for (int k = 0; k < 6; ++k) S[k] += in.S[k * ci + j];
  }
  reinterpret_cast<Key*>(out.keys)[p] = parent_key<Key, BATCH>(ikeys[a]);
  out.count[p] = c;
  out.mask[p] = uint8_t(mask);
  out.w[p] = W;
#pragma unroll
  for (int k = 0; k < 6; ++k) out.S[k * co + p] = S[k];
}

struct LodTotal {
  int64_t* start;
  int64_t* n_out;     // clamped count of the new level
  int64_t* flags;
  int64_t cap;
  __device__ void operator()(int64_t total, int64_t n) const {
    const bool over = total > cap;
    if (over) flag_or_s(flags, VX_FLAG_VOXEL_CAPACITY);
    const int64_t eff = over ? cap : total;
    start[eff] = n;      // only read up to the clamped count
    *n_out = eff;
  }
};


template <class Key, bool BATCH>
__global__ void __launch_bounds__(kBlock) k_lod_reduce(vx_voxels in, const int64_t* __restrict__ start,
                                                       const int64_t* __restrict__ n_ptr, vx_voxels out) {
  const int64_t n = *n_ptr;
  const Key* ikeys = reinterpret_cast<const Key*>(in.keys);
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < n; p += int64_t(gridDim.x) * kBlock)
    lod_parent<Key, BATCH>(in, ikeys, start[p], start[p + 1], out, p);
}

constexpr int kLodBlock = 1024;
constexpr int kLodWaves = kLodBlock / 64;

// The small top levels in one launch (one block): level after level, heads of the parent key
// in chunks, ranks by block scan, children summed as above.  The levels built here stay in LDS
// between levels (in place: every parent's sums are taken into registers before any parent is
// written back), so a level never reads global memory written by the one before.  in_cap of the
// first level <= kTailMax.
constexpr int kTailLevels = 21;
constexpr int kTailChunks = int(kTailMax / kLodBlock);
static_assert(kTailMax % kLodBlock == 0, "whole chunks");
struct TailLevels {
  vx_voxels lv[kTailLevels];    // lv[0] = the input of the first level built here
  int64_t* n[kTailLevels];      // device counts, n[0] the input's
  int count;                    // levels to build: lv[1 .. count]
};

template <class Key>
constexpr size_t tail_lds_bytes() {
  return size_t(kTailMax) * (sizeof(Key) + 4 + 4 + 24);
}

template <class Key, bool BATCH>
__global__ void __launch_bounds__(kLodBlock) k_lod_tail(TailLevels T, int64_t* __restrict__ flags) {
  extern __shared__ double tail_dyn[];
  __shared__ int64_t tmp[kLodWaves + 1];
  Key* lk = reinterpret_cast<Key*>(tail_dyn);
  uint32_t* lc = reinterpret_cast<uint32_t*>(lk + kTailMax);
  float* lw = reinterpret_cast<float*>(lc + kTailMax);
  float* lS = lw + kTailMax;                                 // [6][kTailMax]
  const int tid = threadIdx.x;
  int64_t n = *T.n[0];
  n = n < kTailMax ? n : kTailMax;
  {
    const vx_voxels& in = T.lv[0];
    const Key* k = reinterpret_cast<const Key*>(in.keys);
    for (int64_t i = tid; i < n; i += kLodBlock) {
      lk[i] = k[i];
      lc[i] = in.count[i];
      lw[i] = in.w[i];
#pragma unroll
      for (int c = 0; c < 6; ++c) lS[c * kTailMax + i] = in.S[c * in.cap + i];
    }
  }
  __syncthreads();
  for (int L = 1; L <= T.count; ++L) {
    const vx_voxels& out = T.lv[L];
    // read phase: every parent's sums into registers (chunk q of the children, one per thread)
    int64_t pp[kTailChunks];
    Key pk[kTailChunks];
    uint32_t pc[kTailChunks], pm[kTailChunks];
    float pw[kTailChunks], pS[kTailChunks][6];
    int64_t base = 0;
#pragma unroll
    for (int q = 0; q < kTailChunks; ++q) {
      pp[q] = -1;
      if (int64_t(q) * kLodBlock >= n) continue;     // uniform: no children in this chunk
      const int64_t i = int64_t(q) * kLodBlock + tid;
      const bool head = i < n && (i == 0 || parent_key<Key, BATCH>(lk[i]) != parent_key<Key, BATCH>(lk[i - 1]));
      int64_t tot;
      const int64_t ex = block_exclusive_scan_n<kLodWaves>(int64_t(head), tmp, tot);
      pp[q] = head ? base + ex : -1;
      pk[q] = 0;
      pc[q] = 0;
      pm[q] = 0;
      pw[q] = 0.f;
#pragma unroll
      for (int c = 0; c < 6; ++c) pS[q][c] = 0.f;
      if (head) {
        const Key key = parent_key<Key, BATCH>(lk[i]);
        pk[q] = key;
        for (int64_t j = i; j < n && j < i + 8 && parent_key<Key, BATCH>(lk[j]) == key; ++j) {
          pc[q] += lc[j];
          pm[q] |= 1u << uint32_t(lk[j] & 7);
          pw[q] += lw[j];
#pragma unroll
          for (int c = 0; c < 6; ++c) pS[q][c] += lS[c * kTailMax + j];
        }
      }
      base += tot;
    }
    __syncthreads();                                 // all children read before any is overwritten
    const int64_t cap = out.cap;
    Key* ok = reinterpret_cast<Key*>(out.keys);
#pragma unroll
    for (int q = 0; q < kTailChunks; ++q) {
      const int64_t p = pp[q];
      if (p >= 0 && p < cap) {
        lk[p] = pk[q];
        lc[p] = pc[q];
        lw[p] = pw[q];
#pragma unroll
        for (int c = 0; c < 6; ++c) lS[c * kTailMax + p] = pS[q][c];
        ok[p] = pk[q];
        out.count[p] = pc[q];
        out.mask[p] = uint8_t(pm[q]);
        out.w[p] = pw[q];
#pragma unroll
        for (int c = 0; c < 6; ++c) out.S[c * cap + p] = pS[q][c];
      }
    }
    const bool over = base > cap;
    if (tid == 0) {
      if (over) flag_or_s(flags, VX_FLAG_VOXEL_CAPACITY);
      *T.n[L] = over ? cap : base;
    }
    n = over ? cap : base;
    __syncthreads();
  }
}

// level counts of a pyramid build: entry 0 is the leaf count clamped to [0, cap], the other
// count - 1 entries (levels and the flag word) start at zero
__global__ void k_lod_init(const int64_t* src, int64_t cap, int64_t* n_levels, int64_t count) {
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
    if (i == 0) {
      const int64_t v = *src;
      n_levels[0] = v < 0 ? 0 : (v > cap ? cap : v);
    } else {
      n_levels[i] = 0;
    }
  }
}

void lod_init(const int64_t* src, int64_t cap, int64_t* n_levels, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_lod_init, dim3(1), dim3(64), 0, s, src, cap, n_levels, count);
}

void lod_level(bool key64, const vx_voxels& in, const int64_t* n_in, const vx_voxels& out, int64_t* n_out,
               int64_t* flags, int64_t* pstart, int64_t* partial, int grid_blocks, hipStream_t s, bool batch) {
  {
    VX_TIMED("lod_heads", s);
    if (batch)
      device_scan(HeadIn<uint64_t, 3, true>{(const uint64_t*)in.keys}, HeadOut{pstart},
                  LodTotal{pstart, n_out, flags, out.cap}, n_in, 0, partial, s);
    else if (key64)
      device_scan(HeadIn<uint64_t, 3>{(const uint64_t*)in.keys}, HeadOut{pstart},
                  LodTotal{pstart, n_out, flags, out.cap}, n_in, 0, partial, s);
    else
      device_scan(HeadIn<uint32_t, 3>{(const uint32_t*)in.keys}, HeadOut{pstart},
                  LodTotal{pstart, n_out, flags, out.cap}, n_in, 0, partial, s);
  }
  VX_TIMED("lod_reduce", s);
  const dim3 grid(grid_blocks);
  if (batch)
    hipLaunchKernelGGL((k_lod_reduce<uint64_t, true>), grid, dim3(kBlock), 0, s, in, pstart, n_out, out);
  else if (key64)
    hipLaunchKernelGGL((k_lod_reduce<uint64_t, false>), grid, dim3(kBlock), 0, s, in, pstart, n_out, out);
  else
    hipLaunchKernelGGL((k_lod_reduce<uint32_t, false>), grid, dim3(kBlock), 0, s, in, pstart, n_out, out);
}

void lod_tail(bool key64, bool batch, const vx_voxels* lv, int64_t* const* n, int count, int64_t* flags,
              hipStream_t s) {
  if (count < 1) return;
  VX_TIMED("lod_tail", s);
  TailLevels T;
  for (int i = 0; i <= count && i < kTailLevels; ++i) {
    T.lv[i] = lv[i];
    T.n[i] = n[i];
  }
  T.count = count < kTailLevels ? count : kTailLevels - 1;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_lod_tail<uint64_t, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(tail_lds_bytes<uint64_t>()));
    (void)hipFuncSetAttribute((const void*)k_lod_tail<uint64_t, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(tail_lds_bytes<uint64_t>()));
    (void)hipFuncSetAttribute((const void*)k_lod_tail<uint32_t, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              int(tail_lds_bytes<uint32_t>()));
    attr = true;
  }
  if (batch)
    hipLaunchKernelGGL((k_lod_tail<uint64_t, true>), dim3(1), dim3(kLodBlock), tail_lds_bytes<uint64_t>(), s, T, flags);
  else if (key64)
    hipLaunchKernelGGL((k_lod_tail<uint64_t, false>), dim3(1), dim3(kLodBlock), tail_lds_bytes<uint64_t>(), s, T,
                       flags);
  else
    hipLaunchKernelGGL((k_lod_tail<uint32_t, false>), dim3(1), dim3(kLodBlock), tail_lds_bytes<uint32_t>(), s, T,
                       flags);
}

}  // namespace vx
