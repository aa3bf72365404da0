// vx_internal.hpp -- device helpers shared by the libvx kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vx.h"

namespace vx {

constexpr int kBlock = 256;          // threads per block: 4 waves of 64
constexpr int kWaves = kBlock / 64;
constexpr int kGrid = 1024;          // persistent grid of the streaming kernels: 4 blocks per CU
constexpr int kPrimGrid = 4096;      // per-primitive streaming passes (prep, record count and emission):
                                     // enough blocks to fill every SIMD with the waves its registers allow
constexpr int kPatchShift = 33;      // batched keys: patch id above a 33-bit Morton code (R <= 2048)
constexpr int kTileBits = 4;         // leaf tiles of 16^3 voxels
constexpr int kUnitCand = 3072;      // the largest unit budget: candidates (so pairs) a unit keeps in LDS

// ---------------------------------------------------------------------------------------------
// Kernel timing (measurement only): events around every launch when enabled.
// ---------------------------------------------------------------------------------------------
void timing_begin(const char* name, hipStream_t s);
void timing_end(hipStream_t s);

struct TimedLaunch {
  hipStream_t s;
  TimedLaunch(const char* name, hipStream_t st) : s(st) { timing_begin(name, st); }
  ~TimedLaunch() { timing_end(s); }
};
#define VX_CAT2(a, b) a##b
#define VX_CAT(a, b) VX_CAT2(a, b)
#define VX_TIMED(name, stream) ::vx::TimedLaunch VX_CAT(vx_timed_, __LINE__)(name, stream)

// ---------------------------------------------------------------------------------------------
// Morton keys: x bit b -> key bit 3b, y -> 3b+1, z -> 3b+2.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;                       // 21 bits
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
__device__ __forceinline__ uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
// inverse of the Morton spread: every third bit of x, from bit 0
__device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x | (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x | (x >> 4)) & 0x100f00f00f00f00full;
  x = (x | (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x | (x >> 16)) & 0x1f00000000ffffull;
  x = (x | (x >> 32)) & 0x1fffffull;
  return uint32_t(x);
}

// ---------------------------------------------------------------------------------------------
// Wave and block scans (wave64).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T u = __shfl_up(v, off, 64);
    if (l >= off) v += u;
  }
  return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Exclusive scan over the block; returns this thread's exclusive prefix and the block total.
// `tmp` holds kWaves + 1 entries of LDS.  Contains __syncthreads().
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* tmp, T& total) {
  const int w = threadIdx.x >> 6;
  T inc = wave_inclusive_scan(v);
  if (lane_id() == 63) tmp[w] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    T x = tmp[i];
    if (i < w) base += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

// The same for a block of NW waves; `tmp` holds NW + 1 entries.
template <int NW, class T>
__device__ __forceinline__ T block_exclusive_scan_n(T v, T* tmp, T& total) {
  const int w = threadIdx.x >> 6;
  T inc = wave_inclusive_scan(v);
  if (lane_id() == 63) tmp[w] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    T x = tmp[i];
    if (i < w) base += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

// ---------------------------------------------------------------------------------------------
// Device-wide exclusive scan with a fixed grid (reduce, scan the partials, apply).
// The element count may live in device memory (n_ptr), so the launch needs no host sync.
// In:    int64_t operator()(int64_t i)            value of element i
// Out:   void operator()(int64_t i, int64_t excl, int64_t v)
// Total: void operator()(int64_t total, int64_t n)  called once, by one thread
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ int64_t scan_n(const int64_t* n_ptr, int64_t n_const) {
  return n_ptr ? *n_ptr : n_const;
}
constexpr int kScanRun = 4;   // consecutive elements per thread in a round of the apply pass
__device__ __forceinline__ int64_t scan_chunk(int64_t n) {
  int64_t c = (n + kGrid - 1) / kGrid;
  return (c + kBlock - 1) / kBlock * kBlock;
}

template <class In>
__global__ void __launch_bounds__(kBlock) k_scan_partial(In in, const int64_t* n_ptr, int64_t n_const,
                                                         int64_t* partial) {
  __shared__ int64_t red[kWaves];
  const int64_t n = scan_n(n_ptr, n_const);
  const int64_t chunk = scan_chunk(n);
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  int64_t acc = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) acc += in(i);
  acc = wave_sum(acc);
  if (lane_id() == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int i = 0; i < kWaves; ++i) t += red[i];
    partial[blockIdx.x] = t;
  }
}

// Every block adds up the partials of the blocks before it (kGrid int64 values, read from L2),
// so no separate pass scans the partials; block 0 also forms the total.
template <class In, class Out, class Total>
__global__ void __launch_bounds__(kBlock) k_scan_apply(In in, Out out, Total total, const int64_t* n_ptr,
                                                       int64_t n_const, const int64_t* partial) {
  __shared__ int64_t tmp[kWaves + 1];
  const int64_t n = scan_n(n_ptr, n_const);
  const int64_t chunk = scan_chunk(n);
  const int64_t b0 = int64_t(blockIdx.x) * chunk;
  const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  int64_t pre = 0, all = 0;
  for (int i = threadIdx.x; i < kGrid; i += kBlock) {
    const int64_t v = partial[i];
    if (i < int(blockIdx.x)) pre += v;
    all += v;
  }
  int64_t base;
  {
    int64_t t;
    (void)block_exclusive_scan(pre, tmp, base);
    if (blockIdx.x == 0) {
      (void)block_exclusive_scan(all, tmp, t);
      if (threadIdx.x == 0) total(t, n);
    }
  }
  if (b0 >= b1) return;
  // each thread takes kScanRun consecutive elements per round: one block scan per
  // kBlock * kScanRun elements
  for (int64_t t0 = b0; t0 < b1; t0 += int64_t(kBlock) * kScanRun) {
    const int64_t i0 = t0 + int64_t(threadIdx.x) * kScanRun;
    int64_t v[kScanRun], run = 0;
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      v[j] = i0 + j < b1 ? in(i0 + j) : 0;
      run += v[j];
    }
    int64_t tot;
    int64_t ex = base + block_exclusive_scan(run, tmp, tot);
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      if (i0 + j < b1) out(i0 + j, ex, v[j]);
      ex += v[j];
    }
    base += tot;
  }
}

template <class In, class Out, class Total>
inline void device_scan(In in, Out out, Total total, const int64_t* n_ptr, int64_t n_const, int64_t* partial,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_scan_partial<In>, dim3(kGrid), dim3(kBlock), 0, s, in, n_ptr, n_const, partial);
  hipLaunchKernelGGL((k_scan_apply<In, Out, Total>), dim3(kGrid), dim3(kBlock), 0, s, in, out, total, n_ptr,
                     n_const, partial);
}

// ---------------------------------------------------------------------------------------------
// The tuning of one call (vx_tuning resolved): tile edge, unit budget and the grid sizes of the
// persistent streaming kernels.  It changes the decomposition of the work, never a result.
// ---------------------------------------------------------------------------------------------
enum { kTuneUnit = 0, kTunePlan, kTuneCompact, kTuneLod, kTuneCluster, kTuneCount };
static_assert(kTuneCount == VX_TUNE_COUNT, "one grid per tuned kernel");
struct Tuning {
  int tile_bits;      // 2..4
  int unit_budget;    // 1024, 1536, 2048 or 3072 candidates
  int grids[kTuneCount];
};
// defaults for NULL or zero fields (kind 0 triangles, 1 fibers); false on an invalid value
bool resolve_tuning(const vx_tuning* t, int kind, Tuning* out);

// ---------------------------------------------------------------------------------------------
// Workspace carving (256-byte aligned sub-buffers).
// ---------------------------------------------------------------------------------------------
struct Carver {
  uintptr_t base;
  size_t off = 0;
  explicit Carver(void* p) : base(reinterpret_cast<uintptr_t>(p)) {}
  template <class T>
  T* take(int64_t n) {
    size_t bytes = size_t(n > 0 ? n : 1) * sizeof(T);
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += bytes;
    return p;
  }
};

// internal control block (device): effective counts that later kernels iterate over
enum { CTL_N_CAND = 0, CTL_N_CHUNKS, CTL_N_PAIRS, CTL_N_VOX, CTL_N_REC, CTL_N_TILES, CTL_N_UNITS, CTL_SIZE = 8 };

// ---------------------------------------------------------------------------------------------
// per-voxel sums: count, w and S = sum w M, accumulated pair by pair in primitive order
// ---------------------------------------------------------------------------------------------
struct Moment {
  float W, xx, yy, zz, xy, xz, yz;
};
// t: unit normal (KIND 0, M = n n^T) or unit tangent (KIND 1, M = I - t t^T)
template <int KIND>
__device__ __forceinline__ void accum_pair(Moment& m, float wj, float4 t) {
  const float ax = wj * t.x, ay = wj * t.y;
  m.W += wj;
  if (KIND == 0) {
    m.xx = fmaf(ax, t.x, m.xx);
    m.yy = fmaf(ay, t.y, m.yy);
    m.zz = fmaf(wj * t.z, t.z, m.zz);
    m.xy = fmaf(ax, t.y, m.xy);
    m.xz = fmaf(ax, t.z, m.xz);
    m.yz = fmaf(ay, t.z, m.yz);
  } else {
    m.xx += wj - ax * t.x;
    m.yy += wj - ay * t.y;
    m.zz += wj - wj * t.z * t.z;
    m.xy = fmaf(-ax, t.y, m.xy);
    m.xz = fmaf(-ax, t.z, m.xz);
    m.yz = fmaf(-ay, t.z, m.yz);
  }
}

// ---------------------------------------------------------------------------------------------
// launchers implemented in the .hip files
// ---------------------------------------------------------------------------------------------
struct PairBufs {
  void* keys;       // uint32 or uint64
  float* w;
  uint32_t* prim;
};

void launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);

// sort pairs by key (stable LSD radix); returns the buffer index (0 = a, 1 = b) holding the result
constexpr int kRadixBuckets = 512;          // digit values of the record sort (hist is kRadixBuckets x kGrid)
int radix_sort_pairs(bool key64, int key_bits, PairBufs a, PairBufs b, const int64_t* n_dev, int64_t cap,
                     int32_t* hist, int64_t* partial, hipStream_t s);

// head flags of sorted keys (SHIFT 0: the key, 3: the parent key) and segment starts
template <class Key, bool BATCH>
__device__ __forceinline__ Key parent_key(Key k) {
  if (!BATCH) return k >> 3;
  const Key lowmask = (Key(1) << kPatchShift) - 1;
  return (k & ~lowmask) | ((k & lowmask) >> 3);
}
template <class Key, int SHIFT, bool BATCH = false>
struct HeadIn {
  const Key* k;
  __device__ int64_t operator()(int64_t i) const {
    if (SHIFT == 0) return i == 0 || k[i] != k[i - 1];
    return i == 0 || parent_key<Key, BATCH>(k[i]) != parent_key<Key, BATCH>(k[i - 1]);
  }
};
struct HeadOut {
  int64_t* start;
  __device__ void operator()(int64_t i, int64_t ex, int64_t v) const {
    if (v) start[ex] = i;
  }
};

// SGGX-H lobes (sggxh.hip; arguments checked by the caller)
vx_status sggxh_run(const vx_grid* g, const vx_voxels* leaf, const vx_voxels* out, const int64_t* n_levels,
                    int levels, int K, int N, const vx_lobes* lobes, int64_t* stats, hipStream_t s);

// sub-voxel occupancy (occupancy.hip; arguments checked by the caller)
size_t occupancy_ws_bytes(int64_t n_prims, int64_t max_cand, int64_t max_pairs, bool key64);
vx_status occupancy_run(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                        int64_t n_fib, float radius, const vx_voxels* leaf, const vx_voxels* out,
                        const int64_t* n_levels, int levels, int64_t max_cand, int64_t max_pairs,
                        const vx_occupancy* occ, void* ws, int64_t* stats, hipStream_t s);

// the sampling voxelizer (kind 0 triangles, 1 fibers; arguments checked by the caller)
size_t sample_ws_bytes(int kind, int64_t n_prims, int64_t max_samples, int64_t max_vox, int log2R, int sub);
vx_status sample_voxelize(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                          int64_t n_fib, const vx_sampling* sp, int64_t max_samples, void* ws, const vx_voxels* out,
                          int64_t* stats, hipStream_t s);

// one LoD level: parent reduce of `in` (n_in on the device) into `out`; n_out receives the
// new count clamped to out.cap, and flags the capacity bit when it had to be clamped; pstart
// receives every parent's first child
void lod_level(bool key64, const vx_voxels& in, const int64_t* n_in, const vx_voxels& out, int64_t* n_out,
               int64_t* flags, int64_t* pstart, int64_t* partial, int grid, hipStream_t s, bool batch = false);
void lod_init(const int64_t* src, int64_t cap, int64_t* n_levels, int64_t count, hipStream_t s);
// levels lv[1 .. count] from lv[0] in one single-block launch (small levels, no lobes):
// n[i] the device count of lv[i]
constexpr int64_t kTailMax = 2048;
void lod_tail(bool key64, bool batch, const vx_voxels* lv, int64_t* const* n, int count, int64_t* flags,
              hipStream_t s);

// lobe clustering of one level (cluster.hip): parents [0, *n_par) with children
// [pstart[p], pstart[p+1]) whose lobes are cw[k * cap_c + c], cS[(j * Kc + k) * cap_c + c];
// narrow_first: many parents are expected to gather at most 8 lobes (a launch choice only)
void cluster_level(const int64_t* pstart, const int64_t* n_par, const float* cw, const float* cS, const uint8_t* cnl,
                   int Kc, int64_t cap_c, int K, int iters, const vx_lobes& out, int grid, hipStream_t s,
                   bool narrow_first = false);

// the front half of voxelize (prims.hip): pairs in emission order (by primitive, then candidate)
struct FrontWs {
  int64_t* ctl;
  uint8_t* fstart;     // [n_prims + 8] fibers: point i starts a fiber (space shared with a later stage)
  int32_t* rec;
  float4* dirs;
  int64_t* cand_cnt;
  int64_t* cand_off;
  uint64_t* masks;
  int64_t* chunk_prim;
  int64_t* wave_off;
  PairBufs pa;
  int64_t* partial;
  int64_t* rcnt = nullptr;   // triangles, tiled path: tiles of 2^tb voxels each candidate box overlaps
  int tb = 0;
  ulonglong2* box = nullptr; // tiled path: each primitive's candidate box, packed (pack_box)
};

// A primitive's candidate box for the passes that need only the box: first (x) and last (y)
// voxel per axis, 21 bits each (grids up to 2^20 voxels per axis), from record words 9..14.  An
// empty box packs its first voxel twice (it has no records, so no pass reads it).
__host__ __device__ inline ulonglong2 pack_box(const int32_t* r) {
  uint64_t lo = 0, hi = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int32_t l = r[9 + a], h = r[12 + a] > 0 ? r[9 + a] + r[12 + a] - 1 : r[9 + a];
    lo |= uint64_t(uint32_t(l) & 0x1fffffu) << (21 * a);
    hi |= uint64_t(uint32_t(h) & 0x1fffffu) << (21 * a);
  }
  return make_ulonglong2(lo, hi);
}
__host__ __device__ inline void unpack_box(const ulonglong2& b, int32_t lo[3], int32_t hi[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = int32_t((b.x >> (21 * a)) & 0x1fffffu);
    hi[a] = int32_t((b.y >> (21 * a)) & 0x1fffffu);
  }
}
void front_ws_carve(Carver& cv, int64_t n_prims, int64_t max_cand, int64_t max_pairs, bool key64, FrontWs* f);
struct Lat;
// batched patches: per-patch lattices and point ranges (device), keys carry the patch id above
// bit kPatchShift
struct BatchLattice {
  const Lat* lats;
  const int64_t* pt_begin;   // [n_patches + 1]
  int n_patches;
};
// weights = false: the pairs' weights are left 0 (for callers that need only keys and primitives)
void voxelize_front(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                    int64_t n_fib, float radius, int64_t max_cand, int64_t max_pairs, const FrontWs& w,
                    int64_t* stats, hipStream_t s, const BatchLattice* batch, bool weights = true);
// its first step: clear stats and control, snap the primitives, write records and candidate counts
void prep_prims(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                int64_t n_fib, float radius, const FrontWs& w, int64_t* stats, hipStream_t s,
                const BatchLattice* batch, int64_t* zero_extra = nullptr, int64_t zero_extra_n = 0);

// the differentiable two-lobe fit (fit.hip)
size_t fit_ws_bytes(int64_t n_pts, int64_t max_cand, int64_t max_pairs, const int64_t* caps, int hi, int log2R);
vx_status fit_forward_run(const vx_grid* g, const vx_voxels* levels, const int64_t* n_levels, int lo, int hi,
                          const float* const* params, const int64_t* rows, const void* const* bound, const float* dirs,
                          int ndir, float* loss, int64_t* stats, void* ws, const int64_t* caps, hipStream_t s);
vx_status fit_backward_run(const vx_grid* g, const float* pts, int64_t n_pts, const int64_t* offsets, int64_t n_fib,
                           float radius, int64_t max_cand, int64_t max_pairs, const vx_voxels* levels,
                           const int64_t* n_levels, int lo, int hi, const float* const* params, const int64_t* rows,
                           const void* const* bound, const float* dirs, int ndir, const float* dloss,
                           float* const* dparams, float* dpts, int64_t* stats, void* ws, const int64_t* caps,
                           hipStream_t s);

// the voxelize pass by tiles (tiles.hip); tb = tile bits per axis
size_t tile_ws_bytes(int64_t n_prims, int64_t max_rec, int64_t max_units, int64_t max_vox, bool key64);
// leaf eigen-fit + compact SGGX code, and its decoding (compact.hip)
void sggx_compact_run(const float* w, const float* S, const int64_t* n, int64_t cap, double eps, float* lam,
                      float* vec, uint8_t* code, hipStream_t s);
void sggx_decode_run(const uint8_t* code, const int64_t* n, int64_t cap, float* S, hipStream_t s);

// tb: tile bits of this call (the tuning's, at most log2 of the grid)
vx_status tile_voxelize(int kind, const vx_grid* g, const float* data, int64_t n_prims, const int64_t* offsets,
                        int64_t n_fib, float radius, int64_t max_rec, int64_t max_units, void* ws,
                        const vx_voxels* out, int64_t* stats, hipStream_t s, const BatchLattice* batch, int tb,
                        const Tuning& tu);

}  // namespace vx
