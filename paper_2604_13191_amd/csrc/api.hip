// api.hip -- the C ABI of libvx.so (declared in include/vx.h): argument checks, workspace
// sizing, orchestration of the kernels on the caller's stream, and kernel timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "geom.hpp"
#include "vx_internal.hpp"

namespace vx {

// ---------------------------------------------------------------------------------------------
// timing: one event pair per launch while enabled, resolved in vx_timing_collect()
// ---------------------------------------------------------------------------------------------
namespace {
struct Pending {
  std::string name;
  hipEvent_t a, b;
};
struct Acc {
  std::string name;
  double ms = 0;
  int64_t n = 0;
};
std::mutex g_mu;
std::atomic<bool> g_on{false};   // read without the lock: launches pay nothing while timing is off
std::string g_filter;            // time only launches of this name (empty: all)
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::vector<Acc> g_acc;
thread_local std::vector<size_t> g_open;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  (void)hipEventCreate(&e);
  return e;
}
}  // namespace

void timing_begin(const char* name, hipStream_t s) {
  if (!g_on.load(std::memory_order_acquire)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_filter.empty() && g_filter != name) {
    g_open.push_back(SIZE_MAX);
    return;
  }
  Pending p{name, get_event(), get_event()};
  (void)hipEventRecord(p.a, s);
  g_pending.push_back(p);
  g_open.push_back(g_pending.size() - 1);
}

void timing_end(hipStream_t s) {
  if (g_open.empty()) return;                  // this thread opened nothing (timing was off)
  std::lock_guard<std::mutex> lk(g_mu);
  size_t i = g_open.back();
  g_open.pop_back();
  if (i == SIZE_MAX) return;
  (void)hipEventRecord(g_pending[i].b, s);
}

bool resolve_tuning(const vx_tuning* t, int kind, Tuning* out) {
  Tuning u;
  u.tile_bits = kTileBits;
  u.unit_budget = kind == 0 ? 1536 : kUnitCand;
  // persistent grids well above the resident blocks (768 to 1024 per launch), so that no tail of
  // late blocks runs alone; the parent reduce walks children per thread and likes fewer blocks
  const int defaults[kTuneCount] = {16384, 8192, 16384, 512, 8192};
  for (int i = 0; i < kTuneCount; ++i) u.grids[i] = defaults[i];
  if (t) {
    if (t->tile_bits != 0) {
      if (t->tile_bits < 2 || t->tile_bits > kTileBits) return false;
      u.tile_bits = t->tile_bits;
    }
    if (t->unit_budget != 0) {
      const int b = t->unit_budget;
      if (b != 1024 && b != 1536 && b != 2048 && b != 3072) return false;
      u.unit_budget = b;
    }
    for (int i = 0; i < kTuneCount; ++i)
      if (t->grids[i] != 0) {
        if (t->grids[i] < 64 || t->grids[i] > 16384) return false;
        u.grids[i] = t->grids[i];
      }
  }
  *out = u;
  return true;
}

// batched patches: device lattice table and point ranges from the caller's device patch array
__global__ void k_batch_setup(const vx_patch* __restrict__ patches, int n, Lat* __restrict__ lats,
                              int64_t* __restrict__ pt_begin) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    lats[p] = make_lat(&patches[p].grid, 1, patches[p].radius);
    pt_begin[p] = patches[p].pt_begin;
    if (p == n - 1) pt_begin[n] = patches[p].pt_end;
  }
}

// start of every patch's voxels in a level: lower bound of (p << 33) in the sorted keys
__global__ void k_patch_table(const uint64_t* __restrict__ keys, const int64_t* n_ptr, int n_patches,
                              int64_t* __restrict__ table) {
  const int64_t n = *n_ptr;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= n_patches; p += gridDim.x * blockDim.x) {
    const uint64_t k = uint64_t(p) << kPatchShift;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    table[p] = p == n_patches ? n : lo;
  }
}

struct vx_graph_impl {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

}  // namespace vx

struct vx_graph_s : vx::vx_graph_impl {};

using namespace vx;

namespace {

bool grid_ok(const vx_grid* g) {
  if (!g) return false;
  if (!(g->extent > 0.0) || !std::isfinite(g->extent)) return false;
  if (g->log2_res < 1 || g->log2_res > 20) return false;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(g->bmin[a])) return false;
  return true;
}

bool voxels_ok(const vx_voxels* v, bool need_mask) {
  return v && v->keys && v->count && v->w && v->S && v->cap >= 1 && (!need_mask || v->mask);
}

bool ws_ok(void* ws, size_t have, size_t need) {
  return ws && (reinterpret_cast<uintptr_t>(ws) % 256 == 0) && have >= need;
}

constexpr int64_t kMaxPairs = 0x7fffffff;
constexpr int64_t kMaxPrims = 0xffffffffll;   // primitive ids are 32-bit

}  // namespace

extern "C" {

size_t vx_voxelize_workspace_size(int32_t kind, int64_t n_prims, int64_t max_records, int64_t max_units,
                                  int64_t max_voxels, int32_t log2_res) {
  if ((kind != 0 && kind != 1) || n_prims < 0 || n_prims > kMaxPrims || max_records < 0 || max_units < 0 ||
      max_voxels < 1 || log2_res < 1 || log2_res > 20)
    return 0;
  return tile_ws_bytes(n_prims, max_records, max_units, max_voxels, log2_res > 10);
}

static vx_status voxelize_common(int kind, const vx_grid* grid, const float* data, int64_t n_prims,
                                 const int64_t* offsets, int64_t n_fib, float radius, int64_t max_records,
                                 int64_t max_units, void* ws, size_t ws_bytes, const vx_voxels* out,
                                 int64_t* stats, const vx_tuning* tuning, vx_stream stream) {
  Tuning tu;
  if (!resolve_tuning(tuning, kind, &tu)) return VX_ERR_ARG;
  if (!grid_ok(grid) || n_prims < 0 || n_prims > kMaxPrims || max_records < 0 || max_units < 0 || !stats ||
      !voxels_ok(out, false) || (n_prims > 0 && !data))
    return VX_ERR_ARG;
  if (kind == 1) {
    if (n_fib < 0 || !offsets || (n_prims > 0 && n_fib < 1)) return VX_ERR_ARG;
    if (!(radius >= 0.0f) || !std::isfinite(radius)) return VX_ERR_ARG;
    const double rho = std::rint(double(radius) * (std::ldexp(1.0, 23) / grid->extent));
    if (rho > 8388608.0) return VX_ERR_ARG;
  }
  if (!ws_ok(ws, ws_bytes, tile_ws_bytes(n_prims, max_records, max_units, out->cap, grid->log2_res > 10)))
    return VX_ERR_WORKSPACE;
  const int tb = std::min(tu.tile_bits, int(grid->log2_res));
  return tile_voxelize(kind, grid, data, n_prims, offsets, n_fib, radius, max_records, max_units, ws, out, stats,
                       reinterpret_cast<hipStream_t>(stream), nullptr, tb, tu);
}

vx_status vx_voxelize_triangles(const vx_grid* grid, const float* tris, int64_t n_tris, int64_t max_records,
                                int64_t max_units, void* ws, size_t ws_bytes, const vx_voxels* out,
                                int64_t* stats, const vx_tuning* tuning, vx_stream stream) {
  return voxelize_common(0, grid, tris, n_tris, nullptr, 0, 0.0f, max_records, max_units, ws, ws_bytes, out, stats,
                         tuning, stream);
}

vx_status vx_voxelize_fibers(const vx_grid* grid, const float* pts, int64_t n_pts, const int64_t* offsets,
                             int64_t n_fibers, float radius, int64_t max_records, int64_t max_units, void* ws,
                             size_t ws_bytes, const vx_voxels* out, int64_t* stats, const vx_tuning* tuning,
                             vx_stream stream) {
  return voxelize_common(1, grid, pts, n_pts, offsets, n_fibers, radius, max_records, max_units, ws, ws_bytes, out,
                         stats, tuning, stream);
}

static bool sampling_ok(int kind, const vx_sampling* sp) {
  if (!sp) return false;
  if (kind == 0) return sp->max_triangle_samples >= 1 && sp->max_triangle_samples <= (1 << 20);
  return sp->chords_per_segment >= 1 && sp->chords_per_segment <= 1024 && sp->samples_per_chord >= 1 &&
         sp->samples_per_chord <= 65536;
}

size_t vx_sample_workspace_size(int32_t kind, int64_t n_prims, int64_t max_samples, int64_t max_voxels,
                                int32_t log2_res, const vx_sampling* sampling) {
  if ((kind != 0 && kind != 1) || n_prims < 0 || n_prims > kMaxPrims || max_samples < 0 ||
      max_samples > kMaxPairs || max_voxels < 1 || log2_res < 1 || log2_res > 20 || !sampling_ok(kind, sampling))
    return 0;
  if (kind == 1 && n_prims * int64_t(sampling->chords_per_segment) > kMaxPrims + 1) return 0;
  return sample_ws_bytes(kind, n_prims, max_samples, max_voxels, log2_res, sampling->chords_per_segment);
}

static vx_status sample_common(int kind, const vx_grid* grid, const float* data, int64_t n_prims,
                               const int64_t* offsets, int64_t n_fib, const vx_sampling* sp, int64_t max_samples,
                               void* ws, size_t ws_bytes, const vx_voxels* out, int64_t* stats, vx_stream stream) {
  if (!grid_ok(grid) || n_prims < 0 || n_prims > kMaxPrims || max_samples < 0 || max_samples > kMaxPairs ||
      !stats || !voxels_ok(out, false) || (n_prims > 0 && !data) || !sampling_ok(kind, sp))
    return VX_ERR_ARG;
  if (kind == 1) {
    if (n_fib < 0 || !offsets || (n_prims > 0 && n_fib < 1)) return VX_ERR_ARG;
    if (n_prims * int64_t(sp->chords_per_segment) > kMaxPrims + 1) return VX_ERR_ARG;
  }
  if (!ws_ok(ws, ws_bytes, sample_ws_bytes(kind, n_prims, max_samples, out->cap, grid->log2_res,
                                           sp->chords_per_segment)))
    return VX_ERR_WORKSPACE;
  return sample_voxelize(kind, grid, data, n_prims, offsets, n_fib, sp, max_samples, ws, out, stats,
                         reinterpret_cast<hipStream_t>(stream));
}

vx_status vx_sample_triangles(const vx_grid* grid, const float* tris, int64_t n_tris, const vx_sampling* sampling,
                              int64_t max_samples, void* workspace, size_t ws_bytes, const vx_voxels* out,
                              int64_t* stats, vx_stream stream) {
  return sample_common(0, grid, tris, n_tris, nullptr, 0, sampling, max_samples, workspace, ws_bytes, out, stats,
                       stream);
}

vx_status vx_sample_fibers(const vx_grid* grid, const float* pts, int64_t n_pts, const int64_t* offsets,
                           int64_t n_fibers, const vx_sampling* sampling, int64_t max_samples, void* workspace,
                           size_t ws_bytes, const vx_voxels* out, int64_t* stats, vx_stream stream) {
  return sample_common(1, grid, pts, n_pts, offsets, n_fibers, sampling, max_samples, workspace, ws_bytes, out,
                       stats, stream);
}

vx_status vx_build_sggxh(const vx_grid* grid, const vx_voxels* leaf, const vx_voxels* out, const int64_t* n_levels,
                         int32_t levels, int32_t K, int32_t samples, const vx_lobes* lobes, int64_t* stats,
                         vx_stream stream) {
  if (!grid_ok(grid) || !voxels_ok(leaf, false) || !n_levels || levels < 2 || levels > grid->log2_res + 1 ||
      !out || !lobes || K < 1 || K > 8 || samples < 1 || samples > 65536 || !stats)
    return VX_ERR_ARG;
  for (int l = 1; l < levels; ++l) {
    if (!out[l - 1].keys || out[l - 1].cap < 1) return VX_ERR_ARG;
    const vx_lobes& b = lobes[l - 1];
    if (!b.nl || !b.w || !b.S || b.cap < 1) return VX_ERR_ARG;
  }
  return sggxh_run(grid, leaf, out, n_levels, levels, K, samples, lobes, stats, reinterpret_cast<hipStream_t>(stream));
}

size_t vx_occupancy_workspace_size(int32_t kind, int64_t n_prims, int64_t max_cand, int64_t max_pairs,
                                   int32_t log2_res) {
  if ((kind != 0 && kind != 1) || n_prims < 0 || n_prims > kMaxPrims || max_cand < 0 || max_pairs < 0 ||
      max_pairs > kMaxPairs || log2_res < 1 || log2_res > 17)
    return 0;
  return occupancy_ws_bytes(n_prims, max_cand, max_pairs, log2_res > 10);
}

static vx_status occupancy_common(int kind, const vx_grid* grid, const float* data, int64_t n_prims,
                                  const int64_t* offsets, int64_t n_fib, float radius, const vx_voxels* leaf,
                                  const vx_voxels* out, const int64_t* n_levels, int32_t levels, int64_t max_cand,
                                  int64_t max_pairs, const vx_occupancy* occ, void* ws, size_t ws_bytes,
                                  int64_t* stats, vx_stream stream) {
  if (!grid_ok(grid) || grid->log2_res > 17 || n_prims < 0 || n_prims > kMaxPrims || max_cand < 0 ||
      max_pairs < 0 || max_pairs > kMaxPairs || !stats || !n_levels || (n_prims > 0 && !data) ||
      !voxels_ok(leaf, false) || levels < 1 || levels > grid->log2_res + 1 || (levels > 1 && !out) || !occ)
    return VX_ERR_ARG;
  for (int l = 1; l < levels; ++l)
    if (!out[l - 1].keys || out[l - 1].cap < 1) return VX_ERR_ARG;
  for (int l = 0; l < levels; ++l)
    if (!occ[l].mask || !occ[l].hits || occ[l].cap < 1) return VX_ERR_ARG;
  if (kind == 1) {
    if (n_fib < 0 || !offsets || (n_prims > 0 && n_fib < 1)) return VX_ERR_ARG;
    if (!(radius >= 0.0f) || !std::isfinite(radius)) return VX_ERR_ARG;
    const double rho = std::rint(double(radius) * (std::ldexp(1.0, 23) / grid->extent));
    if (rho > 8388608.0) return VX_ERR_ARG;
  }
  if (!ws_ok(ws, ws_bytes, occupancy_ws_bytes(n_prims, max_cand, max_pairs, grid->log2_res > 10)))
    return VX_ERR_WORKSPACE;
  return occupancy_run(kind, grid, data, n_prims, offsets, n_fib, radius, leaf, out, n_levels, levels, max_cand,
                       max_pairs, occ, ws, stats, reinterpret_cast<hipStream_t>(stream));
}

vx_status vx_occupancy_triangles(const vx_grid* grid, const float* tris, int64_t n_tris, const vx_voxels* leaf,
                                 const vx_voxels* out, const int64_t* n_levels, int32_t levels, int64_t max_cand,
                                 int64_t max_pairs, const vx_occupancy* occ, void* workspace, size_t ws_bytes,
                                 int64_t* stats, vx_stream stream) {
  return occupancy_common(0, grid, tris, n_tris, nullptr, 0, 0.0f, leaf, out, n_levels, levels, max_cand, max_pairs,
                          occ, workspace, ws_bytes, stats, stream);
}

vx_status vx_occupancy_fibers(const vx_grid* grid, const float* pts, int64_t n_pts, const int64_t* offsets,
                              int64_t n_fibers, float radius, const vx_voxels* leaf, const vx_voxels* out,
                              const int64_t* n_levels, int32_t levels, int64_t max_cand, int64_t max_pairs,
                              const vx_occupancy* occ, void* workspace, size_t ws_bytes, int64_t* stats,
                              vx_stream stream) {
  return occupancy_common(1, grid, pts, n_pts, offsets, n_fibers, radius, leaf, out, n_levels, levels, max_cand,
                          max_pairs, occ, workspace, ws_bytes, stats, stream);
}

size_t vx_lod_workspace_size(int64_t cap, int32_t levels, int32_t K) {
  if (cap < 1 || levels < 1 || K < 1 || K > 8) return 0;
  Carver cv(nullptr);
  cv.take<int64_t>(cap + 1);   // parent starts
  cv.take<int64_t>(kGrid + 1); // scan partials
  return cv.off + 256;
}

}  // extern "C"

namespace {

vx_status lod_args(const vx_grid* grid, const vx_voxels* leaf, const int64_t* n_leaf, int32_t levels, int32_t K,
                   int32_t kmeans_iters, const vx_voxels* out, const vx_lobes* lobes, const int64_t* n_levels) {
  if (!grid_ok(grid) || !voxels_ok(leaf, false) || !n_leaf || !n_levels || levels < 1 ||
      levels > grid->log2_res + 1 || K < 1 || K > 8 || kmeans_iters < 0)
    return VX_ERR_ARG;
  if (levels > 1 && !out) return VX_ERR_ARG;
  for (int L = 1; L < levels; ++L) {
    if (!voxels_ok(&out[L - 1], true)) return VX_ERR_ARG;
    if (K > 1) {
      if (!lobes) return VX_ERR_ARG;
      const vx_lobes& lb = lobes[L - 1];
      if (!lb.nl || !lb.w || !lb.S || lb.cap < out[L - 1].cap) return VX_ERR_ARG;
    }
  }
  return VX_OK;
}

// the pyramid on the caller's stream; pstart [leaf->cap + 1] and partial [kGrid + 1] are scratch
// that every kernel writes before it reads (no clearing needed)
vx_status lod_run(const vx_grid* grid, const vx_voxels* leaf, const int64_t* n_leaf, int32_t levels, int32_t K,
                  int32_t kmeans_iters, const vx_voxels* out, const vx_lobes* lobes, int64_t* n_levels,
                  int64_t* pstart, int64_t* partial, const Tuning& tu, hipStream_t s) {
  const bool key64 = grid->log2_res > 10;
  lod_init(n_leaf, leaf->cap, n_levels, int64_t(levels) + 1, s);
  int L = 1;
  for (; L < levels; ++L) {
    const vx_voxels& in = L == 1 ? *leaf : out[L - 2];
    if (K == 1 && in.cap <= kTailMax) break;       // the small top levels go in one launch
    lod_level(key64, in, n_levels + L - 1, out[L - 1], n_levels + L, n_levels + levels, pstart,
              partial, tu.grids[kTuneLod], s);
    if (K > 1) {
      if (L == 1)
        cluster_level(pstart, n_levels + 1, leaf->w, leaf->S, nullptr, 1, leaf->cap, K, kmeans_iters, lobes[0],
                      tu.grids[kTuneCluster], s);
      else
        cluster_level(pstart, n_levels + L, lobes[L - 2].w, lobes[L - 2].S, lobes[L - 2].nl, K, lobes[L - 2].cap, K,
                      kmeans_iters, lobes[L - 1], tu.grids[kTuneCluster], s, L == 2);
    }
  }
  if (L < levels) {
    vx_voxels lv[21];
    int64_t* nl[21];
    lv[0] = L == 1 ? *leaf : out[L - 2];
    nl[0] = n_levels + L - 1;
    for (int i = 1; i <= levels - L; ++i) {
      lv[i] = out[L - 2 + i];
      nl[i] = n_levels + L - 1 + i;
    }
    lod_tail(key64, false, lv, nl, levels - L, n_levels + levels, s);
  }
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

// Scratch of the allocation-free pyramid entry point: parent starts of a leaf of up to
// VX_LOD_NOALLOC_MAX_LEAF voxels, then the scan partials.  Each GPU holds its own copy for the
// life of the process; its device address is looked up once per device (the array's name is a
// host-side stand-in and never reaches a kernel).
constexpr int64_t kNoAllocWords = VX_LOD_NOALLOC_MAX_LEAF + 1 + (kGrid + 1);
static __device__ __align__(256) int64_t scratch[kNoAllocWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int64_t* g_scratch_ptr[kMaxDevices] = {};

vx_status scratch_for_current_device(int64_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VX_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return VX_ERR_HIP;
    g_scratch_ptr[dev] = static_cast<int64_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return VX_OK;
}

}  // namespace

extern "C" {

vx_status vx_build_lod(const vx_grid* grid, const vx_voxels* leaf, const int64_t* n_leaf, int32_t levels, int32_t K,
                       int32_t kmeans_iters, const vx_voxels* out, const vx_lobes* lobes, int64_t* n_levels,
                       void* ws, size_t ws_bytes, const vx_tuning* tuning, vx_stream stream) {
  const vx_status st = lod_args(grid, leaf, n_leaf, levels, K, kmeans_iters, out, lobes, n_levels);
  if (st != VX_OK) return st;
  Tuning tu;
  if (!resolve_tuning(tuning, 1, &tu)) return VX_ERR_ARG;
  if (!ws_ok(ws, ws_bytes, vx_lod_workspace_size(leaf->cap, levels, K))) return VX_ERR_WORKSPACE;
  Carver cv(ws);
  int64_t* pstart = cv.take<int64_t>(leaf->cap + 1);
  int64_t* partial = cv.take<int64_t>(kGrid + 1);
  return lod_run(grid, leaf, n_leaf, levels, K, kmeans_iters, out, lobes, n_levels, pstart, partial, tu,
                 reinterpret_cast<hipStream_t>(stream));
}

vx_status vx_build_lod_noalloc(const vx_grid* grid, const vx_voxels* leaf, const int64_t* n_leaf, int32_t levels,
                               int32_t K, int32_t kmeans_iters, const vx_voxels* out, const vx_lobes* lobes,
                               int64_t* n_levels, const vx_tuning* tuning, vx_stream stream) {
  const vx_status st = lod_args(grid, leaf, n_leaf, levels, K, kmeans_iters, out, lobes, n_levels);
  if (st != VX_OK) return st;
  Tuning tu;
  if (!resolve_tuning(tuning, 1, &tu)) return VX_ERR_ARG;
  if (leaf->cap > VX_LOD_NOALLOC_MAX_LEAF) return VX_ERR_CAPACITY;
  int64_t* base = nullptr;
  const vx_status sst = scratch_for_current_device(&base);
  if (sst != VX_OK) return sst;
  return lod_run(grid, leaf, n_leaf, levels, K, kmeans_iters, out, lobes, n_levels, base,
                 base + VX_LOD_NOALLOC_MAX_LEAF + 1, tu, reinterpret_cast<hipStream_t>(stream));
}

size_t vx_fit_workspace_size(int64_t n_pts, int64_t max_cand, int64_t max_pairs, const int64_t* caps, int32_t hi,
                             int32_t log2_res) {
  if (n_pts < 0 || max_cand < 0 || max_pairs < 0 || max_pairs > kMaxPairs || !caps || hi < 1 || hi > 20 ||
      log2_res < 1 || log2_res > 20)
    return 0;
  for (int L = 0; L <= hi; ++L)
    if (caps[L] < 1) return 0;
  return fit_ws_bytes(n_pts, max_cand, max_pairs, caps, hi, log2_res);
}

static bool fit_args_ok(const vx_grid* grid, const vx_voxels* levels, const int64_t* n_levels, int lo, int hi,
                        const float* const* params, const int64_t* rows, const void* const* bound, const float* dirs,
                        int ndir, const int64_t* caps) {
  if (!grid_ok(grid) || !levels || !n_levels || lo < 1 || hi < lo || hi > 20 || hi > grid->log2_res || !params ||
      !rows || !dirs || ndir < 1 || ndir > 256 || !caps)
    return false;
  for (int L = 0; L <= hi; ++L)
    if (!voxels_ok(&levels[L], false) || caps[L] < levels[L].cap) return false;
  for (int L = lo; L <= hi; ++L)
    if (!params[L - lo] || rows[L - lo] < 0 || rows[L - lo] > caps[L] || (bound && !bound[L - lo] && rows[L - lo] > 0))
      return false;
  return true;
}

vx_status vx_fit_forward(const vx_grid* grid, const vx_voxels* levels, const int64_t* n_levels, int32_t lo,
                         int32_t hi, const float* const* params, const int64_t* rows, const void* const* bound,
                         const float* dirs, int32_t ndir, float* loss, int64_t* stats, const int64_t* caps, void* ws,
                         size_t ws_bytes, vx_stream stream) {
  if (!fit_args_ok(grid, levels, n_levels, lo, hi, params, rows, bound, dirs, ndir, caps) || !loss || !stats)
    return VX_ERR_ARG;
  if (!ws_ok(ws, ws_bytes, fit_ws_bytes(0, 0, 0, caps, hi, grid->log2_res))) return VX_ERR_WORKSPACE;
  return fit_forward_run(grid, levels, n_levels, lo, hi, params, rows, bound, dirs, ndir, loss, stats, ws, caps,
                         reinterpret_cast<hipStream_t>(stream));
}

vx_status vx_fit_backward(const vx_grid* grid, const vx_fibers* fib, int64_t max_cand, int64_t max_pairs,
                          const vx_voxels* levels, const int64_t* n_levels, int32_t lo, int32_t hi,
                          const float* const* params, const int64_t* rows, const void* const* bound,
                          const float* dirs, int32_t ndir, const float* dloss, float* const* dparams, float* dpts,
                          int64_t* stats, const int64_t* caps, void* ws, size_t ws_bytes, vx_stream stream) {
  if (!fit_args_ok(grid, levels, n_levels, lo, hi, params, rows, bound, dirs, ndir, caps) || !fib || !dloss ||
      !dparams || !dpts || !stats || max_cand < 0 || max_pairs < 0 || max_pairs > kMaxPairs)
    return VX_ERR_ARG;
  if (fib->n_pts < 0 || fib->n_fibers < 0 || !fib->offsets || (fib->n_pts > 0 && (!fib->pts || fib->n_fibers < 1)))
    return VX_ERR_ARG;
  if (!(fib->radius >= 0.0f) || !std::isfinite(fib->radius)) return VX_ERR_ARG;
  for (int L = lo; L <= hi; ++L)
    if (!dparams[L - lo]) return VX_ERR_ARG;
  if (!ws_ok(ws, ws_bytes, fit_ws_bytes(fib->n_pts, max_cand, max_pairs, caps, hi, grid->log2_res)))
    return VX_ERR_WORKSPACE;
  return fit_backward_run(grid, fib->pts, fib->n_pts, fib->offsets, fib->n_fibers, fib->radius, max_cand, max_pairs,
                          levels, n_levels, lo, hi, params, rows, bound, dirs, ndir, dloss, dparams, dpts, stats, ws,
                          caps, reinterpret_cast<hipStream_t>(stream));
}

size_t vx_batch_workspace_size(int32_t n_patches, int64_t n_pts, int64_t max_records, int64_t max_units,
                               int64_t leaf_cap) {
  if (n_patches < 1 || n_patches > 65536 || n_pts < 0 || n_pts > kMaxPrims || max_records < 0 || max_units < 0 ||
      leaf_cap < 1)
    return 0;
  // batch tables + the tile workspace with 64-bit keys + the pyramid's parent starts
  Carver cv(nullptr);
  cv.take<Lat>(n_patches);
  cv.take<int64_t>(n_patches + 1);
  cv.take<int64_t>(leaf_cap + 1);
  cv.take<int64_t>(kGrid + 1);
  return cv.off + tile_ws_bytes(n_pts, max_records, max_units, leaf_cap, true) + 512;
}

vx_status vx_batch_build(const vx_patch* patches, const vx_patch* patches_dev, int32_t n_patches, const float* pts,
                         int64_t n_pts, const int64_t* offsets, int64_t n_fibers, int32_t levels, int32_t K,
                         int32_t kmeans_iters, int64_t max_records, int64_t max_units, const vx_voxels* out,
                         const vx_lobes* lobes, int64_t* n_levels, int64_t* patch_table, int64_t* stats, void* ws,
                         size_t ws_bytes, const vx_tuning* tuning, vx_stream stream) {
  Tuning tu;
  if (!resolve_tuning(tuning, 1, &tu)) return VX_ERR_ARG;
  if (!patches || !patches_dev || n_patches < 1 || n_patches > 65536 || n_pts < 0 || n_pts > kMaxPrims || !offsets ||
      n_fibers < 0 || (n_pts > 0 && (!pts || n_fibers < 1)) || levels < 1 || K < 1 || K > 8 || kmeans_iters < 0 ||
      max_records < 0 || max_units < 0 || !out || !n_levels || !patch_table || !stats)
    return VX_ERR_ARG;
  int max_levels = 0, min_log2 = 64;
  for (int p = 0; p < n_patches; ++p) {
    const vx_patch& P = patches[p];
    if (!grid_ok(&P.grid) || P.grid.log2_res > 11) return VX_ERR_ARG;
    if (!(P.radius >= 0.0f) || !std::isfinite(P.radius)) return VX_ERR_ARG;
    if (std::rint(double(P.radius) * (std::ldexp(1.0, 23) / P.grid.extent)) > 8388608.0) return VX_ERR_ARG;
    if (P.pt_begin != (p == 0 ? 0 : patches[p - 1].pt_end) || P.pt_end < P.pt_begin) return VX_ERR_ARG;
    max_levels = std::max(max_levels, P.grid.log2_res + 1);
    min_log2 = std::min(min_log2, int(P.grid.log2_res));
  }
  if (patches[n_patches - 1].pt_end != n_pts || levels > max_levels) return VX_ERR_ARG;
  if (!voxels_ok(&out[0], false)) return VX_ERR_ARG;
  for (int L = 1; L < levels; ++L) {
    if (!voxels_ok(&out[L], true)) return VX_ERR_ARG;
    if (K > 1 && (!lobes || !lobes[L - 1].nl || !lobes[L - 1].w || !lobes[L - 1].S || lobes[L - 1].cap < out[L].cap))
      return VX_ERR_ARG;
  }
  const int64_t leaf_cap = out[0].cap;
  if (!ws_ok(ws, ws_bytes, vx_batch_workspace_size(n_patches, n_pts, max_records, max_units, leaf_cap)))
    return VX_ERR_WORKSPACE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Carver cv(ws);
  Lat* lats = cv.take<Lat>(n_patches);
  int64_t* pt_begin = cv.take<int64_t>(n_patches + 1);
  int64_t* pstart = cv.take<int64_t>(leaf_cap + 1);
  int64_t* partial = cv.take<int64_t>(kGrid + 1);
  void* vws = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(ws) + cv.off + 255) & ~uintptr_t(255));
  hipLaunchKernelGGL(k_batch_setup, dim3((n_patches + 255) / 256), dim3(256), 0, s, patches_dev, n_patches, lats,
                     pt_begin);
  BatchLattice bl{lats, pt_begin, n_patches};
  vx_status st = tile_voxelize(1, &patches[0].grid, pts, n_pts, offsets, n_fibers, 0.0f, max_records, max_units, vws,
                               &out[0], stats, s, &bl, std::min(tu.tile_bits, min_log2), tu);
  if (st != VX_OK) return st;
  // the pyramid, with the patch-preserving parent
  lod_init(stats + VX_STAT_VOXELS, leaf_cap, n_levels, int64_t(levels) + 1, s);
  int L = 1;
  for (; L < levels; ++L) {
    if (K == 1 && out[L - 1].cap <= kTailMax) break;
    lod_level(true, out[L - 1], n_levels + L - 1, out[L], n_levels + L, n_levels + levels, pstart,
              partial, tu.grids[kTuneLod], s, true);
    if (K > 1) {
      if (L == 1)
        cluster_level(pstart, n_levels + 1, out[0].w, out[0].S, nullptr, 1, out[0].cap, K, kmeans_iters, lobes[0],
                      tu.grids[kTuneCluster], s);
      else
        cluster_level(pstart, n_levels + L, lobes[L - 2].w, lobes[L - 2].S, lobes[L - 2].nl, K, lobes[L - 2].cap, K,
                      kmeans_iters, lobes[L - 1], tu.grids[kTuneCluster], s, L == 2);
    }
  }
  if (L < levels) {
    vx_voxels lv[21];
    int64_t* nl[21];
    for (int i = 0; i <= levels - L; ++i) {
      lv[i] = out[L - 1 + i];
      nl[i] = n_levels + L - 1 + i;
    }
    lod_tail(true, true, lv, nl, levels - L, n_levels + levels, s);
  }
  for (int L = 0; L < levels; ++L)
    hipLaunchKernelGGL(k_patch_table, dim3((n_patches + 256) / 256), dim3(256), 0, s, (const uint64_t*)out[L].keys,
                       n_levels + L, n_patches, patch_table + int64_t(L) * (n_patches + 1));
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

vx_status vx_graph_begin(vx_stream stream) {
  if (!stream) return VX_ERR_ARG;
  return hipStreamBeginCapture(reinterpret_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal) == hipSuccess
             ? VX_OK
             : VX_ERR_HIP;
}

vx_status vx_graph_end(vx_stream stream, vx_graph* graph) {
  if (!stream || !graph) return VX_ERR_ARG;
  vx_graph g = new vx_graph_s;
  if (hipStreamEndCapture(reinterpret_cast<hipStream_t>(stream), &g->graph) != hipSuccess) {
    delete g;
    return VX_ERR_HIP;
  }
  if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g->graph);
    delete g;
    return VX_ERR_HIP;
  }
  *graph = g;
  return VX_OK;
}

vx_status vx_graph_launch(vx_graph graph, vx_stream stream) {
  if (!graph) return VX_ERR_ARG;
  return hipGraphLaunch(graph->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? VX_OK : VX_ERR_HIP;
}

void vx_graph_destroy(vx_graph graph) {
  if (!graph) return;
  (void)hipGraphExecDestroy(graph->exec);
  (void)hipGraphDestroy(graph->graph);
  delete graph;
}


vx_status vx_check_stats(const int64_t* stats, vx_stream stream) {
  if (!stats) return VX_ERR_ARG;
  if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return VX_ERR_HIP;
  int64_t h[VX_NSTAT];
  if (hipMemcpy(h, stats, sizeof h, hipMemcpyDeviceToHost) != hipSuccess) return VX_ERR_HIP;
  const int64_t f = h[VX_STAT_FLAGS];
  if (f & (VX_FLAG_INPUT | VX_FLAG_OFFSETS)) return VX_ERR_INPUT;
  if (f & (VX_FLAG_FIT_KEYS | VX_FLAG_OCC_LEAF)) return VX_ERR_BINDING;
  if (f & (VX_FLAG_FIT_ROWS | VX_FLAG_CAND_CAPACITY | VX_FLAG_PAIR_CAPACITY | VX_FLAG_VOXEL_CAPACITY | VX_FLAG_RECORD_CAPACITY |
           VX_FLAG_UNIT_CAPACITY))
    return VX_ERR_CAPACITY;
  return VX_OK;
}

const char* vx_status_str(vx_status s) {
  switch (s) {
    case VX_OK: return "ok";
    case VX_ERR_ARG: return "invalid argument";
    case VX_ERR_CAPACITY: return "capacity exceeded";
    case VX_ERR_HIP: return "HIP runtime error";
    case VX_ERR_INPUT: return "non-finite or out-of-range input, or invalid fiber offsets";
    case VX_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case VX_ERR_BINDING: return "arguments bound to other voxels than the level holds";
  }
  return "unknown status";
}

void vx_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
}

void vx_timing_filter(const char* name) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_filter = name ? name : "";
}

void vx_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& p : g_pending) {
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
  g_acc.clear();
}

int32_t vx_timing_collect(char names[][48], double* total_ms, int64_t* launches, int32_t max_entries) {
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipDeviceSynchronize();
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) ms = 0.f;
    Acc* a = nullptr;
    for (auto& x : g_acc)
      if (x.name == p.name) a = &x;
    if (!a) {
      g_acc.push_back(Acc{p.name, 0.0, 0});
      a = &g_acc.back();
    }
    a->ms += ms;
    a->n += 1;
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
  int32_t k = 0;
  for (auto& x : g_acc) {
    if (k < max_entries) {
      std::strncpy(names[k], x.name.c_str(), 47);
      names[k][47] = 0;
      total_ms[k] = x.ms;
      launches[k] = x.n;
    }
    ++k;
  }
  return k;
}

vx_status vx_sggx_compact(const vx_voxels* vox, const int64_t* n_vox, float eps, float* lam, float* vec,
                          uint8_t* code, vx_stream stream) {
  if (!vox || !vox->w || !vox->S || vox->cap < 1 || !n_vox || !code || !(eps > 0.0f) || !(eps <= 1.0f) ||
      reinterpret_cast<uintptr_t>(code) % 2 != 0)
    return VX_ERR_ARG;
  sggx_compact_run(vox->w, vox->S, n_vox, vox->cap, double(eps), lam, vec, code,
                   reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

vx_status vx_sggx_decode(const uint8_t* code, const int64_t* n, int64_t cap, float* S, vx_stream stream) {
  if (!code || !n || !S || cap < 1 || reinterpret_cast<uintptr_t>(code) % 2 != 0) return VX_ERR_ARG;
  sggx_decode_run(code, n, cap, S, reinterpret_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? VX_OK : VX_ERR_HIP;
}

}  // extern "C"
