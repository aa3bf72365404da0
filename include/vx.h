/* vx.h -- C ABI of libvx.so: sparse SGGX voxelization and LoD pyramids on gfx950.
 *
 * The operations follow "Fast Voxelization and Level of Detail for Microgeometry Rendering"
 * (arXiv 2604.13191):
 *   voxelize(primitives, grid bounds, resolution) -> sparse Morton-keyed leaf voxels
 *       Sec. 3.1 (grid transform, node records), Sec. 3.2-3.3 (generating and gathering
 *       everything a primitive contributes to a leaf voxel), Sec. 3.4 and Sec. 4.1 (one SGGX
 *       matrix per voxel, fitted from the voxel's orientation data);
 *   build_lod(voxels, levels, lobes_per_voxel) -> pyramid
 *       Sec. 4.3 (2x2x2 aggregation of SGGX into coarser levels) and Sec. 4.4 (merging the
 *       most similar lobes, with a cap on the number kept per voxel).
 *
 * What this library computes, exactly (the paper samples points; this is the exact-measure
 * reading of the same aggregation):
 *   - Grid: cubic bounds [bmin, bmin + extent)^3, R = 2^log2_res voxels per axis.  Every
 *     vertex is mapped as in Sec. 3.1 and snapped to the lattice of 2^-(23 - log2_res) voxel:
 *         q = rint((double(P) - bmin) * (2^23 / extent))      (IEEE double, round half even)
 *     so a voxel is s = 2^(23 - log2_res) lattice units.  |q| must stay within one grid of the
 *     bounds (q in [-2^23, 2^24]); otherwise the call reports VX_ERR_INPUT.
 *   - A triangle touches voxel v when it meets the closed box [v, v+1]^3; a fiber segment
 *     touches v when its centreline is within distance `radius` of that closed box.  Both
 *     predicates are exact on the lattice.  Voxels outside [0, R)^3 are dropped.
 *   - Weight of a (primitive, voxel) pair: area of the triangle inside the half-open box
 *     [v, v+1)^3, or length of the centreline inside it, in voxel units (voxel^2, voxel).
 *   - Moment: M = n n^T (unit triangle normal) or M = I - t t^T (unit segment tangent); zero
 *     for degenerate primitives.
 *   - Per leaf voxel: count = number of touching primitives, w = sum of weights,
 *     S = sum of weight * M (unnormalised; the SGGX matrix is S / w).
 *   - Key: Morton code, x bit b at key bit 3b, y at 3b+1, z at 3b+2.  Keys are 32-bit when
 *     3 * log2_res <= 30 (log2_res <= 10) and 64-bit otherwise.  Parent key = key >> 3.
 *
 * Memory: every pointer argument is device memory owned by the caller unless stated.  The
 * library allocates nothing on these paths; scratch comes from the caller's workspace whose
 * size the *_workspace_size() calls return.  Work is enqueued on `stream` and returns
 * without synchronising.  Counts are written to device memory; nothing is copied to the host.
 *
 * Errors: arguments the host can check are rejected before anything is enqueued (the
 * return value).  Conditions found on the device (a capacity too small, a non-finite or
 * out-of-range coordinate) set bits in stats[VX_STAT_FLAGS]; the outputs are then invalid,
 * the true required sizes are still written to stats, and vx_check_stats() (which
 * synchronises the stream) turns the flags into a status.  Calls on one stream are ordered;
 * calls that share a workspace must not overlap.
 */
#ifndef VX_H
#define VX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* vx_stream;   /* a hipStream_t; NULL = the null stream */

typedef enum {
  VX_OK = 0,
  VX_ERR_ARG = 1,        /* bad argument (host-checked) */
  VX_ERR_CAPACITY = 2,   /* a device-detected count exceeded the capacity given */
  VX_ERR_HIP = 3,        /* a HIP runtime call failed */
  VX_ERR_INPUT = 4,      /* non-finite or out-of-range coordinate, or invalid fiber offsets */
  VX_ERR_WORKSPACE = 5,  /* workspace pointer NULL, misaligned (256 B) or too small */
  VX_ERR_BINDING = 6     /* arguments bound to other voxels than the level holds (fit parameters,
                            an occupancy leaf from other primitives) */
} vx_status;

/* device flag bits in stats[VX_STAT_FLAGS] */
#define VX_FLAG_CAND_CAPACITY  1
#define VX_FLAG_PAIR_CAPACITY  2
#define VX_FLAG_VOXEL_CAPACITY 4
#define VX_FLAG_INPUT          8
#define VX_FLAG_OFFSETS        16
#define VX_FLAG_RECORD_CAPACITY 32
#define VX_FLAG_UNIT_CAPACITY  64
#define VX_FLAG_FIT_ROWS       128   /* a fitted level's voxel count differs from its parameter rows */
#define VX_FLAG_FIT_KEYS       256   /* a fitted level's keys differ from those its parameters were made for */
#define VX_FLAG_OCC_LEAF       512   /* a primitive touches a voxel missing from the leaf given for occupancy */

/* indices into the int64 stats array (device): candidates tested, touching pairs, leaf voxels,
 * flags, primitive-tile records, work units */
enum {
  VX_STAT_CAND = 0,
  VX_STAT_PAIRS = 1,
  VX_STAT_VOXELS = 2,
  VX_STAT_FLAGS = 3,
  VX_STAT_RECORDS = 4,
  VX_STAT_UNITS = 5,
  VX_NSTAT = 6
};

typedef struct {
  double bmin[3];
  double extent;      /* > 0, cubic bounds */
  int32_t log2_res;   /* 1 .. 20 */
} vx_grid;

/* One level of voxels, structure of arrays, capacity `cap` entries.  Entry i is valid for
 * i < n, where n is written to device memory by the producing call. */
typedef struct {
  void* keys;         /* uint32[cap] (log2_res <= 10) or uint64[cap] */
  uint32_t* count;    /* [cap] primitive-voxel pairs under the voxel */
  float* w;           /* [cap] summed weight */
  float* S;           /* [6 * cap]: S[c * cap + i], c = xx, yy, zz, xy, xz, yz */
  uint8_t* mask;      /* [cap] child mask, bit b = child (key << 3 | b) present; NULL at the leaf */
  int64_t cap;
} vx_voxels;

/* Up to K SGGX lobes per voxel of one level (K > 1 only). */
typedef struct {
  uint8_t* nl;        /* [cap] number of lobes (0 when w == 0) */
  float* w;           /* [K * cap]: w[k * cap + i], sorted by descending weight */
  float* S;           /* [6 * K * cap]: S[(c * K + k) * cap + i] */
  int64_t cap;
} vx_lobes;

/* ------------------------------------------------------------------------------------------
 * Tuning (chosen by the project's autotuner per workload; NULL or zero fields = defaults).  It
 * changes the work decomposition, never a result:
 *   tile_bits    leaf tiles of 2^tile_bits voxels per axis (2, 3 or 4; default 4), the spatial
 *                bins the primitive-tile records are sorted by
 *   unit_budget  candidates one work unit keeps in LDS (1024, 1536, 2048 or 3072; default 1536
 *                for triangles, 3072 for fibers); smaller budgets split crowded tiles further and
 *                let more units share a compute unit
 *   grids        blocks of the persistent kernels: unit kernel, unit planner, leaf compaction,
 *                parent reduce, lobe clustering (each 64 .. 16384; defaults 16384, 8192, 16384,
 *                512, 8192)
 * Invalid values return VX_ERR_ARG.  The library keeps no tuning state of its own.
 * ------------------------------------------------------------------------------------------ */
#define VX_TUNE_COUNT 5
typedef struct {
  int32_t tile_bits;
  int32_t unit_budget;
  int32_t grids[VX_TUNE_COUNT];
} vx_tuning;

/* ------------------------------------------------------------------------------------------
 * Voxelization (Sec. 3.1-3.4).
 *
 * The grid is cut into aligned tiles of 16^3 voxels (Sec. 3.1's blocks); every primitive is
 * listed once per tile its candidate box (closed bounding box, dilated by the radius for
 * fibers, clipped to the grid) overlaps, and tiles with many candidates are split into octants
 * ("units") whose candidates fit on chip.  Capacities:
 * kind: 0 = triangles (n_prims = number of triangles), 1 = fibers (n_prims = number of points).
 * max_records: primitive-tile records (stats[VX_STAT_RECORDS] of a call with 0 reports it).
 * max_units: work units (stats[VX_STAT_UNITS]).
 * max_voxels: the leaf capacity the call will be given (out->cap <= max_voxels).
 * Returns the workspace size in bytes (0 on bad arguments).
 * ------------------------------------------------------------------------------------------ */
size_t vx_voxelize_workspace_size(int32_t kind, int64_t n_prims, int64_t max_records, int64_t max_units,
                                  int64_t max_voxels, int32_t log2_res);

/* tris: float32 [n_tris][3][3] (vertex-major; a soup of non-shared vertices, Sec. 3.2).
 * out: leaf voxels (out->mask unused), sorted by key, unique keys.
 * stats: int64[VX_NSTAT] on the device, overwritten. */
vx_status vx_voxelize_triangles(const vx_grid* grid, const float* tris, int64_t n_tris,
                                int64_t max_records, int64_t max_units, void* workspace, size_t ws_bytes,
                                const vx_voxels* out, int64_t* stats, const vx_tuning* tuning, vx_stream stream);

/* pts: float32 [n_pts][3] polyline nodes (Sec. 3.1 node collections); offsets: int64
 * [n_fibers + 1] (device), offsets[0] = 0, non-decreasing, offsets[n_fibers] = n_pts.  Segment
 * (i, i+1) exists when both points belong to one fiber; radius in world units, >= 0. */
vx_status vx_voxelize_fibers(const vx_grid* grid, const float* pts, int64_t n_pts, const int64_t* offsets,
                             int64_t n_fibers, float radius, int64_t max_records, int64_t max_units,
                             void* workspace, size_t ws_bytes, const vx_voxels* out, int64_t* stats,
                             const vx_tuning* tuning, vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * Sampling voxelizer (Sec. 3.2 sparse data sampling, Sec. 3.3 gathering): the paper's own
 * method, kept as the baseline of the exact path above.  Points are placed on the primitives
 * from their indices (no random numbers) and every point is stored in the voxel containing it:
 *   fibers     every segment (i, i+1) of a fiber is the uniform Catmull-Rom span through points
 *              i-1, i, i+1, i+2 (a fiber's end points repeated), cut at t = j / m (j = 0 .. m)
 *              into m chords; each chord carries n samples at fractions (k + 1/2) / n of it, each
 *              weighing chord length / n, moment I - t t^T of the chord's tangent;
 *   triangles  triangle T gets n_T = max(1, floor(N * area_T / area_max)) samples (the area
 *              relative to the largest triangle's), sample k at (u1, u2) = ((k + 1/2) / n_T,
 *              radical inverse of k in base 2), mapped to barycentric coordinates by Heitz's
 *              low-distortion square-to-triangle map, each weighing area_T / n_T, moment n n^T.
 * Positions are FP64 grid units g = (P - bmin) * 2^log2_res / extent, every operation in a fixed
 * order (the fused multiply-adds are explicit); the sample's voxel is floor(g), samples outside
 * [0, R)^3 are dropped, and n_T's floor is decided on squares (k^2 area_max^2 <= N^2 area_T^2).
 * Per voxel: count = samples, w = summed weight, S = summed weight * moment, summed in sample
 * order (primitive, chord, sample), so the result is reproducible bit for bit.
 * Capacities: max_samples = samples generated (stats[VX_STAT_CAND] of a call with 0 reports it);
 * stats[VX_STAT_PAIRS] = samples inside the grid, stats[VX_STAT_VOXELS] = voxels.
 * Workspace: about 2 * (key + 8) bytes per sample plus 16 bytes per chord or triangle.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t chords_per_segment;    /* fibers: m, 1 .. 1024 */
  int32_t samples_per_chord;     /* fibers: n, 1 .. 65536 */
  int32_t max_triangle_samples;  /* triangles: N, the largest triangle's samples, 1 .. 2^20 */
} vx_sampling;

/* kind: 0 = triangles, 1 = fibers; n_prims as for vx_voxelize_workspace_size; 0 on bad
 * arguments. */
size_t vx_sample_workspace_size(int32_t kind, int64_t n_prims, int64_t max_samples, int64_t max_voxels,
                                int32_t log2_res, const vx_sampling* sampling);

/* tris: float32 [n_tris][3][3] on the device.  out: voxels sorted by key (out->mask unused). */
vx_status vx_sample_triangles(const vx_grid* grid, const float* tris, int64_t n_tris, const vx_sampling* sampling,
                              int64_t max_samples, void* workspace, size_t ws_bytes, const vx_voxels* out,
                              int64_t* stats, vx_stream stream);

/* pts, offsets: as for vx_voxelize_fibers (n_pts * chords_per_segment <= 2^32). */
vx_status vx_sample_fibers(const vx_grid* grid, const float* pts, int64_t n_pts, const int64_t* offsets,
                           int64_t n_fibers, const vx_sampling* sampling, int64_t max_samples, void* workspace,
                           size_t ws_bytes, const vx_voxels* out, int64_t* stats, vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * SGGX-H lobes (Sec. 4.4, the paper's own reduction; vx_build_lod's K > 1 lobes use the
 * deterministic moment metric instead).
 *
 * Level L voxel gathers its children's lobes (level 1: one per leaf voxel; level L > 1: the
 * SGGX-H lobes of level L - 1), drops zero weights, and while more than K remain merges the two
 * closest (w and S added).  Closeness: each lobe's normals are sampled `samples` times -- the
 * SGGX of S / w with 1e-3 of its trace added to the diagonal, n = L u / |L u| for S = L L^T and
 * u uniform on the sphere (rejection from the cube), accepted with probability |L u| /
 * sqrt(tr S); draw d of sample k is SplitMix64 output k 2^32 + d of the seed
 * mix(mix(key + g (L + 1)) + g (slot + 1)), g = 0x9E3779B97F4A7C15, mix = SplitMix64's output
 * function, key the voxel's Morton key, slot the lobe's index among the voxel's positive input
 * lobes -- into 5 bins per axis (floor((n_a + 1) 2.5)); the distance is the Wasserstein-1
 * distance between the per-axis marginals, summed over the axes; a merged lobe pools the samples
 * of its parts.  Closest pair ties go to the first (i, j) in slot order; the survivors are
 * sorted by descending weight.  The sampling is bit-reproducible (integer counts of IEEE double
 * decisions), so the partition is deterministic; w and S are FP32 sums.
 * leaf, out, n_levels: the pyramid of vx_build_lod (levels as there); lobes: levels - 1 outputs
 * (K 1 .. 8, caps at least the levels' counts); samples 1 .. 65536 (the paper uses 5000).
 * stats: int64[VX_NSTAT] (flags only: VX_FLAG_VOXEL_CAPACITY when a level exceeds a cap).
 * ------------------------------------------------------------------------------------------ */
vx_status vx_build_sggxh(const vx_grid* grid, const vx_voxels* leaf, const vx_voxels* out, const int64_t* n_levels,
                         int32_t levels, int32_t K, int32_t samples, const vx_lobes* lobes, int64_t* stats,
                         vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * Sub-voxel occupancy and projected densities (Sec. 3.5 occupancy equation and XY / XZ / YZ
 * projections, Sec. 4.2 the projections at the coarser levels).
 *
 * Every voxel of every level holds 8^3 sub-cells of its edge / 8.  A leaf sub-cell is hit when a
 * primitive touches its closed box (the voxel-level predicate on the same lattice); a coarser
 * voxel's sub-cell, the union of 2 x 2 x 2 sub-cells of one child, is hit when one of those is.
 * Per voxel:
 *   mask   512 bits, sub-cell (i, j, k) in [0, 8)^3 at Morton index m (i bit b at 3b, j at 3b+1,
 *          k at 3b+2): bit m & 63 of word m >> 6 -- word c is octant c of the voxel;
 *   hits   hit sub-cells (occupancy O = hits / 512), and the cells of the XY, XZ and YZ planes
 *          whose column (along z, y, x) holds a hit (the per-axis densities are those / 64).
 * Inputs: the primitives, and the pyramid they were voxelized into: leaf (vx_voxelize_*), out and
 * n_levels (vx_build_lod's, levels as there; n_levels[0] the leaf's count).  log2_res <= 17.
 * The pairs are regenerated by the candidate pipeline (max_cand / max_pairs as reported in
 * stats[VX_STAT_CAND] / stats[VX_STAT_PAIRS] of a call with 0).  A pair whose voxel the leaf lacks
 * sets VX_FLAG_OCC_LEAF (VX_ERR_BINDING); a level over its occupancy capacity sets
 * VX_FLAG_VOXEL_CAPACITY.  The result is exact and independent of scheduling.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  uint64_t* mask;     /* [8 * cap]: word w of voxel i at mask[w * cap + i] */
  uint16_t* hits;     /* [4 * cap]: hits[i] = hit sub-cells, hits[cap + i] = XY cells,
                         hits[2 cap + i] = XZ cells, hits[3 cap + i] = YZ cells */
  int64_t cap;        /* >= the level's voxel count */
} vx_occupancy;

/* kind 0 triangles, 1 fibers; 0 on bad arguments */
size_t vx_occupancy_workspace_size(int32_t kind, int64_t n_prims, int64_t max_cand, int64_t max_pairs,
                                   int32_t log2_res);

/* occ: host array of `levels` device descriptors (level 0 = leaf). */
vx_status vx_occupancy_triangles(const vx_grid* grid, const float* tris, int64_t n_tris, const vx_voxels* leaf,
                                 const vx_voxels* out, const int64_t* n_levels, int32_t levels, int64_t max_cand,
                                 int64_t max_pairs, const vx_occupancy* occ, void* workspace, size_t ws_bytes,
                                 int64_t* stats, vx_stream stream);

vx_status vx_occupancy_fibers(const vx_grid* grid, const float* pts, int64_t n_pts, const int64_t* offsets,
                              int64_t n_fibers, float radius, const vx_voxels* leaf, const vx_voxels* out,
                              const int64_t* n_levels, int32_t levels, int64_t max_cand, int64_t max_pairs,
                              const vx_occupancy* occ, void* workspace, size_t ws_bytes, int64_t* stats,
                              vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * LoD pyramid (Sec. 4.3-4.4).
 *
 * leaf: the voxelize output, with its count at n_leaf (device int64, e.g. &stats[VX_STAT_VOXELS]).
 * levels: total number of levels including the leaf, 1 .. log2_res + 1.
 * out: levels - 1 coarser levels (level L = 1 .. levels-1 at out[L-1]); each sums its 2x2x2
 *   children: keys = child >> 3, count, w and S summed, mask of present children.
 * K: lobes kept per coarse voxel (1 .. 8).  K == 1: `lobes` may be NULL (the level's S is the
 *   single lobe).  K > 1: lobes[L-1] receives, for each level-L voxel, at most K lobes merged
 *   from the lobes of its children (the leaf's lobe is the voxel itself): Ward agglomeration
 *   with cost w_a w_b / (w_a + w_b) * D(S_a / w_a, S_b / w_b),
 *   D(A, B) = 2 tr((A - B)^2) + (tr(A - B))^2, ties to the first pair in child/lobe order, then
 *   kmeans_iters weighted Lloyd passes (nearest centroid in D, ties to the lowest index),
 *   empty clusters dropped, lobes sorted by descending weight.
 * n_levels: int64[levels + 1] on the device; n_levels[L] = voxels at level L (clamped to the
 *   level's cap), n_levels[levels] = flags (VX_FLAG_VOXEL_CAPACITY when a level did not fit).
 * The workspace size depends on leaf->cap (vx_lod_workspace_size(leaf->cap, ...)).
 * ------------------------------------------------------------------------------------------ */
size_t vx_lod_workspace_size(int64_t cap, int32_t levels, int32_t K);

vx_status vx_build_lod(const vx_grid* grid, const vx_voxels* leaf, const int64_t* n_leaf, int32_t levels,
                       int32_t K, int32_t kmeans_iters, const vx_voxels* out, const vx_lobes* lobes,
                       int64_t* n_levels, void* workspace, size_t ws_bytes, const vx_tuning* tuning,
                       vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * vx_build_lod without a workspace, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * kernels and results as vx_build_lod; its scratch (the parent starts and scan partials) lives in
 * a library-owned device array of (VX_LOD_NOALLOC_MAX_LEAF + 1026) int64 (64 MiB) that each GPU
 * the library runs on holds until the process ends.  The call allocates nothing and frees
 * nothing.  leaf->cap above VX_LOD_NOALLOC_MAX_LEAF returns VX_ERR_CAPACITY before any launch.
 * Every call on one GPU shares that GPU's array and it keeps the last call's contents (nothing
 * in it needs to start at zero): calls that overlap on one GPU (other streams or threads)
 * race and must be serialised by the caller.
 * ------------------------------------------------------------------------------------------ */
#define VX_LOD_NOALLOC_MAX_LEAF 8388608

vx_status vx_build_lod_noalloc(const vx_grid* grid, const vx_voxels* leaf, const int64_t* n_leaf, int32_t levels,
                               int32_t K, int32_t kmeans_iters, const vx_voxels* out, const vx_lobes* lobes,
                               int64_t* n_levels, const vx_tuning* tuning, vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * Differentiable two-lobe fit (extension; the projected area of an SGGX lobe is Sec. 4.1's
 * sigma(omega) = sqrt(omega^T S omega)).
 *
 * For every voxel u of levels lo..hi (1 <= lo <= hi, hi <= 20) with w_u > 0, two lobes given by
 * lower-triangular 3x3 matrices L_1, L_2 (12 floats per voxel: L00 L10 L11 L20 L21 L22 of L_1,
 * then of L_2; L L^T is the lobe's SGGX matrix, PSD for any parameters) are fitted to u's
 * children:
 *   f_u(omega)   = |L_1^T omega| + |L_2^T omega|
 *   tau_u(omega) = sum_c sqrt(w_c omega^T S_c omega) / sum_c w_c   (children with w_c > 0)
 *   loss         = sum_{levels lo..hi} sum_u (1/ndir) sum_k (f_u(omega_k) - tau_u(omega_k))^2
 * levels: host array of hi + 1 level descriptors (leaf, then levels 1..hi of vx_build_lod with
 * K = 1); n_levels: their counts (device); params / dparams: host arrays of hi - lo + 1 device
 * pointers, level L at index L - lo, each [rows[L - lo]][12]; row r holds the lobes of the voxel at
 * index r of level L when the parameters were made.  rows: host int64 [hi - lo + 1], the row counts
 * of params (and dparams).  bound_keys: NULL, or a host array of hi - lo + 1 device pointers to the
 * keys (the level's key width, rows[L - lo] entries) that the rows were made for.  Every kernel stays
 * within the rows; a level whose device count differs from its rows sets VX_FLAG_FIT_ROWS and one
 * whose keys differ from bound_keys sets VX_FLAG_FIT_KEYS in stats[VX_STAT_FLAGS] (the loss and
 * gradients are then invalid; vx_check_stats reports VX_ERR_CAPACITY and VX_ERR_BINDING).
 * dirs: device float [ndir][3] unit directions, 1 <= ndir <= 256; caps: host int64 [hi + 1], the
 * capacities of levels 0..hi.
 * The gradient to the control points flows through the leaf sums: the clipped centreline
 * lengths (weights) and the tangents (moments I - t t^T) of the segments, evaluated at the
 * lattice-snapped points; the voxel sets are held fixed (the loss is piecewise smooth).  The
 * backward pass differentiates at FP64 sums of levels 0..hi-1, which it forms itself from the
 * re-emitted (segment, voxel) pairs (each voxel's pairs added in primitive order).
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  const float* pts;          /* device float [n_pts][3] */
  int64_t n_pts;
  const int64_t* offsets;    /* device int64 [n_fibers + 1] */
  int64_t n_fibers;
  float radius;
} vx_fibers;

size_t vx_fit_workspace_size(int64_t n_pts, int64_t max_cand, int64_t max_pairs, const int64_t* caps, int32_t hi,
                             int32_t log2_res);

/* loss: device float [1], overwritten.  stats: device int64 [VX_NSTAT], overwritten (flags only). */
vx_status vx_fit_forward(const vx_grid* grid, const vx_voxels* levels, const int64_t* n_levels, int32_t lo,
                         int32_t hi, const float* const* params, const int64_t* rows, const void* const* bound_keys,
                         const float* dirs, int32_t ndir, float* loss, int64_t* stats, const int64_t* caps,
                         void* workspace, size_t ws_bytes, vx_stream stream);

/* dloss: device float [1] (upstream gradient); dpts: device float [n_pts][3], overwritten;
 * stats: device int64 [VX_NSTAT] for the re-emitted pairs and the binding flags.  max_cand /
 * max_pairs: capacities of the candidate space and of the (primitive, voxel) pairs, which the
 * backward pass lists per primitive (at least stats[VX_STAT_CAND] / stats[VX_STAT_PAIRS] of
 * vx_voxelize_fibers on the same fibers; pairs at most 2^31 - 1). */
vx_status vx_fit_backward(const vx_grid* grid, const vx_fibers* fibers, int64_t max_cand, int64_t max_pairs,
                          const vx_voxels* levels, const int64_t* n_levels, int32_t lo, int32_t hi,
                          const float* const* params, const int64_t* rows, const void* const* bound_keys,
                          const float* dirs, int32_t ndir, const float* dloss, float* const* dparams, float* dpts,
                          int64_t* stats, const int64_t* caps, void* workspace, size_t ws_bytes, vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * Batched fiber patches (extension): many patches of uneven size and resolution voxelized and
 * LoD-built together, by the same kernels as one instance, with one pass over all primitives.
 *
 * Every patch has its own cubic grid (log2_res <= 11) and radius; its points are the range
 * [pt_begin, pt_end) of the shared point array and its fibers must not cross that range.  Keys
 * are 64-bit: (patch << 33) | Morton code, and a parent keeps its patch bits:
 * parent(k) = (k & ~(2^33 - 1)) | ((k & (2^33 - 1)) >> 3).  Patch p's voxels of a level are the
 * contiguous range [patch_table[L][p], patch_table[L][p + 1]).  A patch whose own pyramid is
 * shorter than `levels` keeps its root voxel on the levels above it.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  vx_grid grid;
  int64_t pt_begin;
  int64_t pt_end;
  float radius;
  int32_t reserved;
} vx_patch;

size_t vx_batch_workspace_size(int32_t n_patches, int64_t n_pts, int64_t max_records, int64_t max_units,
                               int64_t leaf_cap);

/* patches: host array (validated) and the same array in device memory (read by the kernels);
 * pts / offsets: device, all patches concatenated (offsets global over all fibers);
 * out: host array of `levels` level descriptors, leaf first (out[0].mask may be NULL);
 * lobes: host array of levels - 1 descriptors when K > 1, else NULL;
 * n_levels: device int64 [levels + 1] (counts, then flags); patch_table: device int64
 * [levels][n_patches + 1]; stats: device int64 [VX_NSTAT] (totals and flags);
 * max_records / max_units / out[0].cap: as for vx_voxelize_fibers, over the whole batch. */
vx_status vx_batch_build(const vx_patch* patches, const vx_patch* patches_dev, int32_t n_patches, const float* pts,
                         int64_t n_pts, const int64_t* offsets, int64_t n_fibers, int32_t levels, int32_t K,
                         int32_t kmeans_iters, int64_t max_records, int64_t max_units, const vx_voxels* out,
                         const vx_lobes* lobes, int64_t* n_levels, int64_t* patch_table, int64_t* stats,
                         void* workspace, size_t ws_bytes, const vx_tuning* tuning, vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * Leaf eigen-fit and compact SGGX storage (Sec. 4.1 "Fitting to SGGX distribution"; Sec. 4.3
 * "Storing data", the compact-SGGX equation).
 *
 * For voxel i < min(*n_vox, vox->cap) with w_i > 0: M = S_i / w_i is diagonalised in FP64
 * (eigenvalues lambda_1 >= lambda_2 >= lambda_3, the projected areas along the eigenvectors;
 * each eigenvector of unit length with its largest-magnitude component positive), the
 * eigenvalues are floored at eps * lambda_1 (a voxel of nearly one orientation still gets a
 * well-defined SGGX), and the SGGX is rebuilt as sum_i lambda_i e_i e_i^T.  Voxels with
 * w_i <= 0 (or M = 0) get the identity.  The rebuilt matrix, scaled so that its largest
 * diagonal entry is 1, is stored in 6 bytes: sigma_a = sqrt(S_aa) as rint(255 sigma_a) for
 * a = x, y, z, then r_ab = S_ab / sqrt(S_aa S_bb) as 128 + rint(127 r_ab) for xy, xz, yz.
 *
 * vox: the level (only w, S and cap are read); n_vox: device int64 [1];
 * eps: in (0, 1]; lam: device float [3 * cap], lam[k * cap + i] (NULL: not written);
 * vec: device float [9 * cap], component c of eigenvector k at vec[(3k + c) * cap + i]
 * (NULL: not written); code: device uint8 [6 * cap], 2-byte aligned, voxel i at
 * code[6i .. 6i + 5].  Entries i >= n are untouched.  Returns VX_ERR_ARG on a NULL
 * required pointer, cap < 1, eps outside (0, 1] or a misaligned code; VX_ERR_HIP if the
 * launch fails.  Asynchronous on `stream`.
 * ------------------------------------------------------------------------------------------ */
vx_status vx_sggx_compact(const vx_voxels* vox, const int64_t* n_vox, float eps, float* lam, float* vec,
                          uint8_t* code, vx_stream stream);

/* Inverse of the byte code: sigma = b / 255, r = (b - 128) / 127, S_aa = sigma_a^2,
 * S_ab = r_ab sigma_a sigma_b (FP64, rounded once to float).  code: device uint8 [6 * cap]
 * (2-byte aligned); n: device int64 [1]; S: device float [6 * cap], S[c * cap + i] with
 * c = xx, yy, zz, xy, xz, yz.  Errors as for vx_sggx_compact. */
vx_status vx_sggx_decode(const uint8_t* code, const int64_t* n, int64_t cap, float* S, vx_stream stream);

/* ------------------------------------------------------------------------------------------
 * Graph capture of a whole call (no host work inside, so it replays as one launch).  `stream`
 * must not be the null stream.  Between begin and end, enqueue library calls on `stream`;
 * vx_graph_launch replays them (with the buffers and sizes of the capture).
 * ------------------------------------------------------------------------------------------ */
typedef struct vx_graph_s* vx_graph;
vx_status vx_graph_begin(vx_stream stream);
vx_status vx_graph_end(vx_stream stream, vx_graph* graph);
vx_status vx_graph_launch(vx_graph graph, vx_stream stream);
void vx_graph_destroy(vx_graph graph);

/* Synchronises `stream`, reads stats (VX_NSTAT int64 on the device) and maps its flags to a
 * status: VX_ERR_INPUT before VX_ERR_BINDING before VX_ERR_CAPACITY before VX_OK. */
vx_status vx_check_stats(const int64_t* stats, vx_stream stream);

const char* vx_status_str(vx_status s);

/* Kernel timing for measurement: when enabled, every kernel launch of the library is
 * bracketed by HIP events on the caller's stream and its duration is accumulated per kernel
 * name once vx_timing_collect() (which synchronises the device) is called. */
void vx_timing_enable(int32_t on);
void vx_timing_reset(void);
/* Restricts timing to launches of one kernel name (NULL or "": every launch), so that a timed
 * region carries events only around the kernel being measured. */
void vx_timing_filter(const char* name);
/* Writes up to max_entries (name, total ms, launches) triples; returns the number of kernels. */
int32_t vx_timing_collect(char names[][48], double* total_ms, int64_t* launches, int32_t max_entries);

#ifdef __cplusplus
}
#endif
#endif /* VX_H */
