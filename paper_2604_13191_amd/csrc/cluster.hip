// cluster.hip -- Sec. 4.4: per coarse voxel, merge the lobes of its children down to at most K.
//
// The paper builds a dendrogram by repeatedly merging the two most similar SGGX lobes of a
// voxel's set (its similarity compares the distributions, not the parameters).  Here the
// similarity is the L2 distance between the lobes' projected-area-squared functions,
// D(A, B) = 2 tr((A - B)^2) + (tr(A - B))^2 for normalised lobes A = S_a / w_a, and merging
// follows Ward's rule (least w_a w_b / (w_a + w_b) * D, ties to the first pair), then a few
// weighted Lloyd passes refine the K clusters.  Merging is additive: (w_a + w_b, S_a + S_b).
//
// Mapping: a group of G lanes (G = 8 at level 1, 8K rounded up to a power of two above)
// handles one parent voxel; lane m holds input lobe m; the cluster sums and the pairwise cost
// matrix live in the group's LDS.  Every reduction has a fixed order (butterflies for the
// argmin, member-order sums for the Lloyd centroids): the result is deterministic.
#include "vx_internal.hpp"

namespace vx {

// D between two normalised lobes a = S_a / w_a, b = S_b / w_b
__device__ __forceinline__ float lobe_dist_n(const float* a, const float* b) {
  float d[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) d[j] = a[j] - b[j];
  const float tr = d[0] + d[1] + d[2];
  const float t2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 2.0f * (d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
  return 2.0f * t2 + tr * tr;
}

// Ward's merge cost w_a w_b / (w_a + w_b) D (reciprocals to 1 ulp)
__device__ __forceinline__ float ward_cost(float wa, float wb, const float* na, const float* nb) {
  return wa * wb * __builtin_amdgcn_rcpf(wa + wb) * lobe_dist_n(na, nb);
}

template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int gi) {
  if (G == 64) return ballot;
  return (ballot >> (gi * G)) & ((uint64_t(1) << G) - 1);
}

// minimum of a 64-bit key over the G lanes of a group: DPP within rows of 16 (xor 1 and 2 by
// quad permutes, then the half-row and row mirrors, each pairing every lane with a partner of
// the other half), then cross-row exchanges for G = 32 and 64
__device__ __forceinline__ uint64_t dpp_min_u64(uint64_t v, int ctrl_tag) {
  const int lo = int(uint32_t(v)), hi = int(uint32_t(v >> 32));
  int olo, ohi;
  switch (ctrl_tag) {
    case 0:
      olo = __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false);
      ohi = __builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 1:
      olo = __builtin_amdgcn_update_dpp(lo, lo, 0x4E, 0xF, 0xF, false);
      ohi = __builtin_amdgcn_update_dpp(hi, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 2:
      olo = __builtin_amdgcn_update_dpp(lo, lo, 0x141, 0xF, 0xF, false);
      ohi = __builtin_amdgcn_update_dpp(hi, hi, 0x141, 0xF, 0xF, false);
      break;
    default:
      olo = __builtin_amdgcn_update_dpp(lo, lo, 0x140, 0xF, 0xF, false);
      ohi = __builtin_amdgcn_update_dpp(hi, hi, 0x140, 0xF, 0xF, false);
      break;
  }
  const uint64_t o = (uint64_t(uint32_t(ohi)) << 32) | uint32_t(olo);
  return o < v ? o : v;
}

template <int G>
__device__ __forceinline__ uint64_t group_min_u64(uint64_t v) {
  v = dpp_min_u64(v, 0);
  v = dpp_min_u64(v, 1);
  if (G > 4) v = dpp_min_u64(v, 2);
  if (G > 8) v = dpp_min_u64(v, 3);
  if (G > 16) {
    const uint64_t o = uint64_t(__shfl_xor((unsigned long long)v, 16, 64));
    v = o < v ? o : v;
  }
  if (G > 32) {
    const uint64_t o = uint64_t(__shfl_xor((unsigned long long)v, 32, 64));
    v = o < v ? o : v;
  }
  return v;
}

template <int G>
struct ClusterLds {
  float lw[64 / G][G];
  float lS[64 / G][6][G];
  float cw[64 / G][G];
  float cS[64 / G][6][G];
  float nS[64 / G][6][G];     // cluster lobes normalised by their weight
  float mat[64 / G][G][G + 1];   // [j][g]: row g's cost to column j (rows padded: no bank clashes)
  int asg[64 / G][G];
};

// One round of one wave: group gi (gi < 64 / G) takes parent p (when live) of a level whose children
// [pstart[p], pstart[p+1]) in the level below carry lobes cw[k * cap_c + c] and
// cS[(j * Kc + k) * cap_c + c] (cnl == nullptr: one lobe per child, present when its weight is
// positive).
// BAND: parents that gather more than G lobes are left to a wider pass, and (LO > 0) those that
// gather at most LO to an earlier, narrower one; with LO = 0 this pass also writes the parents
// that gather no lobe.
template <int G, bool BAND = false, int LO = 0, int SLOTS = 64>
__device__ __forceinline__ void cluster_round(int64_t p, bool live, const int64_t* __restrict__ pstart,
                                              const float* __restrict__ cw, const float* __restrict__ cS,
                                              const uint8_t* __restrict__ cnl, int Kc, int64_t cap_c, int K,
                                              int iters, const vx_lobes& out, ClusterLds<G>& L) {
  const int lane = lane_id();
  const int g = lane % G, gi = lane / G;
  const int64_t cap = out.cap;
  // ---- gather the children's lobes in canonical order (child, then lobe), compacted to lanes
  // 0..n-1.  Lane g takes slots g, g + G, ... of the 8 Kc (child, lobe) slots; n <= G is the
  // caller's guarantee (G >= 8 Kc, or a parent known to gather at most G lobes).
  // All of this lane's slots are loaded first (the weight and moment together with the lobe
  // count, all in bounds whatever the count), then compacted in slot order: one round of
  // dependent loads after the parent's child range instead of one chain per slot.
  const int slots = 8 * Kc;
  constexpr int R = (SLOTS + G - 1) / G;           // slots per lane at most (8 Kc <= SLOTS)
  int64_t cs = 0, ce = 0;
  if (live) {
    cs = pstart[p];
    ce = pstart[p + 1];
  }
  float rw[R], rS[R][6];
  bool rv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int slot = r * G + g;
    rw[r] = 0.f;
    rv[r] = false;
#pragma unroll
    for (int j = 0; j < 6; ++j) rS[r][j] = 0.f;
    if (live && slot < slots) {
      const int ch = slot / Kc, k = slot % Kc;
      const int64_t c = cs + ch;
      if (c < ce) {
        const int nl = cnl ? int(cnl[c]) : 1;
        rw[r] = cw[int64_t(k) * cap_c + c];
#pragma unroll
        for (int j = 0; j < 6; ++j) rS[r][j] = cS[(int64_t(j) * Kc + k) * cap_c + c];
        rv[r] = k < nl && rw[r] > 0.f;
      }
    }
  }
  int n = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t vm = group_bits<G>(__ballot(rv[r]), gi);
    const int m = n + __popcll(vm & ((uint64_t(1) << g) - 1));
    if (rv[r] && m < G) {
      L.lw[gi][m] = rw[r];
#pragma unroll
      for (int j = 0; j < 6; ++j) L.lS[gi][j][m] = rS[r][j];
    }
    n += __popcll(vm);
  }
  if (BAND && (n > G || (LO > 0 && n <= LO))) {
    live = false;                                  // another pass takes this parent
    n = 0;
  }
  n = n < G ? n : G;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const bool mine = g < n;
  float lw = 0.f, lS[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, ln[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (mine) {
    lw = L.lw[gi][g];
    const float il = __builtin_amdgcn_rcpf(lw);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      lS[j] = L.lS[gi][j][g];
      ln[j] = lS[j] * il;
    }
    L.cw[gi][g] = lw;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      L.cS[gi][j][g] = lS[j];
      L.nS[gi][j][g] = ln[j];
    }
  }
  uint64_t act = n == 64 ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
  int cl = g;                                      // the cluster that input lobe g belongs to
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  if (n > K) {
    if constexpr (G <= 8) {
      // ---- Ward agglomeration, few lobes per voxel (G <= 8): clusters and the upper triangle
      // of the cost matrix in LDS, row g written by lane g
      if (mine) {
        for (int j = g + 1; j < n; ++j) {
          float b[6];
#pragma unroll
          for (int t = 0; t < 6; ++t) b[t] = L.nS[gi][t][j];
          L.mat[gi][g][j] = ward_cost(lw, L.cw[gi][j], ln, b);
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      // Each lane caches the minimum of its row (least cost, then least column); a merge of
      // (bi, bj) only invalidates rows whose cached column was bi or bj, and row bi itself.
      float best = INFINITY;
      int bjr = G;
      auto scan_row = [&]() {
        best = INFINITY;
        bjr = G;
        if (mine && ((act >> g) & 1)) {
          for (int j = g + 1; j < n; ++j) {
            if (!((act >> j) & 1)) continue;
            const float c = L.mat[gi][g][j];
            if (c < best) { best = c; bjr = j; }
          }
        }
      };
      scan_row();
      for (int step = n; step > K; --step) {
        // group argmin of (cost, i); the row minimum already carries the smallest j.  Costs are
        // non-negative, so their bits order like the values: one 64-bit key (cost, i, j).
        const uint64_t key = (uint64_t(__float_as_uint(best)) << 32) | (uint64_t(bjr < G ? g : G) << 16) |
                             uint64_t(bjr);
        const uint64_t kmin = group_min_u64<G>(key);
        const int bi = int((kmin >> 16) & 0xffff), bj = int(kmin & 0xffff);
        if (bj < G && cl == bj) cl = bi;
        // merge cluster bj into bi
        if (g == bi && bj < G) {
          const float nw = L.cw[gi][bi] + L.cw[gi][bj];
          const float inw = __builtin_amdgcn_rcpf(nw);
          L.cw[gi][bi] = nw;
#pragma unroll
          for (int t = 0; t < 6; ++t) {
            const float v = L.cS[gi][t][bi] + L.cS[gi][t][bj];
            L.cS[gi][t][bi] = v;
            L.nS[gi][t][bi] = v * inw;
          }
        }
        if (bj < G) act &= ~(uint64_t(1) << bj);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        float cnew = INFINITY;
        if (bj < G && mine && ((act >> g) & 1) && g != bi) {
          float a[6], b[6];
#pragma unroll
          for (int t = 0; t < 6; ++t) { a[t] = L.nS[gi][t][bi]; b[t] = L.nS[gi][t][g]; }
          cnew = ward_cost(L.cw[gi][bi], L.cw[gi][g], a, b);
          if (g < bi) L.mat[gi][g][bi] = cnew; else L.mat[gi][bi][g] = cnew;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // refresh the cached row minima
        if (g == bj) {
          best = INFINITY;
          bjr = G;
        } else if (g == bi || bjr == bi || bjr == bj) {
          scan_row();
        } else if (g < bi && mine && ((act >> g) & 1)) {
          if (cnew < best || (cnew == best && bi < bjr)) { best = cnew; bjr = bi; }
        }
      }
    } else {
      // ---- Ward agglomeration.  Lane g holds cluster g (weight, sums, normalised sums) in
      // registers and row g of the symmetric cost matrix in LDS; a dead cluster costs +inf.
      float cw = lw, cS[6], nS[6];
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        cS[t] = lS[t];
        nS[t] = ln[t];
      }
      // Each lane caches the minimum of its row (least cost, then least column).
      float best = INFINITY;
      int bjr = G;
      if (mine) {
        for (int j = 0; j < n; ++j) {
          float c = INFINITY;
          if (j != g) {
            float b[6];
#pragma unroll
            for (int t = 0; t < 6; ++t) b[t] = L.nS[gi][t][j];
            c = ward_cost(lw, L.cw[gi][j], ln, b);
          }
          L.mat[gi][j][g] = c;
          if (c < best) {
            best = c;
            bjr = j;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const int base = lane - g;                  // the group's first lane
      for (int step = n; step > K; --step) {
        // group argmin of the cached row minima as one 64-bit key (cost, i, j), i < j: costs
        // are non-negative, so their bits order like the values, and the least key is the
        // first pair in (i, j) order among the least costs
        const int lo = g < bjr ? g : bjr, hi = g < bjr ? bjr : g;
        const uint64_t key = bjr < G ? (uint64_t(__float_as_uint(best)) << 32) | (uint64_t(lo) << 16) | uint64_t(hi)
                                     : ~uint64_t(0);
        const uint64_t kmin = group_min_u64<G>(key);
        const int bi = int((kmin >> 16) & 0xffff), bj = int(kmin & 0xffff);
        const bool merge = bj < G;
        if (merge && cl == bj) cl = bi;
        // the merged cluster (bi absorbs bj), computed by every lane from the two lanes' registers
        const int si = base + (merge ? bi : 0), sj = base + (merge ? bj : 0);
        const float mw = __shfl(cw, si, 64) + __shfl(cw, sj, 64);
        const float inw = __builtin_amdgcn_rcpf(mw);
        float mS[6], mn[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          mS[t] = __shfl(cS[t], si, 64) + __shfl(cS[t], sj, 64);
          mn[t] = mS[t] * inw;
        }
        if (merge) {
          act &= ~(uint64_t(1) << bj);
          if (g == bi) {
            cw = mw;
#pragma unroll
            for (int t = 0; t < 6; ++t) {
              cS[t] = mS[t];
              nS[t] = mn[t];
            }
          }
        }
        const bool alive = mine && ((act >> g) & 1);
        float cnew = INFINITY;
        if (merge && alive && g != bi) {
          cnew = ward_cost(mw, cw, mn, nS);
          L.mat[gi][bi][g] = cnew;                // row g, column bi
          L.mat[gi][g][bi] = cnew;                // row bi, column g
        }
        if (merge && mine) L.mat[gi][bj][g] = INFINITY;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // the merged row's minimum over the new costs (least cost, then least column)
        const uint64_t k2 = (uint64_t(__float_as_uint(cnew)) << 32) | uint64_t(g);
        const uint64_t m2 = group_min_u64<G>(k2);
        // refresh the cached row minima: only column bi changed (to cnew) and column bj died.
        // Row bj dies, row bi takes the merged row's minimum; a row whose minimum sat in column bi
        // keeps it if the new cost is no larger, else (or if it sat in column bj) is rescanned;
        // any other row compares the new cost with its minimum (ties to the lower column).  All
        // decided with selects, no branch per case.
        const bool isj = merge && g == bj;
        const bool isi = merge && !isj && g == bi;
        const bool oth = merge && !isj && !isi && alive;
        const bool onbi = oth && bjr == bi, onbj = oth && !onbi && bjr == bj;
        const bool keep_bi = onbi && cnew <= best;
        const bool rescan = (onbi && !(cnew <= best)) || onbj;
        const bool take_new = oth && !onbi && !onbj && (cnew < best || (cnew == best && bi < bjr));
        const float mb = __uint_as_float(uint32_t(m2 >> 32));
        const int mj = mb < INFINITY ? int(m2 & 0xffff) : G;
        best = isj ? INFINITY : (isi ? mb : ((keep_bi || take_new) ? cnew : best));
        bjr = isj ? G : (isi ? mj : (take_new ? bi : bjr));
        if (rescan) {
          best = INFINITY;
          bjr = G;
          if constexpr (G <= 16) {
            // the whole row, its loads issued together (unrolled over the group width; every
            // column is in bounds, those at or past n are replaced by +inf)
            float c[G];
#pragma unroll
            for (int j = 0; j < G; ++j) c[j] = L.mat[gi][j][g];
#pragma unroll
            for (int j = 0; j < G; ++j) c[j] = j < n ? c[j] : INFINITY;
#pragma unroll
            for (int j = 0; j < G; ++j)
              if (c[j] < best) {
                best = c[j];
                bjr = j;
              }
          } else {
            for (int j = 0; j < n; ++j) {
              const float c = L.mat[gi][j][g];
              if (c < best) {
                best = c;
                bjr = j;
              }
            }
          }
        }
      }
      // the clusters back to LDS for the Lloyd passes and the output
      if (mine) {
        L.cw[gi][g] = cw;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
          L.cS[gi][t][g] = cS[t];
          L.nS[gi][t][g] = nS[t];
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    // ---- weighted Lloyd passes over the original lobes.  A pass that moves no lobe to another
    // cluster leaves every cluster as it is, and so does every later one: the group stops there.
    bool conv = false;                             // uniform over the group
    for (int it = 0; it < iters; ++it) {
      int assign = -1;
      if (mine) {
        // nearest active centroid (ties to the lowest index), walking the active set
        float bestd = INFINITY;
        for (uint64_t m = act; m; m &= m - 1) {
          const int k = __ffsll((unsigned long long)m) - 1;
          float b[6];
#pragma unroll
          for (int t = 0; t < 6; ++t) b[t] = L.nS[gi][t][k];
          const float d = lobe_dist_n(ln, b);
          if (d < bestd) { bestd = d; assign = k; }
        }
      }
      conv = group_bits<G>(__ballot(mine && assign != cl), gi) == 0;
      if (__ballot(!conv) == 0) break;             // every group of the wave has converged
      if (conv) continue;
      cl = assign;
      if (mine) L.asg[gi][g] = assign;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      // new cluster sums: one lane per (active cluster, component), adding the members in
      // lobe order (sequential, so the sums are fixed)
      const int na = __popcll(act);
      for (int q = g; q < 7 * na; q += G) {
        const int r = q / 7, t = q - 7 * r;
        uint64_t m = act;
        for (int i = 0; i < r; ++i) m &= m - 1;
        const int k = __ffsll((unsigned long long)m) - 1;
        // the members in lobe order (narrow groups: every member's load issued before the sum)
        float sum = 0.f;
        if constexpr (G <= 16) {
          float v[G];
          bool in[G];
#pragma unroll
          for (int mm = 0; mm < G; ++mm) {
            in[mm] = mm < n && L.asg[gi][mm] == k;
            v[mm] = in[mm] ? (t == 6 ? L.lw[gi][mm] : L.lS[gi][t][mm]) : 0.f;
          }
#pragma unroll
          for (int mm = 0; mm < G; ++mm)
            if (in[mm]) sum += v[mm];
        } else {
          for (int mm = 0; mm < n; ++mm)
            if (L.asg[gi][mm] == k) sum += t == 6 ? L.lw[gi][mm] : L.lS[gi][t][mm];
        }
        if (t == 6) L.cw[gi][k] = sum;
        else L.cS[gi][t][k] = sum;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      uint64_t nact = 0;
      for (uint64_t m = act; m; m &= m - 1) {
        const int k = __ffsll((unsigned long long)m) - 1;
        if (L.cw[gi][k] > 0.f) nact |= uint64_t(1) << k;
      }
      act = nact;
      // the new centroids, normalised
      for (int q = g; q < 6 * na; q += G) {
        const int r = q / 6, t = q - 6 * r;
        uint64_t m = nact;
        for (int i = 0; i < r && m; ++i) m &= m - 1;
        if (!m) continue;
        const int k = __ffsll((unsigned long long)m) - 1;
        L.nS[gi][t][k] = L.cS[gi][t][k] * __builtin_amdgcn_rcpf(L.cw[gi][k]);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  }
  // ---- output: active clusters sorted by descending weight (ties keep cluster order)
  if (live) {
    const int nl = __popcll(act);
    if (g < G && ((act >> g) & 1)) {
      const float wg = L.cw[gi][g];
      int rank = 0;
      for (int k = 0; k < n; ++k) {
        if (!((act >> k) & 1) || k == g) continue;
        const float wk = L.cw[gi][k];
        rank += (wk > wg || (wk == wg && k < g)) ? 1 : 0;
      }
      if (rank < K) {                             // at most K clusters remain; never write past them
        out.w[int64_t(rank) * cap + p] = wg;
#pragma unroll
        for (int t = 0; t < 6; ++t) out.S[(int64_t(t) * K + rank) * cap + p] = L.cS[gi][t][g];
      }
    }
    if (g >= nl && g < K) {
      out.w[int64_t(g) * cap + p] = 0.f;
#pragma unroll
      for (int t = 0; t < 6; ++t) out.S[(int64_t(t) * K + g) * cap + p] = 0.f;
    }
    if (g == 0) out.nl[p] = uint8_t(nl);
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// One level with a fixed group width G (G lanes per parent, 64 / G parents per wave).  With
// BAND, only the parents that gather more than LO and at most G lobes are taken.
template <int G, bool BAND, int LO = 0, int SLOTS = 64>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SLOTS <= 32 ? 4 : 3))) k_cluster(const int64_t* __restrict__ pstart, const int64_t* n_par_ptr,
                                                    const float* __restrict__ cw, const float* __restrict__ cS,
                                                    const uint8_t* __restrict__ cnl, int Kc, int64_t cap_c, int K,
                                                    int iters, vx_lobes out) {
  __shared__ ClusterLds<G> sm[kWaves];
  ClusterLds<G>& L = sm[threadIdx.x >> 6];
  const int64_t n_par = *n_par_ptr;
  constexpr int per_wave = 64 / G;
  const int64_t w0 = (int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6)) * per_wave;
  const int64_t stride = int64_t(gridDim.x) * kWaves * per_wave;
  for (int64_t base = w0; base < n_par; base += stride)
    cluster_round<G, BAND, LO, SLOTS>(base + threadIdx.x % 64 / G, base + threadIdx.x % 64 / G < n_par, pstart, cw,
                                      cS, cnl, Kc, cap_c, K, iters, out, L);
}

// Parents picked by a count, GB lanes each: a wave counts up to 64 parents' (child, lobe) slots
// in use (one parent per lane), then serves those whose count lies in (QLO, QHI], 64 / GB at a
// time.  A wave counts as many parents as spread the level over the grid, at least one round's
// worth: a small level runs one round per wave, all in parallel.
// Without BAND the count bounds the lobes (QHI <= GB); with BAND the round takes a parent only
// when its positive lobes are more than LO and at most GB (the other picks take the rest).
// When few parents are in the band this pass is mostly the count.  The group width changes no
// result.
constexpr int kAnyCount = 1 << 30;
template <int GB, bool BAND, int LO, int QLO, int QHI, int SLOTS>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(GB <= 16 && SLOTS <= 32 ? 4 : 1))) k_cluster_pick(const int64_t* __restrict__ pstart,
                                                         const int64_t* n_par_ptr, const float* __restrict__ cw,
                                                         const float* __restrict__ cS,
                                                         const uint8_t* __restrict__ cnl, int Kc, int64_t cap_c,
                                                         int K, int iters, vx_lobes out) {
  __shared__ ClusterLds<GB> sm[kWaves];
  ClusterLds<GB>& L = sm[threadIdx.x >> 6];
  const int lane = lane_id();
  constexpr int per_r = 64 / GB;                  // parents served per round
  const int gi = lane / GB;
  const int64_t n_par = *n_par_ptr;
  const int64_t waves = int64_t(gridDim.x) * kWaves;
  int64_t per = (n_par + waves - 1) / waves;      // parents counted per wave (uniform)
  per = per < per_r ? per_r : (per > 64 ? 64 : per);
  const int64_t w0 = (int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6)) * per;
  const int64_t stride = waves * per;
  for (int64_t base = w0; base < n_par; base += stride) {
    int nq = 0;
    const int64_t p = base + lane;
    const bool counted = lane < per && p < n_par;
    if (counted) {
      const int64_t cs = pstart[p], ce = pstart[p + 1];
      for (int64_t c = cs; c < ce; ++c) nq += cnl ? (int(cnl[c]) < Kc ? int(cnl[c]) : Kc) : 1;
    }
    static_assert(BAND || QHI <= GB, "without the band check the count must bound the lobes");
    uint64_t m = __ballot(counted && nq > QLO && nq <= QHI);
    while (m) {
      int64_t mine = -1;
#pragma unroll
      for (int k = 0; k < per_r; ++k) {
        if (m) {
          if (k == gi) mine = base + (__ffsll((unsigned long long)m) - 1);
          m &= m - 1;
        }
      }
      // the count includes lobes of zero weight: the round takes a parent only when its positive
      // lobes fall in the band (a narrower pass took fewer, a wider one takes more)
      cluster_round<GB, BAND, LO, SLOTS>(mine < 0 ? 0 : mine, mine >= 0, pstart, cw, cS, cnl, Kc, cap_c, K, iters,
                                         out, L);
    }
  }
}

void cluster_level(const int64_t* pstart, const int64_t* n_par, const float* cw, const float* cS, const uint8_t* cnl,
                   int Kc, int64_t cap_c, int K, int iters, const vx_lobes& out, int grid, hipStream_t s,
                   bool narrow_first) {
  const int need = 8 * Kc;
  // no more blocks than the level's capacity of parents can use (the upper levels are small)
  auto blocks = [&](int per_block) {
    const int64_t b = (out.cap + per_block - 1) / per_block;
    return int(b < grid ? (b < 1 ? 1 : b) : grid);
  };
  // timing names by group width: the first level (one lobe per child) and the levels above
  VX_TIMED(need <= 8 ? "lod_cluster" : "lod_cluster_up", s);
  if (need <= 8)
    hipLaunchKernelGGL((k_cluster<8, false, 0, 8>), dim3(blocks(kWaves * 8)), dim3(kBlock), 0, s, pstart, n_par, cw,
                       cS, cnl, Kc, cap_c, K, iters, out);
  else if (need <= 16)
    hipLaunchKernelGGL((k_cluster<16, false, 0, 16>), dim3(blocks(kWaves * 4)), dim3(kBlock), 0, s, pstart, n_par, cw,
                       cS, cnl, Kc, cap_c, K, iters, out);
  else {
    // parents by the lobes they gather: at most 16 positive lobes at four parents per wave (all
    // parents gathered), 17 to 32 at two and the few above at one (picked after a count).  With
    // narrow_first (the level above the first, whose children hold few lobes: many parents gather
    // at most 8) those with at most 8 slots filled go first at eight per wave, then the others
    // with at most 16 positive lobes at four, each picked after a count.
    const int pgrid = blocks(kWaves * 64) < (grid / 4 > 64 ? grid / 4 : 64) ? blocks(kWaves * 64)
                                                                            : (grid / 4 > 64 ? grid / 4 : 64);
    const int mgrid = blocks(kWaves * 64 / 4);
#define VX_PICK(GRID, GB, BAND, LO, QLO, QHI, SL)                                                                  \
  hipLaunchKernelGGL((k_cluster_pick<GB, BAND, LO, QLO, QHI, SL>), dim3(GRID), dim3(kBlock), 0, s, pstart, n_par, cw, \
                     cS, cnl, Kc, cap_c, K, iters, out)
    if (need <= 32) {
      if (narrow_first) {
        VX_PICK(mgrid, 8, false, 0, -1, 8, 32);
        VX_PICK(mgrid, 16, true, 0, 8, kAnyCount, 32);
      } else {
        hipLaunchKernelGGL((k_cluster<16, true, 0, 32>), dim3(blocks(kWaves * 4)), dim3(kBlock), 0, s, pstart, n_par,
                           cw, cS, cnl, Kc, cap_c, K, iters, out);
      }
      VX_PICK(pgrid, 32, true, 16, 16, kAnyCount, 32);
    } else {
      if (narrow_first) {
        VX_PICK(mgrid, 8, false, 0, -1, 8, 64);
        VX_PICK(mgrid, 16, true, 0, 8, kAnyCount, 64);
      } else {
        hipLaunchKernelGGL((k_cluster<16, true, 0, 64>), dim3(blocks(kWaves * 4)), dim3(kBlock), 0, s, pstart, n_par,
                           cw, cS, cnl, Kc, cap_c, K, iters, out);
      }
      VX_PICK(pgrid, 32, true, 16, 16, kAnyCount, 64);
      VX_PICK(pgrid, 64, true, 32, 32, kAnyCount, 64);
    }
#undef VX_PICK
  }
}

}  // namespace vx
