// Hub path of the sweep: vertices whose degree exceeds the largest LDS bin.
//
// A hub's scan (scanCommunities of Algorithm 1) is spread over many
// workgroups without any table in HBM:
//   k_hub_plan_*  per flagged hub: work items (chunks, label partitions,
//                 merge groups) and their numbering in the step;
//   k_hub_owner   work item -> hub maps;
//   k_hub_chunk   per chunk of HUB_CHUNK entries: gather the neighbour
//                 labels, merge equal labels in an LDS table, and append the
//                 merged (label, weight) pairs to the hub's label partitions;
//   k_hub_part    per group of a hub's partitions: merge the pairs in LDS
//                 (the whole group at once when it holds few pairs) and keep
//                 the heaviest label (smallest id on ties);
//   k_hub_decide  per hub: best over the partitions, update, clear the
//                 partition counters;
//   k_hub_mark    per chunk of a hub that changed: flag the neighbours;
//   k_hub_finish  both in one kernel, per chunk (each chunk re-reads the
//                 hub's partition maxima: for steps with little hub work).
// Every label falls in exactly one partition, so the per-partition maxima
// combine into the strict argmax of Eq. (2).
#include "sweep_kernels.hpp"
#include "tables.hpp"

namespace gvelpa {

// Ordinal of vertex v among the sorted hub ids, -1 if it is no hub.  In
// degree order the hubs are the first n_hubs positions (ids[k] == k) and the
// ordinal is v itself; otherwise a binary search over the ids.
__device__ __forceinline__ int hub_ordinal(const HubArgs &h, int v) {
  if (h.ids_identity) return v >= 0 && v < h.n_hubs ? v : -1;
  int lo = 0, hi = h.n_hubs;  // lower bound of v
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (h.ids[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo < h.n_hubs && h.ids[lo] == v ? lo : -1;
}

__device__ __forceinline__ uint32_t part_of(uint32_t lbl, int pbits) {
  return pbits ? (fmix32(lbl) >> (32 - pbits)) : 0u;
}

// Work items of the step's flagged hubs (chunks, partitions, merge groups),
// numbered hub after hub in frontier order.  Three passes: k_hub_plan_tile
// finds each frontier hub's ordinal and the exclusive prefix of its work
// items inside its tile of PLAN_TILE entries (plus the tile's totals);
// k_hub_plan_top turns the tile totals into tile offsets; k_hub_owner adds
// the offset of its tile to each hub's starts.
constexpr int PLAN_TILE = 256;

__global__ __launch_bounds__(PLAN_TILE) void k_hub_plan_tile(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ u64 wsum[3][PLAN_TILE / 64];
  if (blockIdx.x == 0 && threadIdx.x == 0) *h.ovf_count = 0;
  const int count = *a.fcount;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int tile = blockIdx.x; tile * PLAN_TILE < count; tile += gridDim.x) {
    const int i = tile * PLAN_TILE + threadIdx.x;
    u64 kc = 0, kp = 0, kg = 0;
    if (i < count) {
      const int v = a.front[i];
      int lo = hub_ordinal(h, v);
      if (lo < 0) {  // every hub-bin vertex is listed; never expected
        atomicOr(&a.ctl->error, 4);
        lo = 0;
      } else {
        h.slot_of[lo] = i;
        kc = (u64)h.chunks[lo];
        kp = (u64)1 << h.pbits[lo];
        kg = (u64)hub_merge_groups(h.pbits[lo], h.gbits);
      }
      h.ord[i] = lo;
      h.cur[i] = a.C[v];  // the hub's label before the step (its decision compares with it)
      if (h.own_w) h.own_w[i] = 0;
    }
    u64 xc = kc, xp = kp, xg = kg;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const u64 yc = (u64)__shfl_up((unsigned long long)xc, d, 64);
      const u64 yp = (u64)__shfl_up((unsigned long long)xp, d, 64);
      const u64 yg = (u64)__shfl_up((unsigned long long)xg, d, 64);
      if (lane >= d) {
        xc += yc;
        xp += yp;
        xg += yg;
      }
    }
    if (lane == 63) {
      wsum[0][wv] = xc;
      wsum[1][wv] = xp;
      wsum[2][wv] = xg;
    }
    __syncthreads();
    u64 bc = 0, bp = 0, bg = 0;
    for (int k = 0; k < wv; ++k) {
      bc += wsum[0][k];
      bp += wsum[1][k];
      bg += wsum[2][k];
    }
    if (i < count) {
      h.cstart[i] = bc + xc - kc;
      h.pstart[i] = bp + xp - kp;
      h.gstart[i] = bg + xg - kg;
    }
    if (threadIdx.x == PLAN_TILE - 1) {
      h.blk[3 * tile + 0] = bc + xc;
      h.blk[3 * tile + 1] = bp + xp;
      h.blk[3 * tile + 2] = bg + xg;
    }
    __syncthreads();  // wsum is reused by the next tile
  }
}

// Exclusive offsets of the tiles (in place) and the step's totals.
__global__ __launch_bounds__(1024) void k_hub_plan_top(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ u64 wsum[3][16];
  __shared__ u64 carry[3];
  const int tiles = (*a.fcount + PLAN_TILE - 1) / PLAN_TILE;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x < 3) carry[threadIdx.x] = 0;
  __syncthreads();
  for (int base = 0; base < tiles; base += 1024) {
    const int t = base + threadIdx.x;
    u64 x[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) x[q] = t < tiles ? h.blk[3 * t + q] : 0;
    u64 y[3] = {x[0], x[1], x[2]};
#pragma unroll
    for (int d = 1; d < 64; d <<= 1)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const u64 z = (u64)__shfl_up((unsigned long long)y[q], d, 64);
        if (lane >= d) y[q] += z;
      }
    if (lane == 63)
#pragma unroll
      for (int q = 0; q < 3; ++q) wsum[q][wv] = y[q];
    __syncthreads();
    u64 b[3] = {carry[0], carry[1], carry[2]};
    for (int k = 0; k < wv; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) b[q] += wsum[q][k];
    if (t < tiles)
#pragma unroll
      for (int q = 0; q < 3; ++q) h.blk[3 * t + q] = b[q] + y[q] - x[q];
    __syncthreads();
    if (threadIdx.x == 1023)
#pragma unroll
      for (int q = 0; q < 3; ++q) carry[q] = b[q] + y[q];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.ctl->hub_chunks = carry[0];
    a.ctl->hub_groups = carry[2];
  }
}

// The whole plan in one workgroup for a step with at most PLAN_TILE flagged
// hubs (the usual case in the deterministic mode's colour classes): ordinals,
// starts, totals and owner maps, with no tile offsets to add.
__global__ __launch_bounds__(PLAN_TILE) void k_hub_plan_small(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ u64 wsum[3][PLAN_TILE / 64];
  __shared__ int s_k[PLAN_TILE];
  __shared__ u64 s_start[3][PLAN_TILE];
  if (threadIdx.x == 0) *h.ovf_count = 0;
  const int count = *a.fcount;  // at most PLAN_TILE (the host launches this kernel only then)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = threadIdx.x;
  u64 kc = 0, kp = 0, kg = 0;
  if (i < count) {
    const int v = a.front[i];
    int lo = hub_ordinal(h, v);
    if (lo < 0) {
      atomicOr(&a.ctl->error, 4);
      lo = 0;
    } else {
      h.slot_of[lo] = i;
      kc = (u64)h.chunks[lo];
      kp = (u64)1 << h.pbits[lo];
      kg = (u64)hub_merge_groups(h.pbits[lo], h.gbits);
    }
    h.ord[i] = lo;
    h.cur[i] = a.C[v];  // the hub's label before the step (its decision compares with it)
    s_k[i] = lo;
    if (h.own_w) h.own_w[i] = 0;
  }
  u64 xc = kc, xp = kp, xg = kg;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const u64 yc = (u64)__shfl_up((unsigned long long)xc, d, 64);
    const u64 yp = (u64)__shfl_up((unsigned long long)xp, d, 64);
    const u64 yg = (u64)__shfl_up((unsigned long long)xg, d, 64);
    if (lane >= d) {
      xc += yc;
      xp += yp;
      xg += yg;
    }
  }
  if (lane == 63) {
    wsum[0][wv] = xc;
    wsum[1][wv] = xp;
    wsum[2][wv] = xg;
  }
  __syncthreads();
  u64 bc = 0, bp = 0, bg = 0;
  for (int k = 0; k < wv; ++k) {
    bc += wsum[0][k];
    bp += wsum[1][k];
    bg += wsum[2][k];
  }
  if (i < count) {
    s_start[0][i] = h.cstart[i] = bc + xc - kc;
    s_start[1][i] = h.pstart[i] = bp + xp - kp;
    s_start[2][i] = h.gstart[i] = bg + xg - kg;
  }
  if (i == PLAN_TILE - 1) {
    a.ctl->hub_chunks = bc + xc;
    a.ctl->hub_groups = bg + xg;
  }
  __syncthreads();
  for (int q = 0; q < count; ++q) {
    const int k = s_k[q];
    const int nc = h.chunks[k], ng = hub_merge_groups(h.pbits[k], h.gbits);
    for (int c = threadIdx.x; c < nc; c += PLAN_TILE) h.chunk_owner[s_start[0][q] + c] = q;
    for (int gq = threadIdx.x; gq < ng; gq += PLAN_TILE) h.group_owner[s_start[2][q] + gq] = q;
    if (h.first)
      for (int p = threadIdx.x; p < (1 << h.pbits[k]); p += PLAN_TILE) h.partbest[s_start[1][q] + p] = 0;
  }
}

// Owner maps of the step's work items (chunk / merge group -> frontier entry),
// one workgroup per flagged hub.
__global__ __launch_bounds__(256) void k_hub_owner(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  const int count = *a.fcount;
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const int k = h.ord[i];
    const int kc = h.chunks[k], kg = hub_merge_groups(h.pbits[k], h.gbits);
    const u64 *off = h.blk + 3 * (i / PLAN_TILE);
    const u64 c0 = h.cstart[i] + off[0], p0 = h.pstart[i] + off[1], g0 = h.gstart[i] + off[2];
    __syncthreads();  // every thread has read the tile-relative starts
    if (threadIdx.x == 0) {
      h.cstart[i] = c0;
      h.pstart[i] = p0;
      h.gstart[i] = g0;
    }
    for (int c = threadIdx.x; c < kc; c += 256) h.chunk_owner[c0 + c] = i;
    for (int gq = threadIdx.x; gq < kg; gq += 256) h.group_owner[g0 + gq] = i;
    if (h.first)
      for (int p = threadIdx.x; p < (1 << h.pbits[k]); p += 256) h.partbest[p0 + p] = 0;
  }
}

// One LDS array per workgroup: first the chunk's label table, then - once
// every thread holds its share of the table's slots in registers - the
// partition counters (2 << pbits ints, never more than the table's bytes).
// 32 KB per workgroup keeps five workgroups on a CU, which the gathers need
// to keep enough loads in flight.
template <int WK>
__global__ __launch_bounds__(256) void k_hub_chunk(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  constexpr int BITS = __builtin_ctz(HUB_CHUNK_SLOTS);
  constexpr int PER = HUB_CHUNK_SLOTS / 256;
  static_assert(2 * (1 << HUB_LDS_PBITS) * sizeof(int32_t) <= HUB_CHUNK_SLOTS * sizeof(u64),
                "the partition counters fit in the table's memory");
  __shared__ u64 T[HUB_CHUNK_SLOTS];
  int32_t *hist = reinterpret_cast<int32_t *>(T);
  const u64 total = h.static_order  ? (u64)h.sorder_len
                    : h.static_plan ? (u64)h.static_chunks
                                    : a.ctl->hub_chunks;
  int err = 0;
  for (u64 c = blockIdx.x; c < total; c += gridDim.x) {
    int i, k;
    int64_t j;  // chunk of the hub
    if (h.static_order) {
      const u64 sc = h.sorder[c];
      k = (int)(sc >> 32);
      i = h.slot_of[k];
      if (i < 0) continue;  // the hub is not flagged in this step (uniform in the workgroup)
      j = (int64_t)(uint32_t)sc;
    } else {
      i = h.chunk_owner[c];
      if (h.static_plan && !h.taken[i]) continue;  // a hub not flagged in this step (uniform in the workgroup)
      k = h.ord[i];
      j = (int64_t)(c - h.cstart[i]);
    }
    const int v = a.front[i];
    if (h.static_plan && j == 0 && threadIdx.x == 0) {
      // what the plan records for a flagged hub
      h.cur[i] = a.C[v];
      if (h.own_w) h.own_w[i] = 0;
    }
    const int pb = h.pbits[k];
    const int P = 1 << pb;
    const int64_t eb = a.off[v] + j * HUB_CHUNK;
    const int64_t ee = min(a.off[v + 1], eb + (int64_t)HUB_CHUNK);
    for (int s = threadIdx.x; s < HUB_CHUNK_SLOTS; s += 256) T[s] = EMPTY;
    __syncthreads();
    err |= scan_row<256, 8, BITS, WK>(a.idx, a.w, a.C, eb, ee, v, threadIdx.x, T);
    __syncthreads();
    u64 x[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) x[r] = T[threadIdx.x + r * 256];
    __syncthreads();  // the table's memory is reused from here on
    int32_t *cnt = h.pcnt + h.cnt_base[k];
    u64 *dst = h.pairs + h.pair_base[k];
    if (pb > HUB_LDS_PBITS) {
      // a giant hub: every merged label reserves its partition slot directly
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        if (x[r] == EMPTY) continue;
        const uint32_t p = part_of((uint32_t)(x[r] >> 32), pb);
        const int pos = atomicAdd(&cnt[p], 1);
        if (pos < h.part_cap) {
          dst[(int64_t)p * HUB_PART_CAP + pos] = x[r];
        } else {
          const u64 q = atomicAdd(h.ovf_count, (u64)1);
          if (q < (u64)HUB_OVERFLOW_CAP) {
            uint32_t *o = h.ovf + 4 * q;
            o[0] = (uint32_t)(h.pstart[i] + p);
            o[1] = (uint32_t)(x[r] >> 32);
            o[2] = (uint32_t)x[r];
          } else {
            err |= 8;
          }
        }
      }
      continue;  // no LDS use after the barrier above
    }
    int32_t *pbase = hist + P;
    for (int p = threadIdx.x; p < P; p += 256) hist[p] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r)
      if (x[r] != EMPTY) atomicAdd(&hist[part_of((uint32_t)(x[r] >> 32), pb)], 1);
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += 256) {
      const int n = hist[p];
      if (n) pbase[p] = atomicAdd(&cnt[p], n);
      hist[p] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      if (x[r] == EMPTY) continue;
      const uint32_t p = part_of((uint32_t)(x[r] >> 32), pb);
      const int pos = pbase[p] + atomicAdd(&hist[p], 1);
      if (pos < h.part_cap) {
        dst[(int64_t)p * HUB_PART_CAP + pos] = x[r];
      } else {  // partition full: spill (merged by the partition's workgroup)
        const u64 q = atomicAdd(h.ovf_count, (u64)1);
        if (q < (u64)HUB_OVERFLOW_CAP) {
          uint32_t *o = h.ovf + 4 * q;
          o[0] = (uint32_t)(h.pstart[i] + p);
          o[1] = (uint32_t)(x[r] >> 32);
          o[2] = (uint32_t)x[r];
        } else {
          err |= 8;
        }
      }
    }
    __syncthreads();
  }
  if (err) atomicOr(&a.ctl->error, err);
}

// Merges partitions [mb, mb + mc) of frontier hub i (ordinal k) in one LDS
// table and stores the best key of the union in the first partition's slot
// (zero in the others).  Partitions hold disjoint label sets, so the best of
// the union is the best of the partitions.  n pairs in all; cm[m] (in LDS)
// pairs in partition mb + m when mc > 1 (a merge of several partitions never
// includes one that spilled); a single partition that spilled also merges its
// entries of the overflow area.
template <bool FEAT>
__device__ __forceinline__ int merge_parts(const ScanArgs &a, const HubArgs &h, u64 *T, u64 *red, int i, int k,
                                           int pb, int mb, int mc, int n, bool spilled, const int *cm,
                                           u64 nov) {
  constexpr int BITS = __builtin_ctz(HUB_PART_SLOTS);
  int err = 0;
  const u64 q0 = h.pstart[i] + (u64)mb;  // step-wide id of the first partition
  // a table just large enough to stay at most half full (partitions of
  // later sweeps hold few labels); a partition that spilled takes the full
  // table
  int tb = 6;
  while (tb < BITS && (1 << tb) < 2 * n) ++tb;
  if (spilled) tb = BITS;
  const int slots = 1 << tb;
  for (int s = threadIdx.x; s < slots; s += 256) T[s] = EMPTY;
  __syncthreads();
  // pair f of the merge: pair f - (pairs of the earlier partitions) of the
  // partition it falls in; all loads are in flight at once
  const u64 *src = h.pairs + h.pair_base[k] + (int64_t)mb * HUB_PART_CAP;
  constexpr int R = (HUB_PART_CAP + 255) / 256;
  u64 x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int f = threadIdx.x + r * 256;
    x[r] = EMPTY;
    if (f < n) {
      int64_t at = f;
      if (mc > 1) {
        int m = 0, base = 0;
        while (f >= base + cm[m]) base += cm[m++];
        at = (int64_t)m * HUB_PART_CAP + (f - base);
      }
      x[r] = src[at];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (x[r] != EMPTY) err |= !lds_insert_rt(T, tb, (uint32_t)(x[r] >> 32), (uint32_t)x[r]);
  if (spilled)
    for (u64 s = threadIdx.x; s < nov; s += 256) {
      const uint32_t *o = h.ovf + 4 * s;
      if (o[0] == (uint32_t)q0) err |= !lds_insert_rt(T, tb, o[1], o[2]);
    }
  __syncthreads();
  const TieRule tr = tie_rule_of(a, a.front[i]);
  const u64 best = block_max<256>(table_best_rt<256>(T, slots, threadIdx.x, tr), red);
  for (int m = threadIdx.x; m < mc; m += 256) h.partbest[q0 + m] = m == 0 ? best : 0ull;
  if constexpr (FEAT) {
    __shared__ TabStats tred[4];
    const TabStats t = group_stats<64>(table_stats_rt<256>(T, slots, threadIdx.x));
    if ((threadIdx.x & 63) == 0) tred[threadIdx.x >> 6] = t;
    __syncthreads();
    for (int m = threadIdx.x; m < mc; m += 256) {
      const TabStats z = m == 0 ? merge_stats(merge_stats(tred[0], tred[1]), merge_stats(tred[2], tred[3]))
                                : TabStats{0u, 0u, 0};
      h.part_w2[q0 + m] = z.w2;
      h.part_nd[q0 + m] = z.nd;
    }
    if (threadIdx.x == 0) {
      const uint32_t cur = (uint32_t)a.C[a.front[i]];
      const int pc = (int)part_of(cur, pb);
      if (pc >= mb && pc < mb + mc) h.own_w[i] = table_lookup_rt(T, tb, cur);
    }
  }
  __syncthreads();
  return err;
}

// One work item per aligned group of 2^gbits (at most HUB_PART_GROUP)
// partitions of a hub (all of its partitions, if it has fewer).  Consecutive partitions that did not
// spill are merged together while their pairs stay within
// HUB_PART_GROUP_MAX (once labels have merged, usually the whole group in one
// table); a partition that spilled is merged on its own.
template <bool FEAT>
__global__ __launch_bounds__(256) void k_hub_part(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  static_assert(2 * HUB_PART_GROUP_MAX <= HUB_PART_SLOTS, "a merged batch keeps its table at most half full");
  static_assert(HUB_PART_GROUP_MAX <= HUB_PART_CAP, "a batch's pairs fit the per-thread load registers");
  __shared__ u64 T[HUB_PART_SLOTS];
  __shared__ u64 red[4];
  __shared__ int s_cm[HUB_PART_GROUP];  // pairs offered to each partition of the group, spilled ones included
  const u64 total = h.static_plan ? (u64)h.static_groups : a.ctl->hub_groups;
  const u64 nov = min(*h.ovf_count, (u64)HUB_OVERFLOW_CAP);
  int err = 0;
  for (u64 gq = blockIdx.x; gq < total; gq += gridDim.x) {
    const int i = h.group_owner[gq];
    if (h.static_plan && !h.taken[i]) continue;  // uniform in the workgroup
    const int k = h.ord[i];
    const int pb = h.pbits[k];
    const int G = 1 << min(h.gbits, pb);
    const int g0 = (int)(gq - h.gstart[i]) * G;  // first partition of the group
    if ((int)threadIdx.x < G) s_cm[threadIdx.x] = h.pcnt[h.cnt_base[k] + g0 + threadIdx.x];
    __syncthreads();
    for (int m = 0; m < G;) {
      const bool spilled = s_cm[m] > h.part_cap;
      int e = m + 1, n = min(s_cm[m], h.part_cap);
      if (!spilled)
        while (e < G && s_cm[e] <= h.part_cap && n + s_cm[e] <= HUB_PART_GROUP_MAX) n += s_cm[e++];
      err |= merge_parts<FEAT>(a, h, T, red, i, k, pb, g0 + m, e - m, n, spilled, s_cm + m, nov);
      m = e;
    }
  }
  if (err) atomicOr(&a.ctl->error, 16);
}

// Strict argmax of each flagged hub over its partitions, and the update.
// One wave per hub.
template <bool FEAT>
__global__ __launch_bounds__(256) void k_hub_decide(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  const int count = h.static_plan ? (int)h.static_count : *a.fcount;
  const int lane = threadIdx.x & 63;
  const int sweep = FEAT ? a.ctl->sweep : 0;
  u64 n_changed = 0, n_scanned = 0, n_vert = 0;
  for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < count; i += gridDim.x * 4) {
    if (h.static_plan && !h.taken[i]) {  // not flagged in this step: nothing decided, no marks
      if (lane == 0) h.changed[i] = 0;
      continue;
    }
    const int v = a.front[i];
    const int P = 1 << h.pbits[h.ord[i]];
    const u64 *pb = h.partbest + h.pstart[i];
    int32_t *cnt = h.pcnt + h.cnt_base[h.ord[i]];
    u64 best = 0;
    for (int p = lane; p < P; p += 64) {
      best = pb[p] > best ? pb[p] : best;
      cnt[p] = 0;  // partitions start empty at the next step
    }
    best = group_max<64>(best);
    int changed = 0;
    const int32_t cur = a.C[v];
    if (best != 0) {
      const int32_t cs = (int32_t)key_label(best, tie_rule_of(a, v));
      if (cs != cur) {
        changed = 1;
        if (lane == 0) {
          a.C[v] = cs;
          ++n_changed;
          if (a.chg) a.chg[v] = 1;
        }
      }
    }
    if constexpr (FEAT) {
      TabStats t{0u, 0u, 0};
      const u64 q0 = h.pstart[i];
      for (int p = lane; p < P; p += 64) {
        const u64 key = pb[p];
        TabStats o;
        o.w1 = key ? (uint32_t)(key >> 32) : 0u;
        o.w2 = h.part_w2[q0 + p];
        o.nd = h.part_nd[q0 + p];
        t = merge_stats(t, o);
      }
      t = group_stats<64>(t);
      if (lane == 0)
        write_features(a.f, v, sweep, a.off[v + 1] - a.off[v], t, h.own_w[i], changed != 0, a.f.K[v],
                       record_lastp(a.f.feat + (int64_t)v * FEAT_STRIDE));
    }
    if (lane == 0) {
      h.slot_of[h.ord[i]] = -1;  // not flagged until a later plan says so
      h.changed[i] = changed;
      n_scanned += (u64)(a.off[v + 1] - a.off[v]);
      ++n_vert;
    }
  }
  block_accum<256>(n_changed, n_scanned, n_vert, 0, 0, a.ctl, a.bin);
}

// Neighbour marks of the hubs that changed, one workgroup per chunk.
__global__ __launch_bounds__(256) void k_hub_mark(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  if (__atomic_load_n(&a.ctl->dense_cur, __ATOMIC_RELAXED)) return;  // dense sweep: flags are set at its end
  const u64 total = h.static_plan ? (u64)h.static_chunks : a.ctl->hub_chunks;
  u64 n_marks = 0;
  for (u64 c = blockIdx.x; c < total; c += gridDim.x) {
    const int i = h.chunk_owner[c];
    if (!h.changed[i]) continue;
    const int v = a.front[i];
    const int64_t eb = a.off[v] + (int64_t)(c - h.cstart[i]) * HUB_CHUNK;
    const int64_t ee = min(a.off[v + 1], eb + (int64_t)HUB_CHUNK);
    n_marks += mark_row<256, 8>(a.idx, a.F, eb, ee, v, threadIdx.x);
  }
  block_accum<256>(0, 0, 0, n_marks, 0, a.ctl, a.bin);
}

// Decision and neighbour marks in one pass, one workgroup per chunk of a
// flagged hub: every workgroup of a hub takes the strict argmax over the hub's
// partitions (the same in each), compares its label with the label the hub
// had when the step was planned and, if it differs, flags the neighbours in
// its chunk; the workgroup of the hub's first chunk also writes the label,
// the counts and the features and clears the partition counters.
template <bool FEAT>
__global__ __launch_bounds__(256) void k_hub_finish(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ u64 red[4];
  __shared__ TabStats tred[FEAT ? 4 : 1];
  // a dense sweep sets every flag at its end instead
  const bool marks = a.prune && !__atomic_load_n(&a.ctl->dense_cur, __ATOMIC_RELAXED);
  const u64 total = h.static_plan ? (u64)h.static_chunks : a.ctl->hub_chunks;
  const int sweep = FEAT ? a.ctl->sweep : 0;
  u64 n_changed = 0, n_scanned = 0, n_vert = 0, n_marks = 0;
  for (u64 c = blockIdx.x; c < total; c += gridDim.x) {
    const int i = h.chunk_owner[c];
    if (h.static_plan && !h.taken[i]) continue;  // uniform in the workgroup
    const int k = h.ord[i];
    const int v = a.front[i];
    const int64_t j = (int64_t)(c - h.cstart[i]);  // chunk of the hub
    const int P = 1 << h.pbits[k];
    const u64 *pb = h.partbest + h.pstart[i];
    u64 best = 0;
    for (int p = threadIdx.x; p < P; p += 256) best = pb[p] > best ? pb[p] : best;
    best = block_max<256>(best, red);
    const int32_t cur = h.cur[i];
    const int32_t cs = best != 0 ? (int32_t)key_label(best, tie_rule_of(a, v)) : cur;
    const bool changed = cs != cur;
    if (j == 0) {
      int32_t *cnt = h.pcnt + h.cnt_base[k];
      for (int p = threadIdx.x; p < P; p += 256) cnt[p] = 0;  // partitions start empty at the next step
      if constexpr (FEAT) {
        TabStats t{0u, 0u, 0};
        const u64 q0 = h.pstart[i];
        for (int p = threadIdx.x; p < P; p += 256) {
          const u64 key = pb[p];
          TabStats o;
          o.w1 = key ? (uint32_t)(key >> 32) : 0u;
          o.w2 = h.part_w2[q0 + p];
          o.nd = h.part_nd[q0 + p];
          t = merge_stats(t, o);
        }
        t = group_stats<64>(t);
        if ((threadIdx.x & 63) == 0) tred[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
          t = merge_stats(merge_stats(tred[0], tred[1]), merge_stats(tred[2], tred[3]));
          write_features(a.f, v, sweep, a.off[v + 1] - a.off[v], t, h.own_w[i], changed, a.f.K[v],
                         record_lastp(a.f.feat + (int64_t)v * FEAT_STRIDE));
        }
      }
      if (threadIdx.x == 0) {
        if (changed) {
          a.C[v] = cs;
          ++n_changed;
          if (a.chg) a.chg[v] = 1;
        }
        h.slot_of[k] = -1;  // not flagged until a later plan says so
        n_scanned += (u64)(a.off[v + 1] - a.off[v]);
        ++n_vert;
      }
    }
    if (changed && marks) {
      const int64_t eb = a.off[v] + j * HUB_CHUNK;
      const int64_t ee = min(a.off[v + 1], eb + (int64_t)HUB_CHUNK);
      n_marks += mark_row<256, 8>(a.idx, a.F, eb, ee, v, threadIdx.x);
    }
    __syncthreads();  // red and tred are reused by the next chunk
  }
  block_accum<256>(n_changed, n_scanned, n_vert, n_marks, 0, a.ctl, a.bin);
}

void launch_hub_plan(const ScanArgs &a, const HubArgs &h, int64_t max_hubs, int blocks, int tile_blocks,
                     hipStream_t st) {
  if (max_hubs <= PLAN_TILE) {
    hipLaunchKernelGGL(k_hub_plan_small, dim3(1), dim3(PLAN_TILE), 0, st, a, h);
    return;
  }
  hipLaunchKernelGGL(k_hub_plan_tile, dim3(tile_blocks), dim3(PLAN_TILE), 0, st, a, h);
  hipLaunchKernelGGL(k_hub_plan_top, dim3(1), dim3(1024), 0, st, a, h);
  hipLaunchKernelGGL(k_hub_owner, dim3(blocks), dim3(256), 0, st, a, h);
}

int hub_plan_tiles(int64_t entries) { return (int)((entries + PLAN_TILE - 1) / PLAN_TILE); }

void launch_hub_chunk(int wk, int blocks, hipStream_t st, const ScanArgs &a, const HubArgs &h) {
  if (wk == W_UNIT) hipLaunchKernelGGL(k_hub_chunk<W_UNIT>, dim3(blocks), dim3(256), 0, st, a, h);
  else if (wk == W_U8) hipLaunchKernelGGL(k_hub_chunk<W_U8>, dim3(blocks), dim3(256), 0, st, a, h);
  else hipLaunchKernelGGL(k_hub_chunk<W_U32>, dim3(blocks), dim3(256), 0, st, a, h);
}

void launch_hub_part(int blocks, bool feat, hipStream_t st, const ScanArgs &a, const HubArgs &h) {
  if (feat) hipLaunchKernelGGL(k_hub_part<true>, dim3(blocks), dim3(256), 0, st, a, h);
  else hipLaunchKernelGGL(k_hub_part<false>, dim3(blocks), dim3(256), 0, st, a, h);
}

void launch_hub_finish(int hub_blocks, int chunk_blocks, int prune, bool feat, bool fused, hipStream_t st,
                       const ScanArgs &a, const HubArgs &h) {
  if (fused) {
    if (feat) hipLaunchKernelGGL(k_hub_finish<true>, dim3(chunk_blocks), dim3(256), 0, st, a, h);
    else hipLaunchKernelGGL(k_hub_finish<false>, dim3(chunk_blocks), dim3(256), 0, st, a, h);
    return;
  }
  if (feat) hipLaunchKernelGGL(k_hub_decide<true>, dim3(hub_blocks), dim3(256), 0, st, a, h);
  else hipLaunchKernelGGL(k_hub_decide<false>, dim3(hub_blocks), dim3(256), 0, st, a, h);
  if (prune) hipLaunchKernelGGL(k_hub_mark, dim3(chunk_blocks), dim3(256), 0, st, a, h);
}

}  // namespace gvelpa
