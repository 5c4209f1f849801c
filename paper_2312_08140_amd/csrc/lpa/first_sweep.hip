// Snapshot first sweep (asynchronous mode): the first sweep of a run that
// starts from the initial labels, with every vertex reading the labels as
// they were when the sweep began.
//
// Asynchronous LPA (Section 4.1) lets a vertex read a neighbour's label before
// or after that neighbour's update in the same sweep; reading every label
// before any update is one admissible interleaving.  At the start of a run
// the label of position j is its vertex id orig[j] (Algorithm 1 initialises
// C[v] = v), and in a row without repeated neighbours every label occurs once,
// so the summed weight of a label (scanCommunities) is the weight of its one
// entry.  Eq. (2) then reduces to: the heaviest entry, and among the heaviest
// the smallest id (strict LPA) or the smallest rank (non-strict LPA) - no
// label table at all, and a neighbour's id is read only when its entry
// reaches the running maximum weight of the lane that holds it.  The engine
// uses these kernels only when every row's neighbours are strictly increasing
// (sorted rows, hence no repeated neighbour) and the run starts from the
// initial labels.  With the gate's features on (FEAT), the bin kernels also
// record them: with every label distinct, the two largest label weights are
// the two largest entry weights, the distinct labels are the entries other
// than the vertex itself, and the vertex's own label (its id) has weight 0.
#include "sweep_kernels.hpp"
#include "tables.hpp"

namespace gvelpa {

// Lane `lane` of a group of STRIDE lanes: the largest argmax key among the
// entries lane, lane + STRIDE, ... of [b, e) (vertex v itself skipped), with
// U entries in flight; counts the ids it reads; FEAT: the lane's two largest
// entry weights and its entries in ts.
template <int STRIDE, int U, int WK, bool FEAT = false>
__device__ __forceinline__ u64 first_row(const ScanArgs &a, int64_t b, int64_t e, int v, int lane, TieRule tr,
                                         u64 &reads, TabStats &ts) {
  u64 best = 0;
  uint32_t bw = 0;  // the lane's largest weight so far
  for (int64_t base = b + lane; base < e; base += (int64_t)STRIDE * U) {
    int j[U];
    uint32_t w[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t k = base + (int64_t)r * STRIDE;
      const bool ok = k < e;
      j[r] = ok ? a.idx[k] : -1;
      w[r] = ok ? load_w<WK>(a.w, k) : 0u;
    }
    uint32_t mw = bw;
#pragma unroll
    for (int r = 0; r < U; ++r)
      if (j[r] >= 0 && j[r] != v) {
        mw = w[r] > mw ? w[r] : mw;
        if constexpr (FEAT) {
          ++ts.nd;
          if (w[r] > ts.w1) {
            ts.w2 = ts.w1;
            ts.w1 = w[r];
          } else if (w[r] > ts.w2) {
            ts.w2 = w[r];
          }
        }
      }
    uint32_t lb[U];
#pragma unroll
    for (int r = 0; r < U; ++r)
      lb[r] = (j[r] >= 0 && j[r] != v && w[r] == mw) ? (uint32_t)(a.orig ? a.orig[j[r]] : j[r]) : 0xFFFFFFFFu;
#pragma unroll
    for (int r = 0; r < U; ++r) {
      if (lb[r] == 0xFFFFFFFFu) continue;
      ++reads;
      const u64 key = entry_key(((u64)lb[r] << 32) | w[r], tr);
      best = key > best ? key : best;
    }
    bw = mw;
  }
  return best;
}

// One vertex per GROUP lanes (GROUP <= 64: lanes of one wave; GROUP == BLOCK:
// the whole workgroup).  Counters go to the first-sweep shard slots.
template <int GROUP, int BLOCK, int U, int WK, bool FEAT>
__global__ __launch_bounds__(BLOCK) void k_first_scan(ScanArgs a) {
  static_assert(GROUP <= 64 || GROUP == BLOCK, "a vertex takes lanes of one wave or the whole workgroup");
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  constexpr int GPB = BLOCK / GROUP;
  __shared__ u64 red[BLOCK / 64];
  __shared__ TabStats tred[FEAT && GROUP > 64 ? BLOCK / 64 : 1];
  const int lane = threadIdx.x % GROUP;
  const int grp = threadIdx.x / GROUP;
  const int count = *a.fcount;
  if ((int)blockIdx.x * GPB >= count) return;
  const bool mark_now = a.prune && !__atomic_load_n(&a.ctl->dense_cur, __ATOMIC_RELAXED);
  u64 n_changed = 0, n_scanned = 0, n_vert = 0, n_marks = 0, n_reads = 0;
  for (int i = blockIdx.x * GPB + grp; i < count; i += gridDim.x * GPB) {
    const int v = a.front[i];
    const int64_t b = a.off[v], e = a.off[v + 1];
    const TieRule tr = tie_rule_of(a, v);
    TabStats ts{0u, 0u, 0};
    u64 best = first_row<GROUP, U, WK, FEAT>(a, b, e, v, lane, tr, n_reads, ts);
    if constexpr (GROUP == BLOCK && BLOCK > 64) best = block_max<BLOCK>(best, red);
    else best = group_max<GROUP>(best);
    bool changed = false;
    if (best != 0) {
      const int32_t cs = (int32_t)key_label(best, tr);
      if (cs != a.C[v]) {
        changed = true;
        if (lane == 0) {
          a.C[v] = cs;
          ++n_changed;
          if (a.chg) a.chg[v] = 1;
        }
        if (mark_now) n_marks += mark_row<GROUP, U>(a.idx, a.F, b, e, v, lane);
      }
    }
    if constexpr (FEAT) {
      TabStats t = group_stats<(GROUP < 64 ? GROUP : 64)>(ts);
      if constexpr (GROUP > 64) {
        if ((threadIdx.x & 63) == 0) tred[threadIdx.x >> 6] = t;
        __syncthreads();
        t = tred[0];
        for (int q = 1; q < BLOCK / 64; ++q) t = merge_stats(t, tred[q]);
      }
      if (lane == 0)
        write_features(a.f, v, a.ctl->sweep, e - b, t, 0u, changed, a.f.K[v],
                       record_lastp(a.f.feat + (int64_t)v * FEAT_STRIDE));
    }
    if (lane == 0) {
      n_scanned += (u64)(e - b);
      ++n_vert;
    }
    if constexpr (GROUP == BLOCK && BLOCK > 64) __syncthreads();  // red is reused by the next vertex
  }
  block_accum<BLOCK>(n_changed, n_scanned, n_vert, n_marks, 0, a.ctl, FIRST_SLOT);
  __syncthreads();  // block_accum's staging is reused below
  block_accum<BLOCK>(n_reads, 0, 0, 0, 0, a.ctl, READS_SLOT);
}

// Hub chunks: the chunk's best key, combined per hub with a 64-bit atomic
// maximum in the slot of the hub's first partition (zeroed by k_hub_owner);
// k_hub_finish then takes the maximum over the partitions as usual.
template <int WK>
__global__ __launch_bounds__(256) void k_hub_first_chunk(ScanArgs a, HubArgs h) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ u64 red[4];
  const u64 total = a.ctl->hub_chunks;
  u64 n_reads = 0;
  for (u64 c = blockIdx.x; c < total; c += gridDim.x) {
    const int i = h.chunk_owner[c];
    const int v = a.front[i];
    const int64_t eb = a.off[v] + (int64_t)(c - h.cstart[i]) * HUB_CHUNK;
    const int64_t ee = min(a.off[v + 1], eb + (int64_t)HUB_CHUNK);
    const TieRule tr = tie_rule_of(a, v);
    TabStats ts{0u, 0u, 0};
    const u64 best = block_max<256>(first_row<256, 8, WK>(a, eb, ee, v, threadIdx.x, tr, n_reads, ts), red);
    if (threadIdx.x == 0 && best != 0) atomicMax((unsigned long long *)&h.partbest[h.pstart[i]], best);
    __syncthreads();  // red is reused by the next chunk
  }
  block_accum<256>(n_reads, 0, 0, 0, 0, a.ctl, READS_SLOT);
}

// ---------------------------------------------------------------- launchers

template <int B, int V, int WK, bool FEAT>
static void launch_first_shape(dim3 grid, hipStream_t st, const ScanArgs &a) {
  constexpr BinShape sh = BIN_SHAPES[B][V];
  if constexpr (B <= 3)
    hipLaunchKernelGGL((k_first_scan<sh.group, 256, sh.unroll, WK, FEAT>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((k_first_scan<sh.group, sh.group, sh.unroll, WK, FEAT>), grid, dim3(sh.group), 0, st, a);
}

template <int B, int WK, bool FEAT>
static void launch_first_v(int variant, dim3 grid, hipStream_t st, const ScanArgs &a) {
  switch (variant) {
    case 1: launch_first_shape<B, 1, WK, FEAT>(grid, st, a); break;
    case 2: launch_first_shape<B, 2, WK, FEAT>(grid, st, a); break;
    default: launch_first_shape<B, 0, WK, FEAT>(grid, st, a); break;
  }
}

template <int WK, bool FEAT>
static void launch_first_wk(int bin, int variant, dim3 grid, hipStream_t st, const ScanArgs &a) {
  switch (bin) {
    case 0: launch_first_v<0, WK, FEAT>(variant, grid, st, a); break;
    case 1: launch_first_v<1, WK, FEAT>(variant, grid, st, a); break;
    case 2: launch_first_v<2, WK, FEAT>(variant, grid, st, a); break;
    case 3: launch_first_v<3, WK, FEAT>(variant, grid, st, a); break;
    case 4: launch_first_v<4, WK, FEAT>(variant, grid, st, a); break;
    case 5: launch_first_v<5, WK, FEAT>(variant, grid, st, a); break;
    default: break;
  }
}

void launch_first_bin(int bin, int variant, int wk, bool feat, int blocks, hipStream_t st, const ScanArgs &a) {
  if (feat) {
    if (wk == W_UNIT) launch_first_wk<W_UNIT, true>(bin, variant, dim3(blocks), st, a);
    else if (wk == W_U8) launch_first_wk<W_U8, true>(bin, variant, dim3(blocks), st, a);
    else launch_first_wk<W_U32, true>(bin, variant, dim3(blocks), st, a);
  } else {
    if (wk == W_UNIT) launch_first_wk<W_UNIT, false>(bin, variant, dim3(blocks), st, a);
    else if (wk == W_U8) launch_first_wk<W_U8, false>(bin, variant, dim3(blocks), st, a);
    else launch_first_wk<W_U32, false>(bin, variant, dim3(blocks), st, a);
  }
}

void launch_hub_first_chunk(int wk, int blocks, hipStream_t st, const ScanArgs &a, const HubArgs &h) {
  if (wk == W_UNIT) hipLaunchKernelGGL(k_hub_first_chunk<W_UNIT>, dim3(blocks), dim3(256), 0, st, a, h);
  else if (wk == W_U8) hipLaunchKernelGGL(k_hub_first_chunk<W_U8>, dim3(blocks), dim3(256), 0, st, a, h);
  else hipLaunchKernelGGL(k_hub_first_chunk<W_U32>, dim3(blocks), dim3(256), 0, st, a, h);
}

}  // namespace gvelpa
