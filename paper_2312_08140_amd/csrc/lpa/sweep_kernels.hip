// Label-scan sweep kernels (gfx950, wave64).
//
// One sweep of Algorithm 1 (Section 4.2) over the flagged vertices of a step
// (the whole graph in async mode, one colour class in deterministic mode):
//   k_compact       pruning (Section 4.1.4): keep flagged vertices, clear their
//                   flags before the scan, split them by degree bin;
//   k_scan_group    scanCommunities + best label + update for low/mid degree,
//                   GROUP lanes per vertex, LDS open-addressing table;
//   k_scan_block    the same with one workgroup per vertex;
//   k_hub_*         hubs: many workgroups per vertex, table in HBM;
//   k_end_sweep     dN/N <= tau stop test and per-sweep statistics.
// The update rule is Eq. (2) in its strict form: largest summed weight, the
// smallest label id on ties (Section 2); the vertex itself is skipped
// (Algorithm 1, scanCommunities).
#include "sweep_kernels.hpp"

namespace gvelpa {

// ---------------------------------------------------------------- tables

template <int BITS>
__device__ __forceinline__ bool lds_insert(u64 *T, uint32_t lbl, uint32_t w) {
  constexpr uint32_t MASK = (1u << BITS) - 1;
  uint32_t h = slot_hash(lbl, BITS);
  const u64 mine = ((u64)lbl << 32) | w;
  for (int probe = 0; probe <= (int)MASK; ++probe) {
    const u64 cur = __atomic_load_n(&T[h], __ATOMIC_RELAXED);
    if ((uint32_t)(cur >> 32) == lbl) {
      atomicAdd(&T[h], (u64)w);
      return true;
    }
    if (cur == EMPTY) {
      const u64 old = atomicCAS(&T[h], EMPTY, mine);
      if (old == EMPTY) return true;
      if ((uint32_t)(old >> 32) == lbl) {
        atomicAdd(&T[h], (u64)w);
        return true;
      }
    }
    h = (h + 1) & MASK;
  }
  return false;
}

__device__ __forceinline__ bool hbm_insert(u64 *T, int bits, uint32_t lbl, uint32_t w) {
  const uint32_t mask = (1u << bits) - 1;
  uint32_t h = slot_hash(lbl, bits);
  const u64 mine = ((u64)lbl << 32) | w;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const u64 cur = __atomic_load_n(&T[h], __ATOMIC_RELAXED);
    if ((uint32_t)(cur >> 32) == lbl) {
      atomicAdd(&T[h], (u64)w);
      return true;
    }
    if (cur == EMPTY) {
      const u64 old = atomicCAS(&T[h], EMPTY, mine);
      if (old == EMPTY) return true;
      if ((uint32_t)(old >> 32) == lbl) {
        atomicAdd(&T[h], (u64)w);
        return true;
      }
    }
    h = (h + 1) & mask;
  }
  return false;
}

template <int BLOCK>
__device__ __forceinline__ void block_add3(u64 a, u64 b, int c, Ctl *ctl) {
  __shared__ u64 s_a[BLOCK / 64], s_b[BLOCK / 64];
  __shared__ int s_c[BLOCK / 64];
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    a += shfl_xor_u64(a, m);
    b += shfl_xor_u64(b, m);
    c |= __shfl_xor(c, m, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_a[wv] = a;
    s_b[wv] = b;
    s_c[wv] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 ta = 0, tb = 0;
    int tc = 0;
    for (int k = 0; k < BLOCK / 64; ++k) {
      ta += s_a[k];
      tb += s_b[k];
      tc |= s_c[k];
    }
    if (ta) atomicAdd((u64 *)&ctl->changed, ta);
    if (tb) atomicAdd((u64 *)&ctl->scanned, tb);
    if (tc) atomicOr(&ctl->error, 1);
  }
}

// ---------------------------------------------------------------- run control

// Labels and flags before the first sweep.  A vertex without stored entries
// is processed in sweep 0 like any other (its flag is cleared, its label
// kept) and nothing can mark it again, so its flag is cleared here once a run
// has at least one sweep; such vertices are not in the work lists.
__global__ void k_init_state(const int64_t *off, int32_t *C, uint8_t *F, int64_t n, int set_labels, int set_flags,
                             int clear_isolated) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (set_labels) C[v] = (int32_t)v;
    if (set_flags) F[v] = 1;
    if (clear_isolated && off[v + 1] == off[v]) F[v] = 0;
  }
}

__global__ void k_run_begin(Ctl *ctl, double tau, int max_iters, int64_t n, int32_t *fcount, int nfc,
                            int32_t *host_done) {
  for (int k = threadIdx.x; k < nfc; k += blockDim.x) fcount[k] = 0;
  if (threadIdx.x == 0) {
    ctl->done = max_iters <= 0 ? 1 : 0;
    ctl->sweep = 0;
    ctl->iterations = 0;
    ctl->converged = 0;
    ctl->error = 0;
    ctl->max_iters = max_iters;
    ctl->verify_phase = 0;
    ctl->tau = tau;
    ctl->n = n;
    ctl->changed = ctl->processed = ctl->scanned = ctl->gated = 0;
    ctl->hub_chunks = 0;
    ctl->verify_changed = ctl->total_changed = 0;
    for (int k = 0; k < MAX_REC; ++k)
      ctl->st_changed[k] = ctl->st_processed[k] = ctl->st_scanned[k] = ctl->st_gated[k] = ctl->t_sweep[k] = 0;
    ctl->t_start = wall_clock64();
    if (host_done) {
      __atomic_store_n(host_done, ctl->done, __ATOMIC_RELAXED);
      __threadfence_system();
    }
  }
}

__global__ void k_end_sweep(Ctl *ctl, int32_t *fcount, int nfc, int32_t *host_done) {
  if (__atomic_load_n(&ctl->done, __ATOMIC_RELAXED)) return;
  for (int k = threadIdx.x; k < nfc; k += blockDim.x) fcount[k] = 0;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int s = ctl->sweep;
  const u64 dn = ctl->changed;
  if (s < MAX_REC) {
    ctl->st_changed[s] = dn;
    ctl->st_processed[s] = ctl->processed;
    ctl->st_scanned[s] = ctl->scanned;
    ctl->st_gated[s] = ctl->gated;
    ctl->t_sweep[s] = wall_clock64();
  }
  ctl->total_changed += dn;
  ctl->iterations = s + 1;
  ctl->sweep = s + 1;
  // Algorithm 1: stop when dN / N <= tau (evaluated in double).
  const bool conv = (double)dn / (double)(ctl->n > 0 ? ctl->n : 1) <= ctl->tau;
  if (conv) ctl->converged = 1;
  if (conv || s + 1 >= ctl->max_iters) ctl->done = 1;
  ctl->changed = ctl->processed = ctl->scanned = ctl->gated = 0;
  if (host_done) {
    __atomic_store_n(host_done, ctl->done, __ATOMIC_RELAXED);
    __threadfence_system();
  }
}

// ---------------------------------------------------------------- compaction

__global__ __launch_bounds__(256) void k_compact(CompactArgs a) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ int lcount[NBINS];
  __shared__ int lbase[NBINS];
  __shared__ int s_taken[4];
  int taken_total = 0;
  for (int64_t tile = (int64_t)blockIdx.x * 256; tile < a.len; tile += (int64_t)gridDim.x * 256) {
    if (threadIdx.x < NBINS) lcount[threadIdx.x] = 0;
    __syncthreads();
    const int64_t p = tile + threadIdx.x;
    int v = -1, b = 0, slot = 0;
    bool take = false;
    if (p < a.len) {
      v = a.list[p];
#pragma unroll
      for (int k = 1; k < NBINS; ++k)
        if (p >= a.bounds[k]) b = k;
      take = a.prune ? (a.F[v] != 0) : true;
      if (take) {
        a.F[v] = 0;  // marked processed before its scan
        slot = atomicAdd(&lcount[b], 1);
      }
    }
    __syncthreads();
    if (threadIdx.x < NBINS && lcount[threadIdx.x] > 0)
      lbase[threadIdx.x] = atomicAdd(&a.fcount[threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
    if (take) a.front[a.bounds[b] + lbase[b] + slot] = v;
    taken_total += take ? 1 : 0;
    __syncthreads();
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) taken_total += __shfl_xor(taken_total, m, 64);
  if ((threadIdx.x & 63) == 0) s_taken[threadIdx.x >> 6] = taken_total;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = s_taken[0] + s_taken[1] + s_taken[2] + s_taken[3];
    if (t) atomicAdd((u64 *)&a.ctl->processed, (u64)t);
  }
}

// ---------------------------------------------------------------- low / mid degree

template <int GROUP, int SLOTS, int WK>
__global__ __launch_bounds__(256) void k_scan_group(ScanArgs a) {
  static_assert(GROUP <= 64 && (GROUP & (GROUP - 1)) == 0, "a group lives inside one wave");
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  constexpr int GPB = 256 / GROUP;
  constexpr int BITS = __builtin_ctz(SLOTS);
  __shared__ u64 tab[GPB * SLOTS];
  const int lane = threadIdx.x % GROUP;
  const int grp = threadIdx.x / GROUP;
  u64 *T = tab + grp * SLOTS;
  const int count = *a.fcount;
  u64 n_changed = 0, n_scanned = 0;
  int overflow = 0;
  for (int i = blockIdx.x * GPB + grp; i < count; i += gridDim.x * GPB) {
    const int v = a.front[i];
#pragma unroll
    for (int s = lane; s < SLOTS; s += GROUP) T[s] = EMPTY;
    wave_lds_sync();
    const int64_t b = a.off[v], e = a.off[v + 1];
    for (int64_t k = b + lane; k < e; k += GROUP) {
      const int j = a.idx[k];
      if (j == v) continue;
      overflow |= !lds_insert<BITS>(T, (uint32_t)a.C[j], load_w<WK>(a.w, k));
    }
    wave_lds_sync();
    u64 best = 0;
#pragma unroll
    for (int s = lane; s < SLOTS; s += GROUP) {
      const u64 x = T[s];
      if (x != EMPTY) {
        const u64 kk = entry_key(x);
        best = kk > best ? kk : best;
      }
    }
    best = group_max<GROUP>(best);
    if (best != 0) {
      const int32_t cs = (int32_t)key_label(best);
      if (cs != a.C[v]) {
        if (lane == 0) {
          a.C[v] = cs;
          ++n_changed;
        }
        if (a.prune)
          for (int64_t k = b + lane; k < e; k += GROUP) {
            const int j = a.idx[k];
            if (j != v) a.F[j] = 1;
          }
      }
    }
    if (lane == 0) n_scanned += (u64)(e - b);
    wave_lds_sync();
  }
  block_add3<256>(n_changed, n_scanned, overflow, a.ctl);
}

template <int BLOCK, int SLOTS, int WK>
__global__ __launch_bounds__(BLOCK) void k_scan_block(ScanArgs a) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  constexpr int BITS = __builtin_ctz(SLOTS);
  constexpr int NW = BLOCK / 64;
  __shared__ u64 T[SLOTS];
  __shared__ u64 red[NW];
  const int count = *a.fcount;
  u64 n_changed = 0, n_scanned = 0;
  int overflow = 0;
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const int v = a.front[i];
    for (int s = threadIdx.x; s < SLOTS; s += BLOCK) T[s] = EMPTY;
    __syncthreads();
    const int64_t b = a.off[v], e = a.off[v + 1];
    for (int64_t k = b + threadIdx.x; k < e; k += BLOCK) {
      const int j = a.idx[k];
      if (j == v) continue;
      overflow |= !lds_insert<BITS>(T, (uint32_t)a.C[j], load_w<WK>(a.w, k));
    }
    __syncthreads();
    u64 best = 0;
    for (int s = threadIdx.x; s < SLOTS; s += BLOCK) {
      const u64 x = T[s];
      if (x != EMPTY) {
        const u64 kk = entry_key(x);
        best = kk > best ? kk : best;
      }
    }
    best = group_max<64>(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    best = red[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) best = red[k] > best ? red[k] : best;
    if (best != 0) {
      const int32_t cs = (int32_t)key_label(best);
      if (cs != a.C[v]) {
        __syncthreads();  // every thread has compared against the old label
        if (threadIdx.x == 0) {
          a.C[v] = cs;
          ++n_changed;
        }
        if (a.prune)
          for (int64_t k = b + threadIdx.x; k < e; k += BLOCK) {
            const int j = a.idx[k];
            if (j != v) a.F[j] = 1;
          }
      }
    }
    if (threadIdx.x == 0) n_scanned += (u64)(e - b);
    __syncthreads();
  }
  block_add3<BLOCK>(n_changed, n_scanned, overflow, a.ctl);
}

// ---------------------------------------------------------------- hubs

// Plans the hub step: work items of HUB_CHUNK edges per flagged hub and the
// HBM table of each.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_hub_plan(ScanArgs a, u64 *cstart, int64_t *toff, int32_t *tbits) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ u64 wsum[16];
  __shared__ u64 s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int count = *a.fcount;
  for (int tile = 0; tile < count; tile += 1024) {
    const int i = tile + threadIdx.x;
    u64 c = 0;
    if (i < count) {
      const int v = a.front[i];
      const int64_t deg = a.off[v + 1] - a.off[v];
      c = (u64)((deg + HUB_CHUNK - 1) / HUB_CHUNK);
      int lo = 0, hi = a.n_hubs;  // lower_bound of v among the sorted hub ids
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a.hub_ids[mid] < v) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= a.n_hubs || a.hub_ids[lo] != v) {  // every hub-bin vertex is listed; never expected
        atomicOr(&a.ctl->error, 4);
        lo = 0;
        c = 0;
      }
      toff[i] = a.hub_toff_all[lo];
      tbits[i] = a.hub_tbits_all[lo];
    }
    // block exclusive scan of c
    u64 x = c;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const u64 y = (u64)__shfl_up((unsigned long long)x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    u64 before = 0;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    const u64 carry = s_carry;
    if (i < count) cstart[i] = carry + before + x - c;
    __syncthreads();
    if (threadIdx.x == 1023) s_carry = carry + before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) a.ctl->hub_chunks = s_carry;
}

template <int WK>
__global__ __launch_bounds__(256) void k_hub_scan(ScanArgs a, const u64 *cstart, const int64_t *toff,
                                                  const int32_t *tbits) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  const u64 total = a.ctl->hub_chunks;
  const int count = *a.fcount;
  int overflow = 0;
  for (u64 c = blockIdx.x; c < total; c += gridDim.x) {
    int lo = 0, hi = count;  // last i with cstart[i] <= c
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (cstart[mid] <= c) lo = mid;
      else hi = mid;
    }
    const int v = a.front[lo];
    const int64_t b = a.off[v] + (int64_t)(c - cstart[lo]) * HUB_CHUNK;
    const int64_t e = min(a.off[v + 1], b + (int64_t)HUB_CHUNK);
    u64 *T = a.htab + toff[lo];
    const int bits = tbits[lo];
    for (int64_t k = b + threadIdx.x; k < e; k += 256) {
      const int j = a.idx[k];
      if (j == v) continue;
      overflow |= !hbm_insert(T, bits, (uint32_t)a.C[j], load_w<WK>(a.w, k));
    }
  }
  if (overflow) atomicOr(&a.ctl->error, 2);
}

__global__ __launch_bounds__(256) void k_hub_finish(ScanArgs a, const int64_t *toff, const int32_t *tbits) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ u64 red[4];
  const int count = *a.fcount;
  u64 n_changed = 0, n_scanned = 0;
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const int v = a.front[i];
    u64 *T = a.htab + toff[i];
    const int64_t size = (int64_t)1 << tbits[i];
    u64 best = 0;
    for (int64_t s = threadIdx.x; s < size; s += 256) {
      const u64 x = T[s];
      if (x != EMPTY) {
        const u64 kk = entry_key(x);
        best = kk > best ? kk : best;
        T[s] = EMPTY;  // leave the table clean for the next sweep
      }
    }
    best = group_max<64>(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    best = red[0];
    for (int k = 1; k < 4; ++k) best = red[k] > best ? red[k] : best;
    const int64_t b = a.off[v], e = a.off[v + 1];
    if (best != 0) {
      const int32_t cs = (int32_t)key_label(best);
      if (cs != a.C[v]) {
        __syncthreads();
        if (threadIdx.x == 0) {
          a.C[v] = cs;
          ++n_changed;
        }
        if (a.prune)
          for (int64_t k = b + threadIdx.x; k < e; k += 256) {
            const int j = a.idx[k];
            if (j != v) a.F[j] = 1;
          }
      }
    }
    if (threadIdx.x == 0) n_scanned += (u64)(e - b);
    __syncthreads();
  }
  block_add3<256>(n_changed, n_scanned, 0, a.ctl);
}

// ---------------------------------------------------------------- launchers

static void launch_group_bin(int bin, int wk, dim3 grid, hipStream_t st, const ScanArgs &a) {
#define GVELPA_GROUP_CASE(B, G, S)                                                            \
  case B:                                                                                     \
    if (wk == W_UNIT) hipLaunchKernelGGL((k_scan_group<G, S, W_UNIT>), grid, dim3(256), 0, st, a); \
    else if (wk == W_U8) hipLaunchKernelGGL((k_scan_group<G, S, W_U8>), grid, dim3(256), 0, st, a); \
    else hipLaunchKernelGGL((k_scan_group<G, S, W_U32>), grid, dim3(256), 0, st, a);             \
    break;
  switch (bin) {
    GVELPA_GROUP_CASE(0, 8, 16)
    GVELPA_GROUP_CASE(1, 16, 64)
    GVELPA_GROUP_CASE(2, 64, 256)
    default: break;
  }
#undef GVELPA_GROUP_CASE
}

static void launch_block_bin(int bin, int wk, dim3 grid, hipStream_t st, const ScanArgs &a) {
#define GVELPA_BLOCK_CASE(B, BS, S)                                                             \
  case B:                                                                                       \
    if (wk == W_UNIT) hipLaunchKernelGGL((k_scan_block<BS, S, W_UNIT>), grid, dim3(BS), 0, st, a); \
    else if (wk == W_U8) hipLaunchKernelGGL((k_scan_block<BS, S, W_U8>), grid, dim3(BS), 0, st, a); \
    else hipLaunchKernelGGL((k_scan_block<BS, S, W_U32>), grid, dim3(BS), 0, st, a);             \
    break;
  switch (bin) {
    GVELPA_BLOCK_CASE(3, 256, 1024)
    GVELPA_BLOCK_CASE(4, 256, 4096)
    GVELPA_BLOCK_CASE(5, 512, 8192)
    default: break;
  }
#undef GVELPA_BLOCK_CASE
}

static_assert(BIN_GROUP[0] == 8 && BIN_SLOTS[0] == 16, "bin table and launcher disagree");
static_assert(BIN_GROUP[1] == 16 && BIN_SLOTS[1] == 64, "bin table and launcher disagree");
static_assert(BIN_GROUP[2] == 64 && BIN_SLOTS[2] == 256, "bin table and launcher disagree");
static_assert(BIN_GROUP[3] == 256 && BIN_SLOTS[3] == 1024, "bin table and launcher disagree");
static_assert(BIN_GROUP[4] == 256 && BIN_SLOTS[4] == 4096, "bin table and launcher disagree");
static_assert(BIN_GROUP[5] == 512 && BIN_SLOTS[5] == 8192, "bin table and launcher disagree");

void launch_compact(const CompactArgs &a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, st, a);
}

void launch_scan_bin(int bin, int wk, int blocks, hipStream_t st, const ScanArgs &a) {
  if (bin <= 2) launch_group_bin(bin, wk, dim3(blocks), st, a);
  else launch_block_bin(bin, wk, dim3(blocks), st, a);
}

void launch_hub_plan(const ScanArgs &a, u64 *cstart, int64_t *toff, int32_t *tbits, hipStream_t st) {
  hipLaunchKernelGGL(k_hub_plan, dim3(1), dim3(1024), 0, st, a, cstart, toff, tbits);
}

void launch_hub_scan(int wk, int blocks, hipStream_t st, const ScanArgs &a, const u64 *cstart, const int64_t *toff,
                     const int32_t *tbits) {
  if (wk == W_UNIT) hipLaunchKernelGGL(k_hub_scan<W_UNIT>, dim3(blocks), dim3(256), 0, st, a, cstart, toff, tbits);
  else if (wk == W_U8) hipLaunchKernelGGL(k_hub_scan<W_U8>, dim3(blocks), dim3(256), 0, st, a, cstart, toff, tbits);
  else hipLaunchKernelGGL(k_hub_scan<W_U32>, dim3(blocks), dim3(256), 0, st, a, cstart, toff, tbits);
}

void launch_hub_finish(int blocks, hipStream_t st, const ScanArgs &a, const int64_t *toff, const int32_t *tbits) {
  hipLaunchKernelGGL(k_hub_finish, dim3(blocks), dim3(256), 0, st, a, toff, tbits);
}

void launch_init_state(const int64_t *off, int32_t *C, uint8_t *F, int64_t n, int set_labels, int set_flags,
                       int clear_isolated, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, st, off, C, F, n, set_labels, set_flags,
                     clear_isolated);
}

void launch_run_begin(Ctl *ctl, double tau, int max_iters, int64_t n, int32_t *fcount, int nfc, int32_t *host_done,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_run_begin, dim3(1), dim3(256), 0, st, ctl, tau, max_iters, n, fcount, nfc, host_done);
}

void launch_end_sweep(Ctl *ctl, int32_t *fcount, int nfc, int32_t *host_done, hipStream_t st) {
  hipLaunchKernelGGL(k_end_sweep, dim3(1), dim3(256), 0, st, ctl, fcount, nfc, host_done);
}

}  // namespace gvelpa
