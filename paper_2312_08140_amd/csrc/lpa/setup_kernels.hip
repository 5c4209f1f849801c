// One-off kernels run when a graph is created or first used in a mode:
// CSR validation, weight packing, weighted degrees, degree binning and the
// Jones-Plassmann colouring of the deterministic mode.
#include <math.h>

#include "sweep_kernels.hpp"

namespace gvelpa {

static int grid_for(int64_t items, int per_block, int cap = 8192) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// ---------------------------------------------------------------- validation

__global__ void k_check_offsets(const int64_t *off, int64_t n, CsrCheck *chk) {
  int bad = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    bad |= off[v + 1] < off[v];
  if (bad) atomicOr(&chk->bad_offsets, 1);
}

__global__ void k_check_edges(const int32_t *idx, const float *w, int64_t m, int64_t n, CsrCheck *chk) {
  int bad_i = 0, bad_w = 0, not_one = 0;
  uint32_t wmax = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = idx[e];
    bad_i |= (j < 0) | ((int64_t)j >= n);
    if (w) {
      const float x = w[e];
      const bool ok = (x >= 0.0f) && (x <= 16777216.0f) && (floorf(x) == x);
      bad_w |= !ok;
      if (ok) {
        const uint32_t u = (uint32_t)x;
        wmax = u > wmax ? u : wmax;
        not_one |= u != 1u;
      }
    }
  }
  if (bad_i) atomicOr(&chk->bad_index, 1);
  if (bad_w) atomicOr(&chk->bad_weight, 1);
  if (not_one) atomicOr(&chk->not_all_ones, 1);
  if (wmax) atomicMax(&chk->max_weight, wmax);
}

// Flags a row whose neighbours are not strictly increasing: one wave per row.
__global__ __launch_bounds__(256) void k_check_rows(const int64_t *off, const int32_t *idx, int64_t n, CsrCheck *chk) {
  const int lane = threadIdx.x & 63;
  int bad = 0;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4)
    for (int64_t k = off[r] + lane; k + 1 < off[r + 1]; k += 64) bad |= idx[k] >= idx[k + 1];
  if (bad) atomicOr(&chk->rows_not_strict, 1);
}

__global__ void k_convert_weights(const float *w, int64_t m, int wk, void *out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = (uint32_t)w[e];
    if (wk == W_U8) ((uint8_t *)out)[e] = (uint8_t)u;
    else ((uint32_t *)out)[e] = u;
  }
}

// K_v = summed stored weights of row v (64-bit sums; a sum >= 2^32 is
// reported).  Rows are read with coalesced loads whatever their lengths:
//  * a wave takes 64 consecutive vertices; when their rows hold at most
//    WD_TILE entries together, the wave streams that entry range 64 entries at
//    a time, finds the row of every entry by a binary search over the 64 row
//    starts (held one per lane), adds the weights of each row's run of lanes
//    with a segmented scan, and the last lane of each run adds the run's sum
//    into the row's accumulator in LDS;
//  * otherwise each row of at most 64 entries is summed by its own lane and
//    each longer one, up to WD_BIG entries, by the whole wave;
//  * rows of more than WD_BIG entries are set to 0 here and summed by
//    k_weighted_degree_big in chunks of WD_BIG entries added with atomics.
constexpr int WD_TILE = 4096;
constexpr int64_t WD_BIG = 65536;

template <int WK>
__global__ __launch_bounds__(256) void k_weighted_degree(const int64_t *off, const void *w, int64_t n, uint32_t *K,
                                                         CsrCheck *chk) {
  __shared__ u64 s_acc[4][64];
  int big = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t base = ((int64_t)blockIdx.x * 4 + wv) * 64; base < n; base += waves * 64) {
    const int64_t v = base + lane;
    const int cnt = (int)min((int64_t)64, n - base);  // vertices of the tile
    int64_t b = 0, e = 0;
    if (v < n) {
      b = off[v];
      e = off[v + 1];
    }
    if constexpr (WK == W_UNIT) {
      if (v < n) {
        big |= (u64)(e - b) >= (1ull << 32);
        K[v] = (uint32_t)(e - b);
      }
      continue;
    }
    const int64_t E0 = __shfl(b, 0, 64), E1 = __shfl(e, cnt - 1, 64);
    u64 s = 0;
    if (E1 - E0 <= WD_TILE) {
      const int rb = v < n ? (int)(b - E0) : WD_TILE + 1;  // row start relative to the tile
      s_acc[wv][lane] = 0;
      for (int64_t x0 = E0; x0 < E1; x0 += 64) {
        const int64_t x = x0 + lane;
        const bool ok = x < E1;
        const uint32_t wt = ok ? load_w<WK>(w, x) : 0u;
        // the last row whose start is <= x (rows with no entry start where the next one does)
        const int rx = (int)(x - E0);
        int row = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const int cand = row + step;  // <= 63
          const int start = __shfl(rb, cand, 64);
          if (cand < cnt && start <= rx) row = cand;
        }
        if (!ok) row = 64;  // lanes past the tile form no run with a row
        // inclusive scan of the weights within each run of equal rows (64 * 2^24 < 2^32)
        uint32_t run = wt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t o = __shfl_up(run, d, 64);
          const int orow = __shfl_up(row, d, 64);
          if (lane >= d && orow == row) run += o;
        }
        const int next = __shfl_down(row, 1, 64);
        if (ok && (lane == 63 || next != row)) s_acc[wv][row] += run;  // one last lane per row
      }
      s = s_acc[wv][lane];
    } else {
      const bool longrow = e - b > 64;
      if (!longrow)
        for (int64_t k = b; k < e; ++k) s += load_w<WK>(w, k);
      u64 mask = __ballot(longrow && e - b <= WD_BIG);
      while (mask) {
        const int src = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int64_t bb = __shfl(b, src, 64), ee = __shfl(e, src, 64);
        u64 part = 0;
        int64_t k = bb + lane;
        for (; k + 192 < ee; k += 256)
          part += (u64)load_w<WK>(w, k) + load_w<WK>(w, k + 64) + load_w<WK>(w, k + 128) +
                  load_w<WK>(w, k + 192);
        for (; k < ee; k += 64) part += load_w<WK>(w, k);
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) part += shfl_xor_u64(part, m);
        if (lane == src) s = part;
      }
    }
    if (v < n) {
      big |= s >= (1ull << 32);
      K[v] = e - b > WD_BIG ? 0u : (uint32_t)s;
    }
  }
  if (big) atomicOr(&chk->big_degree, 1);
}

// The rows of more than WD_BIG entries: chunk c of the entries, [c * WD_BIG,
// (c + 1) * WD_BIG), meets at most two such rows (the ones holding its first
// and its last entry; any row between them lies inside the chunk).  Each
// part is summed by the workgroup and added to K with a 32-bit atomic; a part
// or a running sum that reaches 2^32 is reported.
template <int WK>
__global__ __launch_bounds__(256) void k_weighted_degree_big(const int64_t *off, const void *w, int64_t n,
                                                             uint32_t *K, CsrCheck *chk) {
  __shared__ u64 s_red[4];
  __shared__ int64_t s_rows[2];
  const int64_t m = off[n];
  const int64_t chunks = (m + WD_BIG - 1) / WD_BIG;
  for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    const int64_t c0 = c * WD_BIG, c1 = min(m, c0 + WD_BIG);
    if (threadIdx.x < 2) {
      // the row holding entry x: the last r with off[r] <= x (off[n] = m > x)
      const int64_t x = threadIdx.x == 0 ? c0 : c1 - 1;
      int64_t lo = 0, hi = n;  // off[lo] <= x < off[hi]
      while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
      }
      s_rows[threadIdx.x] = lo;
    }
    __syncthreads();
    const int64_t r0 = s_rows[0], r1 = s_rows[1];
    __syncthreads();  // s_rows is rewritten by the next chunk
    for (int q = 0; q < 2; ++q) {
      const int64_t r = q == 0 ? r0 : r1;
      if (q == 1 && r1 == r0) break;
      const int64_t rb = off[r], re = off[r + 1];
      if (re - rb <= WD_BIG) continue;  // uniform across the workgroup
      const int64_t a = max(rb, c0), z = min(re, c1);
      u64 part = 0;
      for (int64_t k = a + threadIdx.x; k < z; k += 256) part += load_w<WK>(w, k);
#pragma unroll
      for (int mm = 32; mm > 0; mm >>= 1) part += shfl_xor_u64(part, mm);
      if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = part;
      __syncthreads();
      if (threadIdx.x == 0) {
        const u64 t = s_red[0] + s_red[1] + s_red[2] + s_red[3];
        bool over = t >= (1ull << 32);
        if (!over) over = (u64)atomicAdd(&K[r], (uint32_t)t) + t >= (1ull << 32);
        if (over) atomicOr(&chk->big_degree, 1);
      }
      __syncthreads();  // s_red is reused by the next part
    }
  }
}

// Multiset fingerprint of (i, j, w) against (j, i, w): equal sums for a
// symmetric graph; any asymmetry changes them with probability ~1 - 2^-64.
__device__ __forceinline__ u64 mix64(u64 z) {  // SplitMix64 output function
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int WK>
__global__ void k_check_symmetric(const int64_t *off, const int32_t *idx, const void *w, int64_t n, u64 *sums) {
  u64 fwd = 0, bwd = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t k = off[v]; k < off[v + 1]; ++k) {
      const u64 j = (uint32_t)idx[k];
      const u64 x = load_w<WK>(w, k);
      fwd += mix64(((u64)v << 32 | j) ^ mix64(x + 0x9E3779B97F4A7C15ull));
      bwd += mix64((j << 32 | (u64)v) ^ mix64(x + 0x9E3779B97F4A7C15ull));
    }
  }
  atomicAdd(&sums[0], fwd);
  atomicAdd(&sums[1], bwd);
}

// Batched handles: no stored entry may join two graphs.
__global__ void k_check_block_diagonal(const int64_t *off, const int32_t *idx, const int32_t *gid, int64_t n,
                                       int32_t *bad) {
  int b = 0;
  for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < n; v += (int64_t)gridDim.x * 4)
    for (int64_t k = off[v] + (threadIdx.x & 63); k < off[v + 1]; k += 64) b |= gid[idx[k]] != gid[v];
  if (b) atomicOr(bad, 1);
}

// ---------------------------------------------------------------- binning

// Key of a vertex: its degree bin, prefixed by its colour in deterministic
// lists; vertices without stored entries are never processed and get no key.
// Counting is privatised in LDS (one global atomic per block and key) when
// the key range fits; each block takes tiles of BIN_TILE consecutive ids.
constexpr int BIN_TILE = 4096;
constexpr int BIN_LDS_KEYS = 16384;

// Group of a vertex in the list order: its colour (deterministic lists), or
// its asynchronous phase fmix32(v ^ PHASE_SEED) mod nphase (async lists).
constexpr uint32_t PHASE_SEED = 0x2545F491u;

// With a colour map cmap, the group is cmap[colour] (asynchronous steps made
// of consecutive colour classes).
__device__ __forceinline__ int vertex_key(const int64_t *off, const int32_t *color, const int32_t *cmap, int nphase,
                                          const BinLimits &lim, int64_t v) {
  const int64_t deg = off[v + 1] - off[v];
  if (deg == 0) return -1;
  int grp;
  if (color) grp = cmap ? cmap[color[v]] : color[v];
  else grp = nphase > 1 ? (int)(fmix32((uint32_t)v ^ PHASE_SEED) % (uint32_t)nphase) : 0;
  return grp * NBINS + bin_of_degree(deg, lim);
}

__global__ __launch_bounds__(256) void k_bin_hist(const int64_t *off, int64_t n, const int32_t *color,
                                                  const int32_t *cmap, int nphase, BinLimits lim, int32_t *hist,
                                                  int nkeys) {
  extern __shared__ int32_t lh[];
  const bool local = nkeys <= BIN_LDS_KEYS;
  if (local) {
    for (int k = threadIdx.x; k < nkeys; k += 256) lh[k] = 0;
    __syncthreads();
  }
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
    const int key = vertex_key(off, color, cmap, nphase, lim, v);
    if (key >= 0) atomicAdd(local ? &lh[key] : &hist[key], 1);
  }
  if (local) {
    __syncthreads();
    for (int k = threadIdx.x; k < nkeys; k += 256)
      if (lh[k]) atomicAdd(&hist[k], lh[k]);
  }
}

__global__ __launch_bounds__(256) void k_bin_scatter(const int64_t *off, int64_t n, const int32_t *color,
                                                     const int32_t *cmap, int nphase, BinLimits lim, int32_t *cursor,
                                                     int32_t *list, int nkeys) {
  extern __shared__ int32_t lh[];  // [0, nkeys): tile counts, then tile bases
  const bool local = 2 * nkeys <= BIN_LDS_KEYS;
  if (!local) {
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
      const int key = vertex_key(off, color, cmap, nphase, lim, v);
      if (key >= 0) list[atomicAdd(&cursor[key], 1)] = (int32_t)v;
    }
    return;
  }
  int32_t *cnt = lh, *base = lh + nkeys;
  for (int64_t t0 = (int64_t)blockIdx.x * BIN_TILE; t0 < n; t0 += (int64_t)gridDim.x * BIN_TILE) {
    for (int k = threadIdx.x; k < nkeys; k += 256) cnt[k] = 0;
    __syncthreads();
    int key[BIN_TILE / 256], pos[BIN_TILE / 256];
#pragma unroll
    for (int r = 0; r < BIN_TILE / 256; ++r) {
      const int64_t v = t0 + r * 256 + threadIdx.x;
      key[r] = v < n ? vertex_key(off, color, cmap, nphase, lim, v) : -1;
      pos[r] = key[r] >= 0 ? atomicAdd(&cnt[key[r]], 1) : 0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nkeys; k += 256)
      if (cnt[k]) base[k] = atomicAdd(&cursor[k], cnt[k]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < BIN_TILE / 256; ++r)
      if (key[r] >= 0) list[base[key[r]] + pos[r]] = (int32_t)(t0 + r * 256 + threadIdx.x);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- colouring

// Priority of vertex id v: (deg(v), fmix32(v ^ seed), v) in lexicographic
// order; the first two parts are packed in pk = deg << 32 | fmix32(v ^ seed).
// Kernels index vertices by storage position; orig[p] (NULL: p) is the id.
__device__ __forceinline__ bool higher(u64 pu, int u, u64 pv, int v, const int32_t *orig) {
  if (pu != pv) return pu > pv;
  return orig ? orig[u] > orig[v] : u > v;
}

__global__ void k_color_prio(const int64_t *off, int32_t *color, u64 *pk, int64_t n, uint32_t seed,
                             const int32_t *orig) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    color[v] = -1;
    const uint32_t id = orig ? (uint32_t)orig[v] : (uint32_t)v;
    pk[v] = ((u64)(off[v + 1] - off[v]) << 32) | fmix32(id ^ seed);
  }
}

// Jones-Plassmann, event driven.  pending[v] counts the neighbours of higher
// priority that are not yet coloured; a vertex whose count reaches zero is
// coloured in the next round with the smallest colour unused by its coloured
// neighbours - exactly its higher-priority neighbours - which is the greedy
// colouring in decreasing priority.  One wave per vertex.
__global__ __launch_bounds__(256) void k_color_pending(const int64_t *off, const int32_t *idx, const u64 *pk,
                                                       int32_t *pending, int32_t *front, int32_t *count, int64_t n,
                                                       const int32_t *orig) {
  const int lane = threadIdx.x & 63;
  for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < n; v += (int64_t)gridDim.x * 4) {
    const u64 pv = pk[v];
    int c = 0;
    for (int64_t k = off[v] + lane; k < off[v + 1]; k += 64) {
      const int u = idx[k];
      c += (u != (int)v && higher(pk[u], u, pv, (int)v, orig)) ? 1 : 0;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m, 64);
    if (lane == 0) {
      pending[v] = c;
      if (c == 0) front[atomicAdd(count, 1)] = (int32_t)v;
    }
  }
}

__global__ __launch_bounds__(256) void k_color_round(const int64_t *off, const int32_t *idx, int32_t *color,
                                                     const u64 *pk, int32_t *pending, const int32_t *work_in,
                                                     int32_t *work_out, int32_t *counts, int r, const int32_t *orig) {
  constexpr int WINDOW = 64 * 32;  // colours tested per pass: one 32-bit word per lane
  __shared__ uint32_t bits_all[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t *bits = bits_all[wv];
  const int gw = blockIdx.x * 4 + wv, nw = gridDim.x * 4;
  const int wlen = counts[r];
  for (int i = gw; i < wlen; i += nw) {
    const int v = work_in[i];
    const int64_t b = off[v], e = off[v + 1];
    int base = 0, found = -1;
    while (found < 0) {
      bits[lane] = 0;
      wave_lds_sync();
      for (int64_t k = b + lane; k < e; k += 64) {
        const int u = idx[k];
        if (u == v) continue;
        const int c = __atomic_load_n(&color[u], __ATOMIC_RELAXED) - base;
        if (c >= 0 && c < WINDOW) atomicOr(&bits[c >> 5], 1u << (c & 31));
      }
      wave_lds_sync();
      const uint32_t free_bits = ~bits[lane];
      int pos = free_bits ? lane * 32 + __builtin_ctz(free_bits) : 0x7FFFFFFF;
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) {
        const int o = __shfl_xor(pos, m, 64);
        pos = o < pos ? o : pos;
      }
      if (pos != 0x7FFFFFFF) found = base + pos;
      else base += WINDOW;
      wave_lds_sync();
    }
    if (lane == 0) __atomic_store_n(&color[v], found, __ATOMIC_RELAXED);
    // release the lower-priority neighbours
    const u64 pv = pk[v];
    for (int64_t k = b + lane; k < e; k += 64) {
      const int u = idx[k];
      if (u != v && higher(pv, v, pk[u], u, orig) && atomicSub(&pending[u], 1) == 1)
        work_out[atomicAdd(&counts[r + 1], 1)] = u;
    }
  }
}

// ---------------------------------------------------------------- launchers

void launch_check_offsets(const int64_t *off, int64_t n, CsrCheck *chk, hipStream_t st) {
  hipLaunchKernelGGL(k_check_offsets, dim3(grid_for(n, 256)), dim3(256), 0, st, off, n, chk);
}
void launch_check_edges(const int32_t *idx, const float *w, int64_t m, int64_t n, CsrCheck *chk, hipStream_t st) {
  hipLaunchKernelGGL(k_check_edges, dim3(grid_for(m, 256)), dim3(256), 0, st, idx, w, m, n, chk);
}
void launch_check_rows(const int64_t *off, const int32_t *idx, int64_t n, CsrCheck *chk, hipStream_t st) {
  hipLaunchKernelGGL(k_check_rows, dim3(grid_for(n, 4)), dim3(256), 0, st, off, idx, n, chk);
}
void launch_convert_weights(const float *w, int64_t m, int wk, void *out, hipStream_t st) {
  hipLaunchKernelGGL(k_convert_weights, dim3(grid_for(m, 256)), dim3(256), 0, st, w, m, wk, out);
}
void launch_weighted_degree(const int64_t *off, const void *w, int wk, int64_t n, uint32_t *K, CsrCheck *chk,
                            hipStream_t st) {
  dim3 g(grid_for(n, 256, 8192)), b(256), gb(8192);
  if (wk == W_UNIT) {
    hipLaunchKernelGGL(k_weighted_degree<W_UNIT>, g, b, 0, st, off, w, n, K, chk);
  } else if (wk == W_U8) {
    hipLaunchKernelGGL(k_weighted_degree<W_U8>, g, b, 0, st, off, w, n, K, chk);
    hipLaunchKernelGGL(k_weighted_degree_big<W_U8>, gb, b, 0, st, off, w, n, K, chk);
  } else {
    hipLaunchKernelGGL(k_weighted_degree<W_U32>, g, b, 0, st, off, w, n, K, chk);
    hipLaunchKernelGGL(k_weighted_degree_big<W_U32>, gb, b, 0, st, off, w, n, K, chk);
  }
}
void launch_check_symmetric(const int64_t *off, const int32_t *idx, const void *w, int wk, int64_t n,
                            CsrCheck *chk, hipStream_t st) {
  // chk->asym is set by the host from the two sums written after the CsrCheck block
  u64 *sums = (u64 *)(chk + 1);
  dim3 g(grid_for(n, 256)), b(256);
  if (wk == W_UNIT) hipLaunchKernelGGL(k_check_symmetric<W_UNIT>, g, b, 0, st, off, idx, w, n, sums);
  else if (wk == W_U8) hipLaunchKernelGGL(k_check_symmetric<W_U8>, g, b, 0, st, off, idx, w, n, sums);
  else hipLaunchKernelGGL(k_check_symmetric<W_U32>, g, b, 0, st, off, idx, w, n, sums);
}
void launch_bin_hist(const int64_t *off, int64_t n, const int32_t *color, const int32_t *cmap, int nphase,
                     const BinLimits &lim, int32_t *hist, int nkeys, hipStream_t st) {
  const size_t lds = nkeys <= BIN_LDS_KEYS ? sizeof(int32_t) * nkeys : 0;
  hipLaunchKernelGGL(k_bin_hist, dim3(grid_for(n, 256, 2048)), dim3(256), lds, st, off, n, color, cmap, nphase, lim,
                     hist, nkeys);
}
void launch_bin_scatter(const int64_t *off, int64_t n, const int32_t *color, const int32_t *cmap, int nphase,
                        const BinLimits &lim, int32_t *cursor, int32_t *list, int nkeys, hipStream_t st) {
  const size_t lds = 2 * nkeys <= BIN_LDS_KEYS ? sizeof(int32_t) * 2 * nkeys : 0;
  hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(n, BIN_TILE, 4096)), dim3(256), lds, st, off, n, color, cmap, nphase,
                     lim, cursor, list, nkeys);
}
uint32_t phase_seed() { return PHASE_SEED; }

__global__ void k_gather_at(const int32_t *idx, const int64_t *at, int64_t count, int32_t *out) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < count; c += (int64_t)gridDim.x * blockDim.x)
    out[c] = idx[at[c]];
}
void launch_gather_at(const int32_t *idx, const int64_t *at, int64_t count, int32_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_at, dim3(grid_for(count, 256)), dim3(256), 0, st, idx, at, count, out);
}

void launch_check_block_diagonal(const int64_t *off, const int32_t *idx, const int32_t *gid, int64_t n, int32_t *bad,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_check_block_diagonal, dim3(grid_for(n, 4, 16384)), dim3(256), 0, st, off, idx, gid, n, bad);
}

void launch_color_init(const int64_t *off, const int32_t *idx, int32_t *color, u64 *pk, int32_t *pending,
                       int32_t *front, int32_t *count, int64_t n, uint32_t seed, const int32_t *orig,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_color_prio, dim3(grid_for(n, 256)), dim3(256), 0, st, off, color, pk, n, seed, orig);
  hipLaunchKernelGGL(k_color_pending, dim3(grid_for(n, 4, 16384)), dim3(256), 0, st, off, idx, pk, pending, front,
                     count, n, orig);
}
void launch_color_round(const int64_t *off, const int32_t *idx, int32_t *color, const u64 *pk, int32_t *pending,
                        const int32_t *work_in, int32_t *work_out, int32_t *counts, int r, int blocks,
                        const int32_t *orig, hipStream_t st) {
  hipLaunchKernelGGL(k_color_round, dim3(blocks), dim3(256), 0, st, off, idx, color, pk, pending, work_in, work_out,
                     counts, r, orig);
}

}  // namespace gvelpa
