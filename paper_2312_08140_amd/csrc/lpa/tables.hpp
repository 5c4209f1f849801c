// LDS open-addressing tables (label -> summed weight) and block reductions
// shared by the scan kernels.
#pragma once
#include "common.hpp"

namespace gvelpa {

// Adds weight w to label lbl in a table of 2^BITS entries (linear probing).
// Entry s of the table lives at T[s * STRIDE] (tables of several groups are
// interleaved so that neighbouring lanes hit neighbouring LDS banks).
// Returns false only if every slot holds another label.
template <int BITS, int STRIDE = 1>
__device__ __forceinline__ bool lds_insert(u64 *T, uint32_t lbl, uint32_t w) {
  constexpr uint32_t MASK = (1u << BITS) - 1;
  uint32_t h = slot_hash(lbl, BITS);
  const u64 mine = ((u64)lbl << 32) | w;
  for (int probe = 0; probe <= (int)MASK; ++probe) {
    u64 *slot = &T[h * STRIDE];
    const u64 cur = __atomic_load_n(slot, __ATOMIC_RELAXED);
    if ((uint32_t)(cur >> 32) == lbl) {
      atomicAdd(slot, (u64)w);
      return true;
    }
    if (cur == EMPTY) {
      const u64 old = atomicCAS(slot, EMPTY, mine);
      if (old == EMPTY) return true;
      if ((uint32_t)(old >> 32) == lbl) {
        atomicAdd(slot, (u64)w);
        return true;
      }
    }
    h = (h + 1) & MASK;
  }
  return false;
}

// lds_insert for a table of 2^bits entries chosen at run time.
__device__ __forceinline__ bool lds_insert_rt(u64 *T, int bits, uint32_t lbl, uint32_t w) {
  const uint32_t mask = (1u << bits) - 1;
  uint32_t h = slot_hash(lbl, bits);
  const u64 mine = ((u64)lbl << 32) | w;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    u64 *slot = &T[h];
    const u64 cur = __atomic_load_n(slot, __ATOMIC_RELAXED);
    if ((uint32_t)(cur >> 32) == lbl) {
      atomicAdd(slot, (u64)w);
      return true;
    }
    if (cur == EMPTY) {
      const u64 old = atomicCAS(slot, EMPTY, mine);
      if (old == EMPTY) return true;
      if ((uint32_t)(old >> 32) == lbl) {
        atomicAdd(slot, (u64)w);
        return true;
      }
    }
    h = (h + 1) & mask;
  }
  return false;
}

// Gathers the labels of the entries [b, e) of row v, lanes lane, lane+G, ...,
// U entries per lane in flight, and adds them to table T.  The vertex itself
// is skipped (scanCommunities of Algorithm 1).
template <int G, int U, int BITS, int WK>
__device__ __forceinline__ int scan_row(const int32_t *__restrict__ idx, const void *__restrict__ w,
                                        const int32_t *C, int64_t b, int64_t e, int v, int lane, u64 *T) {
  int overflow = 0;
  for (int64_t base = b + lane; base < e; base += (int64_t)G * U) {
    int j[U];
    uint32_t wt[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t k = base + (int64_t)r * G;
      j[r] = k < e ? idx[k] : -1;
      wt[r] = k < e ? load_w<WK>(w, k) : 0u;
    }
    uint32_t lbl[U];
#pragma unroll
    for (int r = 0; r < U; ++r) lbl[r] = (j[r] >= 0 && j[r] != v) ? (uint32_t)C[j[r]] : 0xFFFFFFFFu;
#pragma unroll
    for (int r = 0; r < U; ++r)
      if (lbl[r] != 0xFFFFFFFFu) overflow |= !lds_insert<BITS>(T, lbl[r], wt[r]);
  }
  return overflow;
}

// scan_row for an interleaved table (entry s at T[s * STRIDE]).
template <int G, int U, int BITS, int STRIDE, int WK>
__device__ __forceinline__ int scan_row_strided(const int32_t *__restrict__ idx, const void *__restrict__ w,
                                                const int32_t *C, int64_t b, int64_t e, int v, int lane, u64 *T) {
  int overflow = 0;
  for (int64_t base = b + lane; base < e; base += (int64_t)G * U) {
    int j[U];
    uint32_t wt[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t k = base + (int64_t)r * G;
      j[r] = k < e ? idx[k] : -1;
      wt[r] = k < e ? load_w<WK>(w, k) : 0u;
    }
    uint32_t lbl[U];
#pragma unroll
    for (int r = 0; r < U; ++r) lbl[r] = (j[r] >= 0 && j[r] != v) ? (uint32_t)C[j[r]] : 0xFFFFFFFFu;
#pragma unroll
    for (int r = 0; r < U; ++r)
      if (lbl[r] != 0xFFFFFFFFu) overflow |= !lds_insert<BITS, STRIDE>(T, lbl[r], wt[r]);
  }
  return overflow;
}

// Flags the neighbours of v (not v itself) for the next visit; returns the
// number of marks written.
template <int G, int U>
__device__ __forceinline__ u64 mark_row(const int32_t *__restrict__ idx, uint8_t *F, int64_t b, int64_t e, int v,
                                        int lane) {
  u64 marks = 0;
  for (int64_t base = b + lane; base < e; base += (int64_t)G * U) {
    int j[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t k = base + (int64_t)r * G;
      j[r] = k < e ? idx[k] : -1;
    }
    uint8_t f[U];
#pragma unroll
    for (int r = 0; r < U; ++r) f[r] = (j[r] >= 0 && j[r] != v) ? F[j[r]] : (uint8_t)1;
#pragma unroll
    for (int r = 0; r < U; ++r) {
      marks += (j[r] >= 0 && j[r] != v) ? 1 : 0;
      if (!f[r]) F[j[r]] = 1;  // a flag already set is not written again
    }
  }
  return marks;
}

// Largest argmax key among the slots lane, lane+G, ... of T (tie rule t).
template <int G, int SLOTS, int STRIDE = 1>
__device__ __forceinline__ u64 table_best(const u64 *T, int lane, TieRule t) {
  u64 best = 0;
#pragma unroll 4
  for (int s = lane; s < SLOTS; s += G) {
    const u64 x = T[s * STRIDE];
    if (x != EMPTY) {
      const u64 kk = entry_key(x, t);
      best = kk > best ? kk : best;
    }
  }
  return best;
}

// table_best over the first `slots` entries of T (a size chosen at run time).
template <int G>
__device__ __forceinline__ u64 table_best_rt(const u64 *T, int slots, int lane, TieRule t) {
  u64 best = 0;
  for (int s = lane; s < slots; s += G) {
    const u64 x = T[s];
    if (x != EMPTY) {
      const u64 kk = entry_key(x, t);
      best = kk > best ? kk : best;
    }
  }
  return best;
}

// ---------------------------------------------------------------- gate features

// Top-2 label weights and distinct labels among the slots lane, lane+G, ...
struct TabStats {
  uint32_t w1, w2;
  int nd;
};

template <int G, int SLOTS, int STRIDE = 1>
__device__ __forceinline__ TabStats table_stats(const u64 *T, int lane) {
  TabStats r{0u, 0u, 0};
  for (int s = lane; s < SLOTS; s += G) {
    const u64 x = T[s * STRIDE];
    if (x != EMPTY) {
      const uint32_t w = (uint32_t)x;
      ++r.nd;
      if (w > r.w1) {
        r.w2 = r.w1;
        r.w1 = w;
      } else if (w > r.w2) {
        r.w2 = w;
      }
    }
  }
  return r;
}

template <int G>
__device__ __forceinline__ TabStats table_stats_rt(const u64 *T, int slots, int lane) {
  TabStats r{0u, 0u, 0};
  for (int s = lane; s < slots; s += G) {
    const u64 x = T[s];
    if (x != EMPTY) {
      const uint32_t w = (uint32_t)x;
      ++r.nd;
      if (w > r.w1) {
        r.w2 = r.w1;
        r.w1 = w;
      } else if (w > r.w2) {
        r.w2 = w;
      }
    }
  }
  return r;
}

// table_best and table_stats in one pass over the slots.
template <int G, int SLOTS, int STRIDE = 1>
__device__ __forceinline__ u64 table_best_stats(const u64 *T, int lane, TabStats &r, TieRule t) {
  u64 best = 0;
  r = TabStats{0u, 0u, 0};
#pragma unroll 4
  for (int s = lane; s < SLOTS; s += G) {
    const u64 x = T[s * STRIDE];
    if (x != EMPTY) {
      const u64 kk = entry_key(x, t);
      best = kk > best ? kk : best;
      const uint32_t w = (uint32_t)x;
      ++r.nd;
      if (w > r.w1) {
        r.w2 = r.w1;
        r.w1 = w;
      } else if (w > r.w2) {
        r.w2 = w;
      }
    }
  }
  return best;
}

__device__ __forceinline__ TabStats merge_stats(TabStats a, TabStats b) {
  TabStats r;
  r.w1 = a.w1 > b.w1 ? a.w1 : b.w1;
  const uint32_t lo = a.w1 > b.w1 ? b.w1 : a.w1;
  const uint32_t m2 = a.w2 > b.w2 ? a.w2 : b.w2;
  r.w2 = lo > m2 ? lo : m2;
  r.nd = a.nd + b.nd;
  return r;
}

template <int WIDTH>
__device__ __forceinline__ TabStats group_stats(TabStats t) {
#pragma unroll
  for (int m = WIDTH / 2; m > 0; m >>= 1) {
    TabStats o;
    o.w1 = __shfl_xor(t.w1, m, 64);
    o.w2 = __shfl_xor(t.w2, m, 64);
    o.nd = __shfl_xor(t.nd, m, 64);
    t = merge_stats(t, o);
  }
  return t;
}

// Weight of label lbl in table T (0 if absent); read-only probe.
template <int BITS, int STRIDE = 1>
__device__ __forceinline__ uint32_t table_lookup(const u64 *T, uint32_t lbl) {
  constexpr uint32_t MASK = (1u << BITS) - 1;
  uint32_t h = slot_hash(lbl, BITS);
  for (int probe = 0; probe <= (int)MASK; ++probe) {
    const u64 x = T[h * STRIDE];
    if (x == EMPTY) return 0u;
    if ((uint32_t)(x >> 32) == lbl) return (uint32_t)x;
    h = (h + 1) & MASK;
  }
  return 0u;
}

// table_lookup for a table of 2^bits entries chosen at run time.
__device__ __forceinline__ uint32_t table_lookup_rt(const u64 *T, int bits, uint32_t lbl) {
  const uint32_t mask = (1u << bits) - 1;
  uint32_t h = slot_hash(lbl, bits);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const u64 x = T[h];
    if (x == EMPTY) return 0u;
    if ((uint32_t)(x >> 32) == lbl) return (uint32_t)x;
    h = (h + 1) & mask;
  }
  return 0u;
}

// Stores the features of processed vertex v (sweep s) and, when tracing,
// records the decision-time features it had before this processing together
// with whether it changed now.  K = weighted degree of v, lp = sweep of its
// last processing (both loaded ahead by the caller).
__device__ __forceinline__ void write_features(const FeatArgs &f, int v, int s, int64_t deg, TabStats t,
                                               uint32_t wown, bool changed, uint32_t K, int lp) {
  float *st = f.feat + (int64_t)v * FEAT_STRIDE;
  if (f.trace && lp >= 0 && lp < s) {
    const uint32_t hsh = fmix32((uint32_t)v * 0x9E3779B1u ^ (uint32_t)s * 0x85EBCA77u);
    if (hsh < f.tthresh) {
      const u64 pos = atomicAdd(f.tcount, (u64)1);
      if (pos < f.tcap) {
        float x[NFEAT];
        decision_features(st, lp, s, f.max_iters, x);
#pragma unroll
        for (int q = 0; q < NFEAT; ++q) f.tx[pos * NFEAT + q] = x[q];
        f.ty[pos] = changed ? 1 : 0;
      }
    }
  }
  // fast divisions (within 2 ulp): the features only steer a heuristic
  const float inv = K ? __fdividef(1.0f, (float)K) : 0.0f;
  float4 r0, r1;
  r0.x = log2f(1.0f + (float)deg);
  r0.y = (float)(t.w1 - t.w2) * inv;
  r0.z = (float)wown * inv;
  r0.w = changed ? 1.0f : 0.0f;
  r1.x = (float)t.w1 * inv;
  r1.y = deg ? __fdividef((float)t.nd, (float)deg) : 0.0f;
  r1.z = __int_as_float(s);
  r1.w = 0.0f;
  reinterpret_cast<float4 *>(st)[0] = r0;
  reinterpret_cast<float4 *>(st)[1] = r1;
}

// Block-wide maximum (every thread gets the result); red holds BLOCK/64 entries.
template <int BLOCK>
__device__ __forceinline__ u64 block_max(u64 x, u64 *red) {
  x = group_max<64>(x);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  x = red[0];
#pragma unroll
  for (int k = 1; k < BLOCK / 64; ++k) x = red[k] > x ? red[k] : x;
  return x;
}

// Block-wide sums of the per-thread counters (changed, scanned, vertices,
// marks), added to the block's shard of the bin's counters.
template <int BLOCK>
__device__ __forceinline__ void block_accum(u64 changed, u64 scanned, u64 vertices, u64 marks, int err, Ctl *ctl,
                                            int bin) {
  __shared__ u64 s_v[4][BLOCK / 64];
  __shared__ int s_err[BLOCK / 64];
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    changed += shfl_xor_u64(changed, m);
    scanned += shfl_xor_u64(scanned, m);
    vertices += shfl_xor_u64(vertices, m);
    marks += shfl_xor_u64(marks, m);
    err |= __shfl_xor(err, m, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_v[0][wv] = changed;
    s_v[1][wv] = scanned;
    s_v[2][wv] = vertices;
    s_v[3][wv] = marks;
    s_err[wv] = err;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    u64 t = 0;
    for (int k = 0; k < BLOCK / 64; ++k) t += s_v[threadIdx.x][k];
    if (t) atomicAdd(&ctl->shard[blockIdx.x & (NSHARD - 1)][bin].c[threadIdx.x], t);
  } else if (threadIdx.x == 4) {
    int te = 0;
    for (int k = 0; k < BLOCK / 64; ++k) te |= s_err[k];
    if (te) atomicOr(&ctl->error, te);
  }
}

}  // namespace gvelpa
