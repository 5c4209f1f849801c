// Modularity, Eq. (1) (Section 3.2), community form, in exact integers:
//   2m  = sum_v K_v             (K_v: summed stored weights of row v)
//   S1  = sum_c sigma_c         (stored weight with both endpoints in c)
//   S2  = sum_c Sigma_c^2       (Sigma_c = sum of K_v over v in c)
// Q = (S1 * 2m - S2) / (2m)^2 is formed on the host from these integers.
#include "sweep_kernels.hpp"

namespace gvelpa {

static int grid_for(int64_t items, int per_block, int cap = 8192) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

__global__ void k_check_labels(const int32_t *C, int64_t n, int32_t *bad) {
  int b = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    b |= (C[v] < 0) | ((int64_t)C[v] >= n);
  if (b) atomicOr(bad, 1);
}

// Sigma_c = sum of K_v over v in c.  Each workgroup first merges its
// vertices in an LDS table (label -> partial sum), so a community that
// spans the graph costs one global atomic per workgroup, not per vertex.
constexpr int TOT_SLOTS = 2048;

__global__ __launch_bounds__(256) void k_mod_community_totals(const int32_t *C, const uint32_t *K, int64_t n,
                                                              u64 *tot) {
  __shared__ uint32_t keys[TOT_SLOTS];
  __shared__ u64 vals[TOT_SLOTS];
  for (int s = threadIdx.x; s < TOT_SLOTS; s += 256) {
    keys[s] = 0xFFFFFFFFu;
    vals[s] = 0;
  }
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += (int64_t)gridDim.x * 256) {
    const uint32_t k = K[v];
    if (!k) continue;
    const uint32_t c = (uint32_t)C[v];
    uint32_t h = slot_hash(c, 11);
    bool done = false;
    for (int probe = 0; probe < 16 && !done; ++probe, h = (h + 1) & (TOT_SLOTS - 1)) {
      uint32_t cur = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
      if (cur == 0xFFFFFFFFu) cur = atomicCAS(&keys[h], 0xFFFFFFFFu, c) == 0xFFFFFFFFu ? c : keys[h];
      if (cur == c) {
        atomicAdd(&vals[h], (u64)k);
        done = true;
      }
    }
    if (!done) atomicAdd(&tot[c], (u64)k);  // table crowded: direct
  }
  __syncthreads();
  for (int s = threadIdx.x; s < TOT_SLOTS; s += 256)
    if (keys[s] != 0xFFFFFFFFu) atomicAdd(&tot[keys[s]], vals[s]);
}

// Edge-parallel pass: every block takes a contiguous range of stored entries
// and finds the row of its first entry by binary search over the offsets.
constexpr int MOD_EDGES_PER_BLOCK = 4096;

template <int WK>
__global__ __launch_bounds__(256) void k_mod_inside(const int64_t *off, const int32_t *idx, const void *w,
                                                    const int32_t *C, int64_t n, int64_t m, ModAcc *acc) {
  __shared__ u64 s_two_m[4], s_s1[4];
  __shared__ int64_t s_r[2];
  u64 two_m = 0, s1 = 0;
  auto row_of = [&](int64_t e, int64_t lo, int64_t hi) {  // r in [lo, hi) with off[r] <= e < off[r+1]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (off[mid] <= e) lo = mid;
      else hi = mid;
    }
    return lo;
  };
  for (int64_t e0 = (int64_t)blockIdx.x * MOD_EDGES_PER_BLOCK; e0 < m;
       e0 += (int64_t)gridDim.x * MOD_EDGES_PER_BLOCK) {
    const int64_t e1 = min(m, e0 + (int64_t)MOD_EDGES_PER_BLOCK);
    __syncthreads();
    if (threadIdx.x == 0) s_r[0] = row_of(e0, 0, n);
    if (threadIdx.x == 64) s_r[1] = row_of(e1 - 1, 0, n);
    __syncthreads();
    const int64_t r0 = s_r[0], r1 = s_r[1];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
      const int64_t r = row_of(e, r0, r1 + 1);
      const uint32_t x = load_w<WK>(w, e);
      two_m += x;
      if (C[idx[e]] == C[r]) s1 += x;
    }
  }
#pragma unroll
  for (int mm = 32; mm > 0; mm >>= 1) {
    two_m += shfl_xor_u64(two_m, mm);
    s1 += shfl_xor_u64(s1, mm);
  }
  if ((threadIdx.x & 63) == 0) {
    s_two_m[threadIdx.x >> 6] = two_m;
    s_s1[threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&acc->two_m, s_two_m[0] + s_two_m[1] + s_two_m[2] + s_two_m[3]);
    atomicAdd(&acc->s1, s_s1[0] + s_s1[1] + s_s1[2] + s_s1[3]);
  }
}

constexpr int MOD_SQ_BLOCKS = 1024;

// Sum of squares in 128-bit integers; each block writes (lo, hi) of its partial.
__global__ __launch_bounds__(256) void k_mod_squares(const u64 *tot, int64_t n, u64 *partials) {
  __shared__ unsigned __int128 s[256];
  unsigned __int128 acc = 0;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
    const unsigned __int128 t = tot[c];
    acc += t * t;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = (u64)s[0];
    partials[2 * blockIdx.x + 1] = (u64)(s[0] >> 64);
  }
}

void launch_check_labels(const int32_t *C, int64_t n, int32_t *bad, hipStream_t st) {
  hipLaunchKernelGGL(k_check_labels, dim3(grid_for(n, 256)), dim3(256), 0, st, C, n, bad);
}
void launch_mod_community_totals(const int32_t *C, const uint32_t *K, int64_t n, u64 *tot, hipStream_t st) {
  hipLaunchKernelGGL(k_mod_community_totals, dim3(grid_for(n, 256 * 16, 4096)), dim3(256), 0, st, C, K, n, tot);
}
void launch_mod_inside(const int64_t *off, const int32_t *idx, const void *w, int wk, const int32_t *C, int64_t n,
                       int64_t m, ModAcc *acc, hipStream_t st) {
  dim3 g(grid_for(m, MOD_EDGES_PER_BLOCK)), b(256);
  if (wk == W_UNIT) hipLaunchKernelGGL(k_mod_inside<W_UNIT>, g, b, 0, st, off, idx, w, C, n, m, acc);
  else if (wk == W_U8) hipLaunchKernelGGL(k_mod_inside<W_U8>, g, b, 0, st, off, idx, w, C, n, m, acc);
  else hipLaunchKernelGGL(k_mod_inside<W_U32>, g, b, 0, st, off, idx, w, C, n, m, acc);
}
int mod_square_blocks() { return MOD_SQ_BLOCKS; }
void launch_mod_squares(const u64 *tot, int64_t n, u64 *partials, hipStream_t st) {
  hipLaunchKernelGGL(k_mod_squares, dim3(MOD_SQ_BLOCKS), dim3(256), 0, st, tot, n, partials);
}

}  // namespace gvelpa
