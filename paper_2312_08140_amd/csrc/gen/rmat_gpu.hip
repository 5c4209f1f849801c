// R-MAT graphs generated and assembled into CSR on the GPU (gfx950).
//
// An input generator only: none of the label-propagation arithmetic lives
// here.  The draws are the counter-based ones of the host generator
// (graphgen.cpp), so the CSR is bit-identical to the host one:
//   1. count  - every generated edge (u, v), u != v, adds one entry to row u
//               and one to row v (64-bit atomics);
//   2. scan   - row starts of the raw (undeduplicated) entries;
//   3. place  - the edges are drawn again and each direction is written into
//               its row behind an atomic cursor;
//   4. sort   - rows are cut into chunks of at most CHUNK entries; a chunk's
//               entries are sorted by the key (row - first row) << sbits | col
//               and duplicate keys dropped (one radix sort + select-unique per
//               chunk), which leaves every row sorted and duplicate-free, its
//               entry count added per row;
//   5. emit   - final offsets by a scan of those counts, then each chunk's
//               entries copied to the caller's index array in one piece, and
//               the weights computed from the unordered pair.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "gvelpa_gen.h"

namespace {

typedef unsigned long long u64;

constexpr u64 kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ u64 draw(u64 key, u64 ctr) { return mix64(key + (ctr + 1) * kGamma); }
u64 stream_key(u64 seed, u64 stream) { return mix64(seed * kGamma + stream * 0xD1B54A32D192ED03ull); }

struct RmatParams {
  u64 key;
  u64 ta, tb, tc;  // cumulative quadrant thresholds on 32-bit uniforms
  int scale;
  int dpe;         // draws per edge
};

// Edge e of the R-MAT stream; false for a self-loop (dropped).
__device__ __forceinline__ bool rmat_edge(const RmatParams &p, u64 e, uint32_t &u, uint32_t &v) {
  uint32_t su = 0, sv = 0;
  u64 x = 0;
  for (int l = 0; l < p.scale; ++l) {
    if ((l & 1) == 0) x = draw(p.key, e * (u64)p.dpe + (u64)(l >> 1));
    const u64 r = (l & 1) ? (x & 0xFFFFFFFFull) : (x >> 32);
    const uint32_t bit = 1u << (p.scale - 1 - l);
    if (r < p.ta) {
    } else if (r < p.tb) {
      sv |= bit;
    } else if (r < p.tc) {
      su |= bit;
    } else {
      su |= bit;
      sv |= bit;
    }
  }
  u = su;
  v = sv;
  return su != sv;
}

__global__ __launch_bounds__(256) void k_count(RmatParams p, u64 n_edges, u64 *deg) {
  for (u64 e = (u64)blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (u64)gridDim.x * 256) {
    uint32_t u, v;
    if (!rmat_edge(p, e, u, v)) continue;
    atomicAdd(&deg[u], 1ull);
    atomicAdd(&deg[v], 1ull);
  }
}

__global__ __launch_bounds__(256) void k_place(RmatParams p, u64 n_edges, const u64 *start, u64 *cursor,
                                               int32_t *raw) {
  for (u64 e = (u64)blockIdx.x * 256 + threadIdx.x; e < n_edges; e += (u64)gridDim.x * 256) {
    uint32_t u, v;
    if (!rmat_edge(p, e, u, v)) continue;
    raw[start[u] + atomicAdd(&cursor[u], 1ull)] = (int32_t)v;
    raw[start[v] + atomicAdd(&cursor[v], 1ull)] = (int32_t)u;
  }
}

// Sort keys of the raw entries of rows [r0, r1); one wave per row.
__global__ __launch_bounds__(256) void k_keys(const u64 *start, const int32_t *raw, int64_t r0, int64_t r1, int sbits,
                                              u64 *key) {
  const int lane = threadIdx.x & 63;
  const u64 base = start[r0];
  for (int64_t r = r0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < r1; r += (int64_t)gridDim.x * 4)
    for (u64 k = start[r] + lane; k < start[r + 1]; k += 64)
      key[k - base] = ((u64)(r - r0) << sbits) | (u64)(uint32_t)raw[k];
}

// Unique sorted keys of a chunk -> columns at out[i], and per-row counts
// (the lanes of a wave holding one row add their count with one atomic).
__global__ __launch_bounds__(256) void k_unpack(const u64 *key, const int32_t *nsel, int64_t r0, int sbits,
                                                int32_t *out, u64 *rowcount) {
  const int64_t len = *nsel;
  const int lane = threadIdx.x & 63;
  const u64 cmask = (1ull << sbits) - 1;
  for (int64_t base = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); base < len; base += (int64_t)gridDim.x * 256) {
    const int64_t i = base + lane;
    const bool ok = i < len;
    const u64 k = ok ? key[i] : ~0ull;
    const u64 row = k >> sbits;
    if (ok) out[i] = (int32_t)(uint32_t)(k & cmask);
    const u64 prev = __shfl_up(k, 1, 64) >> sbits;
    const bool head = ok && (lane == 0 || prev != row);
    const u64 heads = __ballot(head);
    if (head) {
      const u64 after = heads & ~((2ull << lane) - 1);  // heads of later lanes
      const int end = after ? __builtin_ctzll(after) : 64;
      const int64_t cnt = std::min<int64_t>(end, len - base) - lane;
      atomicAdd(&rowcount[r0 + (int64_t)row], (u64)cnt);
    }
  }
}

__device__ __forceinline__ float pair_weight(u64 wkey, uint32_t u, uint32_t v) {
  const uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
  return (float)(1 + (mix64(wkey ^ (((u64)lo << 32) | hi)) & 7));
}

__global__ __launch_bounds__(256) void k_weights(const int64_t *off, const int32_t *idx, int64_t n, u64 wkey,
                                                 int weighted, float *w) {
  const int lane = threadIdx.x & 63;
  for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < n; r += (int64_t)gridDim.x * 4)
    for (int64_t k = off[r] + lane; k < off[r + 1]; k += 64)
      w[k] = weighted ? pair_weight(wkey, (uint32_t)r, (uint32_t)idx[k]) : 1.0f;
}

__global__ void k_to_i64(const u64 *src, int64_t *dst, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (int64_t)src[i];
}

int grid(int64_t items, int per, int cap = 65536) {
  const int64_t b = (items + per - 1) / per;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

struct Fail {
  int code;
};

#define GV_OK(expr)                                   \
  do {                                                \
    if ((expr) != hipSuccess) {                       \
      (void)hipGetLastError();                        \
      throw Fail{GVGEN_ERR_DEVICE};                   \
    }                                                 \
  } while (0)

struct Scratch {
  std::vector<void *> ptrs;
  void *get(size_t bytes) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{GVGEN_ERR_OUT_OF_MEMORY};
    }
    ptrs.push_back(p);
    return p;
  }
  void put(void *p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
      ptrs.erase(it);
      (void)hipFree(p);
    }
  }
  ~Scratch() {
    for (void *p : ptrs) (void)hipFree(p);
  }
};

// Entries per sort chunk: the chunk's keys (twice) stay within 4 GiB.
constexpr int64_t CHUNK = (int64_t)1 << 28;

}  // namespace

extern "C" {

const char *gvgen_status_string(int status) {
  switch (status) {
    case GVGEN_OK: return "ok";
    case GVGEN_ERR_INVALID_ARG: return "invalid argument";
    case GVGEN_ERR_OUT_OF_MEMORY: return "out of device memory";
    case GVGEN_ERR_DEVICE: return "a HIP call failed";
    default: return "unknown status";
  }
}

int gvgen_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed, int weighted, int device,
               void *hip_stream, gvgen_alloc_fn alloc, int64_t *n_out, int64_t *m_out) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0 || !alloc || !n_out ||
      !m_out || weighted < -1 || weighted > 1 || edge_factor > ((int64_t)1 << 40))
    return GVGEN_ERR_INVALID_ARG;
  const hipStream_t st = (hipStream_t)hip_stream;
  try {
    GV_OK(hipSetDevice(device));
    Scratch S;
    const int64_t n = (int64_t)1 << scale;
    const u64 n_edges = (u64)edge_factor << scale;
    RmatParams p;
    p.ta = (u64)std::llround(a * 4294967296.0);
    p.tb = (u64)std::llround((a + b) * 4294967296.0);
    p.tc = (u64)std::llround((a + b + c) * 4294967296.0);
    p.key = stream_key(seed, 0x524D4154ull);
    p.scale = scale;
    p.dpe = (scale + 1) / 2;
    const u64 wkey = stream_key(seed, 0x57454947ull);
    hipDeviceProp_t prop;
    GV_OK(hipGetDeviceProperties(&prop, device));
    const int gen_blocks = grid((int64_t)std::min<u64>(n_edges, (u64)1 << 40), 256, prop.multiProcessorCount * 32);

    // 1-2. raw row lengths and row starts
    u64 *deg = (u64 *)S.get(sizeof(u64) * (n + 1));
    u64 *start = (u64 *)S.get(sizeof(u64) * (n + 1));
    GV_OK(hipMemsetAsync(deg, 0, sizeof(u64) * (n + 1), st));
    hipLaunchKernelGGL(k_count, dim3(gen_blocks), dim3(256), 0, st, p, n_edges, deg);
    GV_OK(hipGetLastError());
    size_t tb = 0;
    GV_OK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, deg, start, (int)(n + 1), st));
    void *scan_tmp = S.get(tb);
    GV_OK(hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb, deg, start, (int)(n + 1), st));
    std::vector<u64> h_start((size_t)n + 1);
    GV_OK(hipMemcpyAsync(h_start.data(), start, sizeof(u64) * (n + 1), hipMemcpyDeviceToHost, st));
    GV_OK(hipStreamSynchronize(st));
    const u64 raw_total = h_start[n];

    // 3. both directions of every edge into their rows
    int32_t *raw = (int32_t *)S.get(sizeof(int32_t) * std::max<u64>(raw_total, 1));
    GV_OK(hipMemsetAsync(deg, 0, sizeof(u64) * (n + 1), st));  // now the placement cursors
    hipLaunchKernelGGL(k_place, dim3(gen_blocks), dim3(256), 0, st, p, n_edges, start, deg, raw);
    GV_OK(hipGetLastError());

    // 4. per chunk of rows: sort by (row, col), drop duplicates, count per row
    u64 *rowcount = deg;  // cursors are no longer needed
    GV_OK(hipMemsetAsync(rowcount, 0, sizeof(u64) * (n + 1), st));
    const int64_t ch = (int64_t)std::min<u64>(std::max<u64>(raw_total, 1), (u64)CHUNK);
    u64 *kin = (u64 *)S.get(sizeof(u64) * ch);
    u64 *kout = (u64 *)S.get(sizeof(u64) * ch);
    int32_t *nsel = (int32_t *)S.get(sizeof(int32_t));
    size_t sort_b = 0, uniq_b = 0;
    GV_OK(hipcub::DeviceRadixSort::SortKeys(nullptr, sort_b, kin, kout, (int)ch, 0, 64, st));
    GV_OK(hipcub::DeviceSelect::Unique(nullptr, uniq_b, kout, kin, nsel, (int)ch, st));
    const size_t tmp_b = std::max(sort_b, uniq_b);
    void *tmp = S.get(tmp_b);
    const int sbits = scale;  // column bits
    struct Piece {
      int64_t r0, r1;
      u64 e0;
      int32_t kept;
    };
    std::vector<Piece> pieces;
    for (int64_t r0 = 0; r0 < n;) {
      // rows [r0, r1) with at most ch raw entries (a single row always fits:
      // a row holds at most 2 * n_edges / ... entries, checked below)
      int64_t r1 = std::upper_bound(h_start.begin() + r0 + 1, h_start.end(), h_start[r0] + (u64)ch) -
                   h_start.begin() - 1;
      if (r1 <= r0) r1 = r0 + 1;
      const u64 len = h_start[r1] - h_start[r0];
      if (len > (u64)ch) throw Fail{GVGEN_ERR_OUT_OF_MEMORY};  // one row beyond a chunk: not supported
      int rbits = 1;
      while (rbits < 40 && ((int64_t)1 << rbits) < r1 - r0) ++rbits;
      if (sbits + rbits > 64) throw Fail{GVGEN_ERR_INVALID_ARG};
      Piece pc{r0, r1, h_start[r0], 0};
      if (len > 0) {
        hipLaunchKernelGGL(k_keys, dim3(grid(r1 - r0, 4)), dim3(256), 0, st, start, raw, r0, r1, sbits, kin);
        GV_OK(hipGetLastError());
        size_t b1 = tmp_b;
        GV_OK(hipcub::DeviceRadixSort::SortKeys(tmp, b1, kin, kout, (int)len, 0, sbits + rbits, st));
        size_t b2 = tmp_b;
        GV_OK(hipcub::DeviceSelect::Unique(tmp, b2, kout, kin, nsel, (int)len, st));
        hipLaunchKernelGGL(k_unpack, dim3(grid((int64_t)len, 256, prop.multiProcessorCount * 16)), dim3(256), 0, st,
                           kin, nsel, r0, sbits, raw + h_start[r0], rowcount);
        GV_OK(hipGetLastError());
        GV_OK(hipMemcpyAsync(&pc.kept, nsel, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GV_OK(hipStreamSynchronize(st));
      }
      pieces.push_back(pc);
      r0 = r1;
    }
    S.put(kin);
    S.put(kout);
    S.put(tmp);

    // 5. final offsets, indices and weights in the caller's arrays
    int64_t m = 0;
    for (const Piece &pc : pieces) m += pc.kept;
    int64_t *off = (int64_t *)alloc(0, n + 1);
    if (!off) throw Fail{GVGEN_ERR_OUT_OF_MEMORY};
    int32_t *idx = (int32_t *)alloc(1, m);
    if (!idx) throw Fail{GVGEN_ERR_OUT_OF_MEMORY};
    float *w = nullptr;
    if (weighted >= 0) {
      w = (float *)alloc(2, m);
      if (!w) throw Fail{GVGEN_ERR_OUT_OF_MEMORY};
    }
    GV_OK(hipcub::DeviceScan::ExclusiveSum(scan_tmp, tb, rowcount, start, (int)(n + 1), st));
    hipLaunchKernelGGL(k_to_i64, dim3(grid(n + 1, 256, 16384)), dim3(256), 0, st, start, off, n + 1);
    GV_OK(hipGetLastError());
    int64_t at = 0;
    for (const Piece &pc : pieces) {
      if (pc.kept)
        GV_OK(hipMemcpyAsync(idx + at, raw + pc.e0, sizeof(int32_t) * (size_t)pc.kept, hipMemcpyDeviceToDevice, st));
      at += pc.kept;
    }
    if (w && m) {
      hipLaunchKernelGGL(k_weights, dim3(grid(n, 4)), dim3(256), 0, st, off, idx, n, wkey, weighted, w);
      GV_OK(hipGetLastError());
    }
    GV_OK(hipStreamSynchronize(st));
    *n_out = n;
    *m_out = m;
    return GVGEN_OK;
  } catch (Fail f) {
    (void)hipStreamSynchronize(st);
    return f.code;
  }
}

}  // extern "C"
