// Shared device-side definitions of the gfx950 label-propagation library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gvelpa {

typedef unsigned long long u64;

// ---------------------------------------------------------------- sweep bins
// Vertices with at least one stored entry are split by degree.  A bin is
// processed by groups of GROUP lanes sharing an LDS open-addressing table of
// SLOTS 64-bit entries; the last bin ("hub") keeps its tables in HBM.  A
// table never holds more distinct labels than the vertex has entries, so a
// bin's degree limit must stay below its SLOTS (load factor <= 1/2 by default).
constexpr int NBINS = 7;
constexpr int HUB_BIN = NBINS - 1;
constexpr int BIN_GROUP[NBINS - 1] = {8, 16, 64, 256, 256, 512};
constexpr int BIN_SLOTS[NBINS - 1] = {16, 64, 256, 1024, 4096, 8192};
constexpr int DEFAULT_BIN_MAXDEG[NBINS - 1] = {8, 32, 128, 512, 2048, 4096};
constexpr int HUB_CHUNK = 4096;  // edges per hub work item

// Runtime degree limits of bins 0..NBINS-2 (the hub bin takes the rest).
struct BinLimits {
  int32_t maxdeg[NBINS - 1];
};
__host__ __device__ __forceinline__ int bin_of_degree(int64_t deg, const BinLimits &lim) {
#pragma unroll
  for (int b = 0; b < NBINS - 1; ++b)
    if (deg <= lim.maxdeg[b]) return b;
  return NBINS - 1;
}

// Table entry: label in the high word, summed weight in the low word.  The
// weighted degree is validated to stay below 2^32, so adds never carry into
// the label.  An empty slot holds label 0xFFFFFFFF (labels are < 2^31).
constexpr u64 EMPTY = 0xFFFFFFFF00000000ull;

// Argmax key: weight in the high word, ~label in the low word, so the
// largest key is the heaviest label and, among equals, the smallest id.
// 0 means "no candidate" (~label >= 2^31 for every valid label).
__device__ __forceinline__ u64 entry_key(u64 slot) {
  return (slot << 32) | (u64)(~(uint32_t)(slot >> 32));
}
__device__ __forceinline__ uint32_t key_label(u64 key) { return ~(uint32_t)key; }

// Fibonacci hashing of a label into 2^bits slots.
__device__ __forceinline__ uint32_t slot_hash(uint32_t label, int bits) {
  return (label * 0x9E3779B1u) >> (32 - bits);
}

// MurmurHash3 32-bit finaliser (Appleby, public domain): colouring priorities.
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Weight storage inside the library: unit (no array), uint8 or uint32.
enum WeightKind : int { W_UNIT = 0, W_U8 = 1, W_U32 = 2 };

template <int WK>
__device__ __forceinline__ uint32_t load_w(const void *w, int64_t e) {
  if constexpr (WK == W_UNIT) return 1u;
  else if constexpr (WK == W_U8) return (uint32_t)((const uint8_t *)w)[e];
  else return ((const uint32_t *)w)[e];
}

// ---------------------------------------------------------------- run control
constexpr int MAX_REC = 64;

// Device-resident control block of a handle.  Accumulators are reset by the
// run prologue and at the end of every sweep.
struct Ctl {
  int32_t done;        // stop test held or the sweep cap was reached
  int32_t sweep;       // index of the sweep in progress
  int32_t iterations;  // sweeps completed
  int32_t converged;
  int32_t error;       // nonzero: a table overflowed (never expected)
  int32_t max_iters;
  int32_t verify_phase;  // 1 while a verification sweep runs
  int32_t gate_on;
  double tau;
  int64_t n;
  u64 changed, processed, scanned, gated;  // current sweep
  u64 hub_chunks;                          // hub work items of the current step
  u64 st_changed[MAX_REC], st_processed[MAX_REC], st_scanned[MAX_REC], st_gated[MAX_REC];
  u64 t_start, t_sweep[MAX_REC];
  u64 verify_changed, total_changed;
};

// Per-step arguments of the scan kernels.
struct ScanArgs {
  const int64_t *off;
  const int32_t *idx;
  const void *w;
  int32_t *C;
  uint8_t *F;
  const int32_t *front;   // frontier of this (step, bin)
  const int32_t *fcount;  // its length (device)
  Ctl *ctl;
  int prune;
  // hub path
  u64 *htab;
  const int64_t *hub_toff;   // per frontier entry: table offset (entries)
  const int32_t *hub_tbits;  // per frontier entry: log2 table size
  const u64 *hub_cstart;     // per frontier entry: first chunk id (exclusive scan)
  const int32_t *hub_ids;    // sorted ids of every hub vertex
  const int64_t *hub_toff_all;
  const int32_t *hub_tbits_all;
  int32_t n_hubs;
};

// Wave64 helpers.
__device__ __forceinline__ u64 shfl_xor_u64(u64 x, int m) {
  uint32_t lo = __shfl_xor((uint32_t)x, m, 64);
  uint32_t hi = __shfl_xor((uint32_t)(x >> 32), m, 64);
  return ((u64)hi << 32) | lo;
}

template <int WIDTH>
__device__ __forceinline__ u64 group_max(u64 x) {
#pragma unroll
  for (int m = WIDTH / 2; m > 0; m >>= 1) {
    u64 y = shfl_xor_u64(x, m);
    x = y > x ? y : x;
  }
  return x;
}

__device__ __forceinline__ void wave_lds_sync() {
  // orders LDS traffic of the lanes of one wave (a group lives in one wave)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace gvelpa
