// Shared device-side definitions of the gfx950 label-propagation library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gvelpa {

typedef unsigned long long u64;

// ---------------------------------------------------------------- sweep bins
// Vertices with at least one stored entry are split by degree.  Bins 0-3 are
// processed by GROUP lanes of one wave per vertex (one lane per vertex in bin
// 0), bins 4-5 by a workgroup per vertex; each vertex owns an LDS open-addressing table of SLOTS 64-bit
// entries.  A table never holds more distinct labels than the vertex has
// entries, so a bin's degree limit must stay below its SLOTS (the defaults
// keep the load factor <= 1/2).  The last bin ("hub") splits a vertex over
// many workgroups (see the hub kernels).
constexpr int NBINS = 7;
constexpr int HUB_BIN = NBINS - 1;
constexpr int BIN_SLOTS[NBINS - 1] = {8, 32, 128, 512, 2048, 8192};
constexpr int DEFAULT_BIN_MAXDEG[NBINS - 1] = {4, 16, 64, 256, 1024, 4096};

// Kernel shapes of a bin: lanes per vertex (bins 0-3: lanes of one wave,
// bins 4-5: a workgroup), table slots (fixed per bin: BIN_SLOTS), row entries
// in flight per lane, and (reg) a table in registers instead of LDS: one
// thread per vertex holds its whole row and sums equal labels by comparing
// the entries pairwise (the bin's rows have fewer entries than its slots;
// the default of bin 0).  Variant 0 is the default; the others are the
// tuner's candidates.
constexpr int NVARIANTS = 3;
struct BinShape {
  int group, slots, unroll, reg;
};
constexpr BinShape BIN_SHAPES[NBINS - 1][NVARIANTS] = {
    {{1, 8, 8, 1}, {1, 8, 4}, {2, 8, 2}},
    {{2, 32, 8}, {4, 32, 4}, {2, 32, 4}},
    {{8, 128, 8}, {16, 128, 4}, {8, 128, 4}},
    {{32, 512, 8}, {64, 512, 4}, {32, 512, 4}},
    {{128, 2048, 8}, {256, 2048, 4}, {128, 2048, 4}},
    {{256, 8192, 16}, {256, 8192, 8}, {512, 8192, 8}},
};

// Hub path: a hub's entries are cut into chunks of HUB_CHUNK; a chunk's labels
// are merged in LDS and scattered into 2^pbits label partitions (by hash),
// each of capacity HUB_PART_CAP entries in HBM; one workgroup then merges each
// partition in an LDS table of HUB_PART_SLOTS.  Partitions are sized for at
// most HUB_PART_TARGET distinct labels; a partition that fills up spills into
// a shared overflow area, so results never depend on the label distribution.
// Hubs with more than 2^HUB_LDS_PBITS partitions reserve their slots with one
// global atomic per merged label instead of an LDS histogram per chunk.
constexpr int HUB_CHUNK = 2048;
constexpr int HUB_CHUNK_SLOTS = 4096;
constexpr int HUB_PART_TARGET = 1024;
constexpr int HUB_PART_CAP = 1536;
constexpr int HUB_PART_SLOTS = 2048;
constexpr int HUB_PART_GROUP_BITS = 4;   // most partitions merged together when they hold few pairs: 16
constexpr int HUB_PART_GROUP = 1 << HUB_PART_GROUP_BITS;
constexpr int HUB_PART_GROUP_MAX = 1024;  // most pairs of a merged group

// Merge work items of a hub with 2^pbits partitions, in groups of 2^gbits.
__host__ __device__ constexpr int hub_merge_groups(int pbits, int gbits) {
  return pbits > gbits ? 1 << (pbits - gbits) : 1;
}
constexpr int HUB_MAX_PBITS = 21;  // partitions for hubs of up to 2^31 entries
constexpr int HUB_LDS_PBITS = 12;  // up to here the chunk kernel counts its partitions in LDS
constexpr int64_t HUB_OVERFLOW_CAP = 1 << 22;  // shared spill area for over-full partitions
// Most partition maxima (chunks x partitions over a step's hubs) for which a
// step decides and marks its hubs in one kernel, every chunk re-reading its
// hub's maxima (8 MB of reads at most).
constexpr int64_t HUB_FUSED_READS = 1 << 20;

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

// Tie rule among the heaviest labels of a vertex.  Strict LPA (Section 2,
// Section 4.1.5) takes the smallest label id.  Non-strict LPA (Section 4.1.5:
// a pick by a modulo operation on the label id) takes the label of smallest
// rank r(c) = ((c + 1) * M) mod P, P = 2^31 - 1 prime, M = A^(1 + (id mod 64))
// mod P for the vertex's id, A = 1580030173: distinct labels get distinct
// ranks, and the pick changes with the vertex like a random one.  Ranks are
// turned back into labels with the inverse multiplier (A^-1 = 1989098352).
constexpr uint32_t TIE_P = 2147483647u;
constexpr uint32_t TIE_A = 1580030173u;
constexpr uint32_t TIE_A_INV = 1989098352u;

struct TieTables {
  uint32_t mult[64], inv[64];
};
constexpr TieTables make_tie_tables() {
  TieTables t{};
  u64 m = 1, i = 1;
  for (int k = 0; k < 64; ++k) {
    m = m * TIE_A % TIE_P;
    i = i * TIE_A_INV % TIE_P;
    t.mult[k] = (uint32_t)m;
    t.inv[k] = (uint32_t)i;
  }
  return t;
}
static_assert((u64)TIE_A * TIE_A_INV % TIE_P == 1, "inverse multiplier");

// a * b mod 2^31 - 1 for a, b < 2^31 (Mersenne reduction)
__device__ __forceinline__ uint32_t mulmod_p(uint32_t a, uint32_t b) {
  u64 x = (u64)a * b;
  x = (x & TIE_P) + (x >> 31);
  x = (x & TIE_P) + (x >> 31);
  return (uint32_t)(x >= TIE_P ? x - TIE_P : x);
}

// mult = 0: strict rule
struct TieRule {
  uint32_t mult, inv;
};

__device__ __forceinline__ uint32_t tie_rank(uint32_t lbl, TieRule t) {
  if (!t.mult) return lbl;
  const uint32_t c1 = lbl + 1u;  // in [1, 2^31 - 1]
  return mulmod_p(c1 >= TIE_P ? c1 - TIE_P : c1, t.mult);
}
__device__ __forceinline__ uint32_t rank_label(uint32_t r, TieRule t) {
  if (!t.mult) return r;
  const uint32_t c1 = mulmod_p(r, t.inv);
  return (c1 == 0 ? TIE_P : c1) - 1u;
}

// Argmax key: weight in the high word, ~rank in the low word, so the
// largest key is the heaviest label and, among equals, the smallest id
// (strict) or rank (non-strict).  0 means "no candidate" (~rank >= 2^31 for
// every valid rank).
__device__ __forceinline__ u64 entry_key(u64 slot, TieRule t) {
  return (slot << 32) | (u64)(~tie_rank((uint32_t)(slot >> 32), t));
}
__device__ __forceinline__ uint32_t key_label(u64 key, TieRule t) { return rank_label(~(uint32_t)key, t); }

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
// Sweep counters are added per workgroup into one of NSHARD copies (a
// 64-byte line per copy and slot) rather than into one address: thousands of
// workgroups adding to a single counter serialise on it.  Slots 0..NBINS-1
// belong to the scan kernels of a bin (changed, scanned entries, vertices,
// marks), slot NBINS to the compaction (processed, gated, listed, unused),
// FIRST_SLOT to the kernels of a snapshot first sweep (changed, scanned
// entries, vertices, marks) and READS_SLOT to the neighbour ids they read.
// k_end_sweep folds and clears them.
constexpr int NSHARD = 64;
constexpr int FIRST_SLOT = NBINS + 1;
constexpr int READS_SLOT = NBINS + 2;
constexpr int NSLOT = NBINS + 3;
struct alignas(64) Shard {
  u64 c[4];
  u64 pad[4];
};

struct Ctl {
  int32_t done;        // stop test held or the sweep cap was reached
  int32_t sweep;       // index of the sweep in progress
  int32_t iterations;  // sweeps completed
  int32_t converged;
  int32_t error;       // nonzero: a table overflowed (never expected)
  int32_t max_iters;
  int32_t verify_phase;  // while a verification sweep runs: 1 over the flagged vertices, 2 over all
  int32_t gate_on;       // 1: flagged vertices pass the gate before processing
  int32_t verified;      // last verification sweep changed <= tau * n labels
  // Dense sweeps (asynchronous mode): when most vertices change, every
  // neighbour would be flagged anyway; the sweep then writes no marks and all
  // flags are set once at its end (pruning is exact, so processing a vertex
  // that would not have been flagged changes nothing).
  int32_t dense_enabled, dense_cur, dense_prev, pad0;
  // batched runs: graphs still running, graphs stopped without meeting the
  // stop test, the verification mode (0 none, 1 over the flagged vertices, 2
  // over all), the sweep cap of each graph's method, graphs whose last
  // verification sweep failed
  int32_t batch, batch_remaining, batch_capped, batch_mode;
  int32_t batch_iters, batch_unverified, pad1, pad2;
  double dense_frac;
  int64_t n_active;
  double tau;
  int64_t n;
  u64 changed, processed, scanned, gated;  // current sweep
  u64 hub_chunks, hub_groups;              // hub work items of the current step
  u64 st_changed[MAX_REC], st_processed[MAX_REC], st_scanned[MAX_REC], st_gated[MAX_REC];
  u64 t_start, t_sweep[MAX_REC];
  u64 verify_changed, total_changed, verify_scanned;
  // run totals per bin (byte accounting of the kernels)
  u64 bin_vertices[NBINS], bin_edges[NBINS], bin_changed[NBINS], bin_marks[NBINS];
  u64 compact_listed, compact_taken;
  // run totals of the snapshot first sweep's kernels
  u64 first_vertices, first_edges, first_changed, first_marks, first_reads;
  Shard shard[NSHARD][NSLOT];
};

// ---------------------------------------------------------------- gate
// Learned active-set gate: an 8-32-32-1 network predicts whether a flagged
// vertex will change label.  Its inputs, for vertex v at sweep s:
//   x0 = log2(1 + deg v)            x4 = s / max_iters
//   x1 = (W1 - W2) / K_v            x5 = W1 / K_v
//   x2 = W(own label) / K_v         x6 = distinct labels / deg v
//   x3 = 1 if v changed when last processed
//   x7 = min(s - sweep of last processing, 8) / 8
// with W1 >= W2 the two largest label weights of v's last scan and K_v its
// weighted degree.  x0-x3, x5, x6 are stored per vertex when it is processed,
// in a 32-byte record with the sweep of that processing (written with two
// 16-byte stores): {x0, x1, x2, x3}, {x5, x6, last sweep (int bits, -1 =
// never), 0}.
constexpr int NFEAT = 8;
constexpr int FEAT_STRIDE = 8;  // floats per vertex record
constexpr int FEAT_LASTP = 6;   // slot of the last sweep
constexpr int GATE_PARAMS = 32 * 8 + 32 + 32 * 32 + 32 + 32 + 1;  // 1377

struct FeatArgs {
  float *feat;         // [n][FEAT_STRIDE] records of the last processing
  const uint32_t *K;   // weighted degrees
  float *tx;           // trace features [tcap][NFEAT]
  uint8_t *ty;         // trace targets (1 = the vertex changed)
  u64 *tcount;
  u64 tcap;
  uint32_t tthresh;    // a sample is kept when its hash is below this
  int trace;
  int max_iters;
};

__device__ __forceinline__ int record_lastp(const float *rec) { return __float_as_int(rec[FEAT_LASTP]); }

__device__ __forceinline__ void decision_features(const float *st, int lastp, int s, int max_iters, float *x) {
  x[0] = st[0];
  x[1] = st[1];
  x[2] = st[2];
  x[3] = st[3];
  x[4] = (float)s / (float)(max_iters > 0 ? max_iters : 1);
  x[5] = st[4];
  x[6] = st[5];
  const int age = s - lastp;
  x[7] = (float)(age < 8 ? age : 8) * 0.125f;
}

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
  int bin;
  uint8_t *chg;  // batched runs: set to 1 for every vertex that changes (per-graph dN)
  FeatArgs f;    // gate features and traces (kernels built with FEAT)
  int nonstrict;        // 1: non-strict tie rule (tie_rank)
  const int32_t *orig;  // vertex id at each storage position (NULL: positions are ids)
};

// Tie rule of the vertex at storage position v.
static __device__ __constant__ TieTables c_tie = make_tie_tables();
__device__ __forceinline__ TieRule tie_rule_of(const ScanArgs &a, int v) {
  if (!a.nonstrict || v < 0) return TieRule{0u, 0u};
  const uint32_t k = (uint32_t)(a.orig ? a.orig[v] : v) & 63u;
  return TieRule{c_tie.mult[k], c_tie.inv[k]};
}

// Hub metadata (per hub, sorted by id) and per-step scratch.
struct HubArgs {
  int32_t n_hubs;
  int32_t part_cap;          // entries kept per partition before spilling (<= HUB_PART_CAP)
  const int32_t *ids;        // sorted hub ids
  const int32_t *chunks;     // chunks of each hub
  const int32_t *pbits;      // log2 partitions of each hub
  const int64_t *pair_base;  // first pair slot of each hub (partition p at pair_base + p * HUB_PART_CAP)
  const int64_t *cnt_base;   // first partition counter of each hub
  u64 *pairs;                // (label << 32 | weight) entries
  int32_t *pcnt;             // entries written per (hub, partition); zero between steps
  u64 *partbest;             // best key per (frontier hub, partition) of the step
  uint32_t *ovf;             // spill entries: (global part, label, weight, unused)
  u64 *ovf_count;
  int32_t *ord;              // per frontier entry: hub ordinal
  u64 *cstart;               // per frontier entry: first chunk id of the step
  u64 *pstart;               // per frontier entry: first partition id of the step
  u64 *gstart;               // per frontier entry: first merge group id of the step
  int32_t *chunk_owner;      // per chunk id of the step: frontier entry
  int32_t *group_owner;      // per merge group id of the step: frontier entry
  uint32_t *part_w2;         // FEAT: second largest label weight of each partition
  int32_t *part_nd;          // FEAT: distinct labels of each partition
  uint32_t *own_w;           // FEAT: per frontier entry, weight of the hub's own label
  int32_t first;             // snapshot first sweep: k_hub_owner zeroes the partition maxima
  u64 *blk;                  // per tile of frontier hubs: work items (chunks, partitions, groups), then offsets
  int32_t gbits;             // log2 partitions per merge group (0: every partition its own work item)
  int32_t ids_identity;      // ids[k] == k for every hub (degree order): a hub's ordinal is its position
  // Chunks of all hubs in increasing storage position of their first
  // neighbour, (hub ordinal << 32 | chunk of the hub); with static_order the
  // chunk kernel walks them instead of the step's chunk ids, so that the
  // chunks running at the same time gather labels from nearby positions.
  const u64 *sorder;
  int64_t sorder_len;
  int32_t static_order;
  int32_t *slot_of;          // per hub ordinal: its frontier entry in the current step, -1 when not flagged
  int32_t *cur;              // per frontier entry: the hub's label when the step was planned
  int32_t *changed;          // per frontier entry: 1 if the hub took a new label (k_hub_decide)
  // Static plan (deterministic colour steps): the work items of every hub of
  // the step's colour are planned once; the "frontier" is the colour's hub
  // list, taken[i] says whether the compaction took hub i in this step, and
  // the kernels skip the others.  The counts replace the plan's totals.
  const uint8_t *taken;
  int32_t static_plan;
  int64_t static_count, static_chunks, static_groups;
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
