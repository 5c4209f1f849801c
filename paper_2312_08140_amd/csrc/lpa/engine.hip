// Host engine behind the C ABI of include/gvelpa.h: device memory, work
// lists, the sweep schedule of both modes, HIP-graph capture and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <thread>
#include <string>
#include <tuple>
#include <vector>

#include "gvelpa.h"
#include "sweep_kernels.hpp"

using namespace gvelpa;

namespace gvelpa {
// The failing HIP call behind the last LPA_ERR_DEVICE of this thread.
void note_hip_error(int err, const char *what, const char *file, int line);
}  // namespace gvelpa

namespace {

struct Status {
  int code;
};

thread_local std::string last_error;

#define HIP_OK(expr)                                      \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) {                               \
      note_hip_error(_e, #expr, __FILE__, __LINE__);      \
      throw Status{LPA_ERR_DEVICE};                       \
    }                                                     \
  } while (0)

enum TimedKind {
  TK_COMPACT = 0,
  TK_BIN0 = 1,  // .. TK_BIN0 + 5
  TK_HUB_PLAN = 7,
  TK_HUB_SCAN = 8,
  TK_HUB_FINISH = 9,
  TK_END_SWEEP = 10,
  TK_HUB_PART = 11,
  TK_OTHER = 12,
  TK_GATE = 13,
  TK_FIRST = 14  // scan kernels of a snapshot first sweep (bins and hub chunks)
};

}  // namespace

struct lpa_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  // deterministic sweeps under capture: the bins of a colour step on a second
  // branch of the graph, beside the hub kernels (fork after the compaction,
  // join before the next step)
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int64_t n = 0, m = 0;
  int64_t n_active = 0;  // vertices with >= 1 stored entry
  // graph
  int64_t *off = nullptr;
  int32_t *idx = nullptr;
  void *w = nullptr;
  int wk = W_UNIT;
  uint32_t *K = nullptr;
  std::vector<int64_t> h_off;
  // state
  int32_t *C = nullptr;
  uint8_t *F = nullptr;
  bool has_labels = false;
  // bins
  BinLimits lim{};
  int32_t variant[NBINS - 1] = {0, 0, 0, 0, 0, 0};  // kernel shape of each bin (BIN_SHAPES)
  bool lists_ready = false;
  // asynchronous mode: the first `early_sweeps` sweeps run in sched[0]'s
  // steps, later sweeps (and verification) in sched[1]'s
  struct AsyncSched {
    int nphase = 16;                  // steps per sweep
    int32_t *list = nullptr;          // vertices by (step, bin)
    std::vector<int64_t> start;       // nphase * NBINS + 1 list bounds
    std::vector<int64_t> hub_chunks, hub_parts;  // hub work per step
  } sched[3];  // early, late, verification (one step: it changes few labels)
  int early_sweeps = 2;
  bool async_by_colour = true;      // steps made of consecutive colour classes (else a hash of the id)
  bool hubs_last = false;           // a step runs the hub bin after the others (else first)
  int32_t snapshot_kernels = 0;     // leading kernels of each step of a run's first sweep that read the
                                    // initial labels (snapshot first sweep; 0 = none, NBINS = all)
  bool rows_strict = false;         // every row's neighbours strictly increase (no repeated neighbour)
  // deterministic schedule
  int32_t *color = nullptr;
  int32_t ncol = 0;
  uint32_t color_seed = 0;
  bool colored = false;
  int32_t color_rounds = 0;
  bool dlists_ready = false;
  int32_t *dlist = nullptr;
  std::vector<int64_t> dstart;  // ncol * NBINS + 1
  // frontier
  int32_t *front = nullptr;
  int32_t *fcount = nullptr;
  int fcount_cap = 0;
  // hubs (sorted by id) and per-step scratch
  int32_t n_hubs = 0;
  int32_t hub_gbits = HUB_PART_GROUP_BITS;  // merge groups of the sweep being emitted
  int64_t hub_chunks_total = 0, hub_parts_total = 0;
  int32_t hub_part_cap = HUB_PART_CAP;
  std::vector<int32_t> h_hub_ids, h_hub_chunks, h_hub_parts;
  std::vector<int64_t> col_hub_chunks, col_hub_parts;  // per colour class (deterministic grids)
  std::vector<int64_t> col_hub_reads;  // per colour class: sum over its hubs of chunks x partitions
  // static hub plans of the colour classes (their hubs in list order): per hub
  // its ordinal and first chunk / partition / merge group inside its class,
  // owners of the class's chunks and groups, and the taken flags the
  // compaction writes; offsets of each class into these arrays
  int32_t *col_ord = nullptr, *col_chunk_owner = nullptr, *col_group_owner = nullptr;
  u64 *col_cstart = nullptr, *col_pstart = nullptr;
  uint8_t *col_taken = nullptr;
  std::vector<int64_t> col_hub_off, col_chunk_off, col_group_off;
  std::vector<int32_t> h_color;
  int32_t *hub_ids = nullptr, *hub_chunks = nullptr, *hub_pbits = nullptr;
  int64_t *hub_pair_base = nullptr, *hub_cnt_base = nullptr;
  u64 *hub_pairs = nullptr;
  int32_t *hub_pcnt = nullptr;
  u64 *hub_partbest = nullptr;
  uint32_t *hub_ovf = nullptr;
  u64 *hub_ovf_count = nullptr;
  int32_t *hub_ord = nullptr;
  u64 *hub_cstart = nullptr, *hub_pstart = nullptr, *hub_gstart = nullptr, *hub_blk = nullptr;
  int32_t *hub_chunk_owner = nullptr, *hub_group_owner = nullptr, *hub_changed = nullptr;
  bool hub_ids_identity = false;  // the hubs are positions 0 .. n_hubs - 1
  u64 *hub_sorder = nullptr;      // chunks of all hubs by the position of their first neighbour
  int64_t hub_sorder_len = 0;
  int32_t *hub_slot_of = nullptr;  // per hub ordinal: frontier entry in the current step, or -1
  int32_t *hub_cur = nullptr;      // per frontier entry: label before the step
  bool hub_static_ok = false;      // the sweeps being emitted may walk the hub chunks in position order
  uint32_t *hub_part_w2 = nullptr, *hub_own_w = nullptr;
  int32_t *hub_part_nd = nullptr;
  // control
  Ctl *ctl = nullptr;
  int32_t *host_done = nullptr;
  int32_t *host_done_dev = nullptr;
  void *scratch_small = nullptr;  // CsrCheck + sums, ModAcc, counters
  int wall_khz = 100000;
  // graphs
  // (mode, prune, sweeps per launch, features, schedule)
  std::map<std::tuple<int, int, int, int, int>, hipGraphExec_t> graphs;
  // learned gate
  bool nonstrict = false;         // the sweeps being emitted use the non-strict tie rule
  bool feat_on = false;           // the sweeps being emitted write gate features
  FeatArgs cur_feat{};
  float *gate_f = nullptr;        // parameters rounded to bf16, held as fp32
  float gate_z = 0.0f;            // logit threshold
  bool gate_loaded = false;
  bool gate_active = false;       // the sweeps being emitted apply the gate
  uint8_t *gskip = nullptr;       // per vertex: gated out in the current sweep
  float *feat = nullptr;          // [n][FEAT_STRIDE] records
  // storage order (reorder.hip): position p holds vertex orig[p]; vertex v sits at pos[v]
  int32_t *orig = nullptr, *pos = nullptr;
  int32_t *perm_tmp = nullptr;    // staging of permuted copies in and out
  float *tx = nullptr;            // trace
  uint8_t *ty = nullptr;
  u64 *tcount = nullptr;
  int64_t tcap = 0;
  uint32_t tthresh = 0xFFFFFFFFu;
  // memory
  std::vector<std::pair<void *, size_t>> owned;  // device allocations and their sizes
  size_t budget = 0, used = 0;
  int cu_count = 256;
  // batched handle (graph g owns vertices [bvptr[g], bvptr[g+1]))
  int32_t ngraphs = 0;
  int32_t nlive = 0;
  int64_t *bvptr = nullptr;
  int32_t *bgid = nullptr, *bgdone = nullptr, *bgiters = nullptr, *bgconv = nullptr;
  int32_t *bgphase = nullptr, *bgcap = nullptr, *bgverified = nullptr, *bgvchanged = nullptr;
  uint8_t *bchg = nullptr;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
};

namespace {

void *dalloc(lpa_graph *g, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  if (g->budget && g->used + bytes > g->budget) throw Status{LPA_ERR_OUT_OF_MEMORY};
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    throw Status{LPA_ERR_OUT_OF_MEMORY};
  }
  g->owned.emplace_back(p, bytes);
  g->used += bytes;
  return p;
}

void dfree(lpa_graph *g, void *p) {
  if (!p) return;
  auto it = std::find_if(g->owned.begin(), g->owned.end(), [p](const auto &o) { return o.first == p; });
  if (it != g->owned.end()) {
    g->used -= it->second;
    g->owned.erase(it);
    (void)hipFree(p);
  }
}

template <class T>
T *dalloc_n(lpa_graph *g, int64_t count) {
  return (T *)dalloc(g, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
}

void drop_graphs(lpa_graph *g) {
  for (auto &kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
  g->graphs.clear();
}

struct Events {
  hipEvent_t e[6] = {};
  Events() {
    for (auto &x : e) HIP_OK(hipEventCreate(&x));
  }
  ~Events() {
    for (auto &x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

int grid_cap(int64_t items, int per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// ---------------------------------------------------------------- host validation

// Checks of a host CSR before any device work; returns a status and fills
// max_weight / not_all_ones for the choice of the internal weight format.
int validate_host(int64_t n, int64_t m, const int64_t *off, const int32_t *idx, const float *w, bool check_sym,
                  uint32_t *max_weight, bool *not_all_ones) {
  if (off[0] != 0 || off[n] != m) return LPA_ERR_INVALID_CSR;
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 65536) nt = 1;
  std::vector<int> bad_off(nt, 0), bad_idx(nt, 0), bad_w(nt, 0), big(nt, 0), ones(nt, 0);
  std::vector<uint32_t> wmax(nt, 0);
  std::vector<u64> fwd(nt, 0), bwd(nt, 0);
  auto mix = [](u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  // each thread keeps its results in locals and stores them once: per-entry
  // stores into the shared per-thread vectors would bounce their cache lines
  // between the threads on every entry
  auto work = [&](unsigned t) {
    const int64_t v0 = n * t / nt, v1 = n * (t + 1) / nt;
    uint32_t l_wmax = 0;
    int l_ones = 0, l_big = 0;
    u64 l_fwd = 0, l_bwd = 0;
    auto done = [&]() {
      wmax[t] = l_wmax;
      ones[t] = l_ones;
      big[t] = l_big;
      fwd[t] = l_fwd;
      bwd[t] = l_bwd;
    };
    for (int64_t v = v0; v < v1; ++v) {
      if (off[v + 1] < off[v] || off[v] < 0 || off[v + 1] > m) {
        bad_off[t] = 1;
        return done();
      }
      u64 deg = 0;
      for (int64_t e = off[v]; e < off[v + 1]; ++e) {
        const int32_t j = idx[e];
        if (j < 0 || (int64_t)j >= n) {
          bad_idx[t] = 1;
          return done();
        }
        uint32_t x = 1;
        if (w) {
          const float f = w[e];
          if (!(f >= 0.0f) || f > 16777216.0f || std::floor(f) != f) {
            bad_w[t] = 1;
            return done();
          }
          x = (uint32_t)f;
          l_wmax = std::max(l_wmax, x);
          l_ones |= x != 1u;
        }
        deg += x;
        if (check_sym) {
          const u64 hx = mix(x + 0x9E3779B97F4A7C15ull);
          l_fwd += mix(((u64)v << 32 | (uint32_t)j) ^ hx);
          l_bwd += mix(((u64)(uint32_t)j << 32 | (u64)v) ^ hx);
        }
      }
      if (deg >= (1ull << 32)) l_big = 1;
    }
    done();
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto &x : th) x.join();
  u64 f = 0, b = 0;
  uint32_t mx = 0;
  bool no = false;
  for (unsigned t = 0; t < nt; ++t) {
    if (bad_off[t] || bad_idx[t]) return LPA_ERR_INVALID_CSR;
    if (bad_w[t]) return LPA_ERR_WEIGHT_NOT_INTEGRAL;
    if (big[t]) return LPA_ERR_TOO_LARGE;
    f += fwd[t];
    b += bwd[t];
    mx = std::max(mx, wmax[t]);
    no |= ones[t] != 0;
  }
  if (check_sym && f != b) return LPA_ERR_INVALID_CSR;
  *max_weight = mx;
  *not_all_ones = no;
  return LPA_OK;
}

// ---------------------------------------------------------------- timing

void tk_begin(lpa_graph *g, hipStream_t st) {
  if (!g->timing) return;
  if (g->ev_used == g->ev_pool.size()) {
    hipEvent_t a, b;
    HIP_OK(hipEventCreate(&a));
    HIP_OK(hipEventCreate(&b));
    g->ev_pool.push_back({a, b});
    g->ev_kind.push_back(0);
  }
  HIP_OK(hipEventRecord(g->ev_pool[g->ev_used].first, st));
}

void tk_end(lpa_graph *g, hipStream_t st, int kind) {
  if (!g->timing) return;
  HIP_OK(hipEventRecord(g->ev_pool[g->ev_used].second, st));
  g->ev_kind[g->ev_used] = kind;
  ++g->ev_used;
}

// ---------------------------------------------------------------- lists

void build_lists(lpa_graph *g, const int32_t *color, const int32_t *cmap, int nphase, int nkeys, int32_t *list,
                 std::vector<int64_t> &starts) {
  int32_t *hist = dalloc_n<int32_t>(g, nkeys);
  HIP_OK(hipMemsetAsync(hist, 0, sizeof(int32_t) * nkeys, g->stream));
  launch_bin_hist(g->off, g->n, color, cmap, nphase, g->lim, hist, nkeys, g->stream);
  std::vector<int32_t> h(nkeys);
  HIP_OK(hipMemcpyAsync(h.data(), hist, sizeof(int32_t) * nkeys, hipMemcpyDeviceToHost, g->stream));
  HIP_OK(hipStreamSynchronize(g->stream));
  starts.assign(nkeys + 1, 0);
  for (int k = 0; k < nkeys; ++k) starts[k + 1] = starts[k] + h[k];
  std::vector<int32_t> cur(nkeys);
  for (int k = 0; k < nkeys; ++k) cur[k] = (int32_t)starts[k];
  HIP_OK(hipMemcpyAsync(hist, cur.data(), sizeof(int32_t) * nkeys, hipMemcpyHostToDevice, g->stream));
  launch_bin_scatter(g->off, g->n, color, cmap, nphase, g->lim, hist, list, nkeys, g->stream);
  HIP_OK(hipStreamSynchronize(g->stream));
  dfree(g, hist);
}

void build_hubs(lpa_graph *g) {
  void **bufs[] = {(void **)&g->hub_ids, (void **)&g->hub_chunks, (void **)&g->hub_pbits,
                   (void **)&g->hub_pair_base, (void **)&g->hub_cnt_base, (void **)&g->hub_pairs,
                   (void **)&g->hub_pcnt, (void **)&g->hub_partbest, (void **)&g->hub_ovf,
                   (void **)&g->hub_ovf_count, (void **)&g->hub_ord, (void **)&g->hub_cstart,
                   (void **)&g->hub_pstart, (void **)&g->hub_gstart, (void **)&g->hub_blk, (void **)&g->hub_chunk_owner,
                   (void **)&g->hub_group_owner,
                   (void **)&g->hub_changed, (void **)&g->hub_part_w2, (void **)&g->hub_own_w,
                   (void **)&g->hub_part_nd, (void **)&g->hub_sorder, (void **)&g->hub_slot_of, (void **)&g->hub_cur};
  for (void **b : bufs) {
    dfree(g, *b);
    *b = nullptr;
  }
  std::vector<int32_t> ids;
  const int32_t lim = g->lim.maxdeg[NBINS - 2];
  for (int64_t v = 0; v < g->n; ++v)
    if (g->h_off[v + 1] - g->h_off[v] > lim) ids.push_back((int32_t)v);
  const size_t nh = ids.size();
  g->n_hubs = (int32_t)nh;
  g->hub_ids_identity = true;
  for (size_t k = 0; k < nh; ++k) g->hub_ids_identity &= ids[k] == (int32_t)k;
  std::vector<int32_t> chunks(nh), pbits(nh);
  std::vector<int64_t> pair_base(nh), cnt_base(nh);
  int64_t pairs = 0, parts = 0, nch = 0;
  for (size_t k = 0; k < nh; ++k) {
    const int64_t deg = g->h_off[ids[k] + 1] - g->h_off[ids[k]];
    chunks[k] = (int32_t)((deg + HUB_CHUNK - 1) / HUB_CHUNK);
    int pb = 0;
    while (pb < HUB_MAX_PBITS && ((int64_t)HUB_PART_TARGET << pb) < deg) ++pb;
    pbits[k] = pb;
    pair_base[k] = pairs;
    cnt_base[k] = parts;
    pairs += ((int64_t)1 << pb) * HUB_PART_CAP;
    parts += (int64_t)1 << pb;
    nch += chunks[k];
  }
  g->hub_chunks_total = nch;
  g->hub_parts_total = parts;
  g->hub_chunk_owner = dalloc_n<int32_t>(g, std::max<int64_t>(1, nch));
  g->hub_group_owner = dalloc_n<int32_t>(g, std::max<int64_t>(1, parts));  // groups of one partition at most
  g->h_hub_ids = ids;
  g->h_hub_chunks = chunks;
  g->h_hub_parts.resize(nh);
  for (size_t k = 0; k < nh; ++k) g->h_hub_parts[k] = 1 << pbits[k];  // bounds the merge work items of any group size
  const int64_t n1 = std::max<int64_t>(1, (int64_t)nh);
  g->hub_ids = dalloc_n<int32_t>(g, n1);
  g->hub_chunks = dalloc_n<int32_t>(g, n1);
  g->hub_pbits = dalloc_n<int32_t>(g, n1);
  g->hub_pair_base = dalloc_n<int64_t>(g, n1);
  g->hub_cnt_base = dalloc_n<int64_t>(g, n1);
  g->hub_ord = dalloc_n<int32_t>(g, n1);
  g->hub_cstart = dalloc_n<u64>(g, n1);
  g->hub_pstart = dalloc_n<u64>(g, n1);
  g->hub_gstart = dalloc_n<u64>(g, n1);
  g->hub_blk = dalloc_n<u64>(g, 3 * (hub_plan_tiles(n1) + 1));
  g->hub_cur = dalloc_n<int32_t>(g, n1);
  g->hub_changed = dalloc_n<int32_t>(g, n1);
  g->hub_own_w = dalloc_n<uint32_t>(g, n1);
  g->hub_part_w2 = dalloc_n<uint32_t>(g, std::max<int64_t>(1, parts));
  g->hub_part_nd = dalloc_n<int32_t>(g, std::max<int64_t>(1, parts));
  g->hub_pairs = dalloc_n<u64>(g, std::max<int64_t>(1, pairs));
  g->hub_pcnt = dalloc_n<int32_t>(g, std::max<int64_t>(1, parts));
  g->hub_partbest = dalloc_n<u64>(g, std::max<int64_t>(1, parts));
  g->hub_ovf_count = dalloc_n<u64>(g, 1);
  g->hub_ovf = dalloc_n<uint32_t>(g, nh ? 4 * HUB_OVERFLOW_CAP : 4);
  HIP_OK(hipMemsetAsync(g->hub_pcnt, 0, sizeof(int32_t) * std::max<int64_t>(1, parts), g->stream));
  HIP_OK(hipMemsetAsync(g->hub_ovf_count, 0, sizeof(u64), g->stream));
  g->hub_slot_of = dalloc_n<int32_t>(g, n1);
  HIP_OK(hipMemsetAsync(g->hub_slot_of, 0xFF, sizeof(int32_t) * n1, g->stream));  // -1: no hub flagged
  // Chunk order of a step that holds every hub: all chunks by the storage
  // position of their first neighbour (rows are sorted, so a chunk covers a
  // position range beginning there); ties by hub and chunk.
  g->hub_sorder_len = 0;
  const char *hub_order = std::getenv("GVELPA_HUB_ORDER");  // testing: "frontier" keeps the step's chunk ids
  if (nch > 0 && !(hub_order && std::strcmp(hub_order, "frontier") == 0)) {
    std::vector<int64_t> at((size_t)nch);
    std::vector<u64> kj((size_t)nch);
    size_t c = 0;
    for (size_t k = 0; k < nh; ++k)
      for (int32_t j = 0; j < chunks[k]; ++j, ++c) {
        at[c] = g->h_off[ids[k]] + (int64_t)j * HUB_CHUNK;
        kj[c] = ((u64)k << 32) | (uint32_t)j;
      }
    int64_t *at_d = dalloc_n<int64_t>(g, nch);
    int32_t *pos_d = dalloc_n<int32_t>(g, nch);
    HIP_OK(hipMemcpyAsync(at_d, at.data(), sizeof(int64_t) * nch, hipMemcpyHostToDevice, g->stream));
    launch_gather_at(g->idx, at_d, nch, pos_d, g->stream);
    std::vector<int32_t> pos((size_t)nch);
    HIP_OK(hipMemcpyAsync(pos.data(), pos_d, sizeof(int32_t) * nch, hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipStreamSynchronize(g->stream));
    dfree(g, at_d);
    dfree(g, pos_d);
    std::vector<int64_t> perm((size_t)nch);
    for (int64_t q = 0; q < nch; ++q) perm[(size_t)q] = q;
    std::sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) {
      return pos[(size_t)x] != pos[(size_t)y] ? pos[(size_t)x] < pos[(size_t)y] : x < y;
    });
    std::vector<u64> sorted((size_t)nch);
    for (int64_t q = 0; q < nch; ++q) sorted[(size_t)q] = kj[(size_t)perm[(size_t)q]];
    g->hub_sorder = dalloc_n<u64>(g, nch);
    HIP_OK(hipMemcpyAsync(g->hub_sorder, sorted.data(), sizeof(u64) * nch, hipMemcpyHostToDevice, g->stream));
    g->hub_sorder_len = nch;
  }
  if (nh) {
    HIP_OK(hipMemcpyAsync(g->hub_ids, ids.data(), sizeof(int32_t) * nh, hipMemcpyHostToDevice, g->stream));
    HIP_OK(hipMemcpyAsync(g->hub_chunks, chunks.data(), sizeof(int32_t) * nh, hipMemcpyHostToDevice, g->stream));
    HIP_OK(hipMemcpyAsync(g->hub_pbits, pbits.data(), sizeof(int32_t) * nh, hipMemcpyHostToDevice, g->stream));
    HIP_OK(hipMemcpyAsync(g->hub_pair_base, pair_base.data(), sizeof(int64_t) * nh, hipMemcpyHostToDevice,
                          g->stream));
    HIP_OK(hipMemcpyAsync(g->hub_cnt_base, cnt_base.data(), sizeof(int64_t) * nh, hipMemcpyHostToDevice,
                          g->stream));
  }
  HIP_OK(hipStreamSynchronize(g->stream));
}

HubArgs hub_args(lpa_graph *g) {
  HubArgs h{};
  h.n_hubs = g->n_hubs;
  h.ids_identity = g->hub_ids_identity ? 1 : 0;
  h.sorder = g->hub_sorder;
  h.sorder_len = g->hub_sorder_len;
  h.slot_of = g->hub_slot_of;
  h.cur = g->hub_cur;
  h.changed = g->hub_changed;
  h.part_cap = g->hub_part_cap;
  h.ids = g->hub_ids;
  h.chunks = g->hub_chunks;
  h.pbits = g->hub_pbits;
  h.pair_base = g->hub_pair_base;
  h.cnt_base = g->hub_cnt_base;
  h.pairs = g->hub_pairs;
  h.pcnt = g->hub_pcnt;
  h.partbest = g->hub_partbest;
  h.ovf = g->hub_ovf;
  h.ovf_count = g->hub_ovf_count;
  h.ord = g->hub_ord;
  h.cstart = g->hub_cstart;
  h.pstart = g->hub_pstart;
  h.chunk_owner = g->hub_chunk_owner;
  h.gstart = g->hub_gstart;
  h.blk = g->hub_blk;
  h.gbits = g->hub_gbits;
  h.group_owner = g->hub_group_owner;
  h.part_w2 = g->hub_part_w2;
  h.part_nd = g->hub_part_nd;
  h.own_w = g->hub_own_w;
  return h;
}

void ensure_fcount(lpa_graph *g, int need) {
  if (g->fcount_cap >= need) return;
  dfree(g, g->fcount);
  g->fcount = dalloc_n<int32_t>(g, need);
  g->fcount_cap = need;
  HIP_OK(hipMemsetAsync(g->fcount, 0, sizeof(int32_t) * need, g->stream));
}

void ensure_colored(lpa_graph *g, uint32_t seed);

// Asynchronous lists: every flagged vertex of a step is processed at once;
// the steps of a sweep are either nphase groups by a hash of the id, or runs
// of consecutive colour classes holding about n_active / nphase vertices each.
void build_async(lpa_graph *g, lpa_graph::AsyncSched &sc) {
  if (!sc.list) sc.list = dalloc_n<int32_t>(g, g->n_active);
  const bool by_colour = g->async_by_colour && sc.nphase > 1;  // a one-step sweep needs no grouping
  std::vector<int32_t> cmap;
  if (by_colour) {
    std::vector<int64_t> csize(std::max(1, g->ncol), 0);
    for (int64_t v = 0; v < g->n; ++v)
      if (g->h_off[v + 1] > g->h_off[v]) csize[g->h_color[v]] += 1;
    cmap.assign(csize.size(), 0);
    const double per = std::max(1.0, (double)g->n_active / sc.nphase);
    int64_t before = 0;
    for (size_t c = 0; c < csize.size(); ++c) {
      cmap[c] = std::min(sc.nphase - 1, (int)((double)before / per));
      before += csize[c];
    }
  }
  int32_t *d_cmap = nullptr;
  if (!cmap.empty()) {
    d_cmap = dalloc_n<int32_t>(g, (int64_t)cmap.size());
    HIP_OK(hipMemcpyAsync(d_cmap, cmap.data(), sizeof(int32_t) * cmap.size(), hipMemcpyHostToDevice, g->stream));
  }
  build_lists(g, by_colour ? g->color : nullptr, d_cmap, sc.nphase, sc.nphase * NBINS, sc.list, sc.start);
  dfree(g, d_cmap);
  ensure_fcount(g, sc.nphase * NBINS);
  sc.hub_chunks.assign(sc.nphase, 0);
  sc.hub_parts.assign(sc.nphase, 0);
  for (size_t k = 0; k < g->h_hub_ids.size(); ++k) {
    const uint32_t v = (uint32_t)g->h_hub_ids[k];
    int ph = 0;
    if (by_colour) ph = cmap[g->h_color[v]];
    else if (sc.nphase > 1) ph = (int)(fmix32(v ^ phase_seed()) % (uint32_t)sc.nphase);
    sc.hub_chunks[ph] += g->h_hub_chunks[k];
    sc.hub_parts[ph] += g->h_hub_parts[k];
  }
}

void ensure_lists(lpa_graph *g) {
  if (g->lists_ready) return;
  drop_graphs(g);
  if (!g->front) g->front = dalloc_n<int32_t>(g, g->n_active);
  build_hubs(g);
  if (g->async_by_colour && (g->sched[0].nphase > 1 || g->sched[1].nphase > 1))
    ensure_colored(g, g->colored ? g->color_seed : 0u);
  build_async(g, g->sched[0]);
  if (g->sched[1].nphase != g->sched[0].nphase) build_async(g, g->sched[1]);
  g->sched[2].nphase = 1;
  if (g->sched[0].nphase != 1 && g->sched[1].nphase != 1) build_async(g, g->sched[2]);
  g->lists_ready = true;
}

// the schedule of an asynchronous sweep: 0 early, 1 late, 2 verification
const lpa_graph::AsyncSched &async_sched(const lpa_graph *g, int which) {
  const lpa_graph::AsyncSched &e = g->sched[0], &l = g->sched[1];
  if (which == 0) return e;
  if (which == 1) return l.nphase == e.nphase ? e : l;
  if (e.nphase == 1) return e;  // verification: a single step
  if (l.nphase == 1) return l;
  return g->sched[2];
}

int max_phases(const lpa_graph *g) { return std::max(g->sched[0].nphase, g->sched[1].nphase); }

void ensure_colored(lpa_graph *g, uint32_t seed) {
  if (g->colored && g->color_seed == seed) return;
  drop_graphs(g);
  if (!g->color) g->color = dalloc_n<int32_t>(g, g->n);
  int32_t *work[2] = {dalloc_n<int32_t>(g, g->n), dalloc_n<int32_t>(g, g->n)};
  int32_t *pending = dalloc_n<int32_t>(g, g->n);
  u64 *pk = dalloc_n<u64>(g, g->n);
  constexpr int MAX_ROUNDS = 1 << 22, BATCH = 64;
  int32_t *counts = dalloc_n<int32_t>(g, MAX_ROUNDS + 2);
  HIP_OK(hipMemsetAsync(counts, 0, sizeof(int32_t) * (MAX_ROUNDS + 2), g->stream));
  launch_color_init(g->off, g->idx, g->color, pk, pending, work[0], counts, g->n, seed, g->orig, g->stream);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((g->n + 3) / 4, (int64_t)g->cu_count * 16));
  int r = 0;
  for (;;) {
    // rounds are queued in batches; a round with an empty list exits at once
    for (int k = 0; k < BATCH && r < MAX_ROUNDS; ++k, ++r)
      launch_color_round(g->off, g->idx, g->color, pk, pending, work[r & 1], work[(r + 1) & 1], counts, r, blocks,
                         g->orig,
                         g->stream);
    int32_t left = 0;
    HIP_OK(hipMemcpyAsync(&left, counts + r, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipStreamSynchronize(g->stream));
    if (left == 0) break;
    if (r >= MAX_ROUNDS) throw Status{LPA_ERR_INTERNAL};
  }
  g->color_rounds = r;
  dfree(g, work[0]);
  dfree(g, work[1]);
  dfree(g, pending);
  dfree(g, pk);
  dfree(g, counts);
  // number of classes = 1 + largest colour
  std::vector<int32_t> &hc = g->h_color;
  hc.assign((size_t)g->n, 0);
  if (g->n) HIP_OK(hipMemcpy(hc.data(), g->color, sizeof(int32_t) * g->n, hipMemcpyDeviceToHost));
  int32_t mx = -1;
  for (int32_t c : hc) mx = std::max(mx, c);
  g->ncol = mx + 1;
  g->color_seed = seed;
  g->colored = true;
  g->dlists_ready = false;
  if (g->async_by_colour && (g->sched[0].nphase > 1 || g->sched[1].nphase > 1)) g->lists_ready = false;
}

// Static hub plans of the colour classes: each class's hub-bin list segment, in
// list order, with every hub's work items numbered inside the class (merge
// groups of one partition, as the deterministic mode merges).
void build_colour_hub_plans(lpa_graph *g) {
  void **bufs[] = {(void **)&g->col_ord, (void **)&g->col_chunk_owner, (void **)&g->col_group_owner,
                   (void **)&g->col_cstart, (void **)&g->col_pstart, (void **)&g->col_taken};
  for (void **b : bufs) {
    dfree(g, *b);
    *b = nullptr;
  }
  const int ncol = std::max(1, g->ncol);
  g->col_hub_off.assign(ncol + 1, 0);
  g->col_chunk_off.assign(ncol + 1, 0);
  g->col_group_off.assign(ncol + 1, 0);
  const size_t nh = g->h_hub_ids.size();
  if (nh == 0) return;
  std::vector<int32_t> list((size_t)g->n_active);
  HIP_OK(hipMemcpyAsync(list.data(), g->dlist, sizeof(int32_t) * g->n_active, hipMemcpyDeviceToHost, g->stream));
  HIP_OK(hipStreamSynchronize(g->stream));
  std::vector<int32_t> ord, cown, gown;
  std::vector<u64> cst, pst;
  ord.reserve(nh);
  cst.reserve(nh);
  pst.reserve(nh);
  for (int c = 0; c < ncol; ++c) {
    const int64_t b0 = g->dstart[(size_t)c * NBINS + HUB_BIN], b1 = g->dstart[(size_t)c * NBINS + HUB_BIN + 1];
    u64 nc = 0, np = 0;
    for (int64_t q = b0; q < b1; ++q) {
      const int32_t v = list[(size_t)q];
      const auto it = std::lower_bound(g->h_hub_ids.begin(), g->h_hub_ids.end(), v);
      if (it == g->h_hub_ids.end() || *it != v) throw Status{LPA_ERR_INTERNAL};  // every hub-bin vertex is a hub
      const int32_t k = (int32_t)(it - g->h_hub_ids.begin());
      const int32_t s = (int32_t)(q - b0);
      ord.push_back(k);
      cst.push_back(nc);
      pst.push_back(np);
      for (int32_t j = 0; j < g->h_hub_chunks[k]; ++j) cown.push_back(s);
      for (int32_t j = 0; j < g->h_hub_parts[k]; ++j) gown.push_back(s);
      nc += (u64)g->h_hub_chunks[k];
      np += (u64)g->h_hub_parts[k];
    }
    g->col_hub_off[c + 1] = (int64_t)ord.size();
    g->col_chunk_off[c + 1] = (int64_t)cown.size();
    g->col_group_off[c + 1] = (int64_t)gown.size();
  }
  auto up = [&](auto *&dst, const auto &src) {
    using T = typename std::decay<decltype(src[0])>::type;
    dst = dalloc_n<T>(g, std::max<int64_t>(1, (int64_t)src.size()));
    if (!src.empty())
      HIP_OK(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, g->stream));
  };
  up(g->col_ord, ord);
  up(g->col_cstart, cst);
  up(g->col_pstart, pst);
  up(g->col_chunk_owner, cown);
  up(g->col_group_owner, gown);
  g->col_taken = dalloc_n<uint8_t>(g, (int64_t)nh);
  HIP_OK(hipStreamSynchronize(g->stream));
}

void ensure_dlists(lpa_graph *g) {
  ensure_lists(g);
  if (g->dlists_ready) return;
  drop_graphs(g);
  if (!g->dlist) g->dlist = dalloc_n<int32_t>(g, g->n_active);
  const int nkeys = std::max(1, g->ncol) * NBINS;
  build_lists(g, g->color, nullptr, 0, nkeys, g->dlist, g->dstart);
  ensure_fcount(g, nkeys);
  g->col_hub_chunks.assign(std::max(1, g->ncol), 0);
  g->col_hub_parts.assign(std::max(1, g->ncol), 0);
  g->col_hub_reads.assign(std::max(1, g->ncol), 0);
  for (size_t k = 0; k < g->h_hub_ids.size(); ++k) {
    const int c = g->h_color[g->h_hub_ids[k]];
    g->col_hub_chunks[c] += g->h_hub_chunks[k];
    g->col_hub_parts[c] += g->h_hub_parts[k];
    g->col_hub_reads[c] += (int64_t)g->h_hub_chunks[k] * g->h_hub_parts[k];
  }
  build_colour_hub_plans(g);
  g->dlists_ready = true;
}

// ---------------------------------------------------------------- sweep emission

BatchArgs batch_args(lpa_graph *g) {
  BatchArgs b{};
  b.ngraphs = g->ngraphs;
  b.vptr = g->bvptr;
  b.gid = g->bgid;
  b.chg = g->bchg;
  b.gdone = g->bgdone;
  b.giters = g->bgiters;
  b.gconv = g->bgconv;
  b.gphase = g->bgphase;
  b.gcap = g->bgcap;
  b.gverified = g->bgverified;
  b.gvchanged = g->bgvchanged;
  b.off = g->off;
  b.F = g->F;
  return b;
}

FeatArgs feat_args(lpa_graph *g, int max_iters, bool trace) {
  FeatArgs f{};
  f.feat = g->feat;
  f.K = g->K;
  f.tx = g->tx;
  f.ty = g->ty;
  f.tcount = g->tcount;
  f.tcap = (u64)g->tcap;
  f.tthresh = g->tthresh;
  f.trace = trace && g->tcap > 0;
  f.max_iters = max_iters;
  return f;
}

ScanArgs base_args(lpa_graph *g, int prune) {
  ScanArgs a{};
  a.f = g->cur_feat;
  a.chg = g->ngraphs ? g->bchg : nullptr;
  a.off = g->off;
  a.idx = g->idx;
  a.w = g->w;
  a.C = g->C;
  a.F = g->F;
  a.ctl = g->ctl;
  a.prune = prune;
  a.nonstrict = g->nonstrict ? 1 : 0;
  a.orig = g->orig;
  return a;
}

// One step: compact the flagged vertices of `list` (bin segments given by
// absolute `bounds` into list/front), then process the bins, hubs first.
// side: a second stream joined to the capture; the step's bin kernels go there
// while the hub kernels stay on st (a deterministic colour step: its vertices
// are pairwise non-adjacent, so bins and hubs neither read nor write each
// other's labels, and both only set flags).
void emit_step(lpa_graph *g, hipStream_t st, const int32_t *list, const int64_t *bounds, int32_t *fcount, int prune,
               int64_t hub_chunks, int64_t hub_parts, int snap_kernels = 0, hipStream_t side = nullptr,
               bool fuse_finish = false, int colour = -1) {
  const int64_t base = bounds[0];
  const int64_t len = bounds[NBINS] - base;
  if (len <= 0) return;
  CompactArgs ca{};
  ca.list = list + base;
  ca.len = len;
  for (int b = 0; b <= NBINS; ++b) ca.bounds[b] = (int32_t)(bounds[b] - base);
  ca.F = g->F;
  ca.front = g->front + base;
  ca.fcount = fcount;
  ca.ctl = g->ctl;
  ca.prune = prune;
  ca.gid = g->ngraphs ? g->bgid : nullptr;
  ca.gdone = g->ngraphs ? g->bgdone : nullptr;
  ca.gskip = g->gate_active ? g->gskip : nullptr;
  ca.f = g->cur_feat;
  // a colour step of the deterministic mode uses its class's static hub plan:
  // the compaction marks which of the class's hubs it takes
  const bool static_hubs = colour >= 0 && g->col_taken && g->hub_gbits == 0 &&
                           bounds[HUB_BIN + 1] > bounds[HUB_BIN];
  if (static_hubs) {
    ca.hub_taken = g->col_taken + g->col_hub_off[colour];
    ca.ovf_count = g->hub_ovf_count;
  }
  tk_begin(g, st);
  launch_compact(ca, grid_cap(len, 2048, 4096), st);
  tk_end(g, st, TK_COMPACT);
  const int max_blocks = g->cu_count * 8;
  bool fork = false;  // the step's bin kernels run on the side branch
  if (side)
    for (int b = 0; b < HUB_BIN; ++b) fork |= bounds[b + 1] > bounds[b];
  if (fork) {
    HIP_OK(hipEventRecord(g->fork_ev, st));
    HIP_OK(hipStreamWaitEvent(side, g->fork_ev, 0));
  }
  const hipStream_t bst = fork ? side : st;  // stream of the bin kernels
  for (int k = 0; k < NBINS; ++k) {
    // bins from the hubs down to degree 1, or (hubs_last) the hubs after the others
    const int b = !g->hubs_last ? NBINS - 1 - k : (k < NBINS - 1 ? NBINS - 2 - k : HUB_BIN);
    const int64_t seg = bounds[b + 1] - bounds[b];
    if (seg <= 0) continue;
    // this kernel reads the initial labels (with the gate's features on, only
    // the bin kernels do: the hub kernels' features need their partitions)
    const bool first = k < snap_kernels && !(b == HUB_BIN && g->feat_on);
    ScanArgs a = base_args(g, prune);
    a.bin = b;
    a.front = g->front + bounds[b];
    a.fcount = fcount + b;
    if (b == HUB_BIN && first) {
      // snapshot first sweep: one best key per chunk, maximum per hub
      HubArgs h = hub_args(g);
      h.first = 1;
      tk_begin(g, st);
      launch_hub_plan(a, h, seg, grid_cap(seg, 1, max_blocks), std::max(1, std::min(hub_plan_tiles(seg), max_blocks)),
                      st);
      tk_end(g, st, TK_HUB_PLAN);
      tk_begin(g, st);
      launch_hub_first_chunk(g->wk, grid_cap(hub_chunks, 1, max_blocks * 2), st, a, h);
      tk_end(g, st, TK_FIRST);
      a.bin = FIRST_SLOT;
      tk_begin(g, st);
      launch_hub_finish(grid_cap(seg, 4, max_blocks), grid_cap(hub_chunks, 1, max_blocks * 2), prune, false,
                        fuse_finish, st, a, h);
      tk_end(g, st, TK_HUB_FINISH);
    } else if (b == HUB_BIN) {
      HubArgs h = hub_args(g);
      // a step that may hold every hub walks their chunks in position order
      h.static_order = g->hub_static_ok && g->hub_sorder_len > 0 && seg == g->n_hubs;
      if (static_hubs) {
        // the class's static plan: its hub list is the frontier, untaken hubs are skipped
        const int64_t ho = g->col_hub_off[colour];
        h.static_plan = 1;
        h.taken = g->col_taken + ho;
        h.static_count = seg;
        h.static_chunks = g->col_chunk_off[colour + 1] - g->col_chunk_off[colour];
        h.static_groups = g->col_group_off[colour + 1] - g->col_group_off[colour];
        h.ord = g->col_ord + ho;
        h.cstart = g->col_cstart + ho;
        h.pstart = g->col_pstart + ho;
        h.gstart = g->col_pstart + ho;  // one partition per merge group
        h.chunk_owner = g->col_chunk_owner + g->col_chunk_off[colour];
        h.group_owner = g->col_group_owner + g->col_group_off[colour];
        h.cur += ho;
        h.changed += ho;
        h.own_w += ho;
        a.front = g->dlist + bounds[HUB_BIN];
      } else {
        tk_begin(g, st);
        launch_hub_plan(a, h, seg, grid_cap(seg, 1, max_blocks),
                        std::max(1, std::min(hub_plan_tiles(seg), max_blocks)), st);
        tk_end(g, st, TK_HUB_PLAN);
      }
      tk_begin(g, st);
      launch_hub_chunk(g->wk, grid_cap(hub_chunks, 1, max_blocks * 2), st, a, h);
      tk_end(g, st, TK_HUB_SCAN);
      tk_begin(g, st);
      launch_hub_part(grid_cap(hub_parts, 1, max_blocks * 2), g->feat_on, st, a, h);
      tk_end(g, st, TK_HUB_PART);
      tk_begin(g, st);
      launch_hub_finish(grid_cap(seg, 4, max_blocks), grid_cap(hub_chunks, 1, max_blocks * 2), prune, g->feat_on,
                        fuse_finish, st, a, h);
      tk_end(g, st, TK_HUB_FINISH);
    } else if (first) {
      const int per_block = bin_vertices_per_block(b, g->variant[b]);
      tk_begin(g, st);
      launch_first_bin(b, g->variant[b], g->wk, g->feat_on, grid_cap(seg, per_block, max_blocks), st, a);
      tk_end(g, st, TK_FIRST);
    } else {
      const int per_block = bin_vertices_per_block(b, g->variant[b]);
      tk_begin(g, bst);
      launch_scan_bin(b, g->variant[b], g->wk, g->feat_on, grid_cap(seg, per_block, max_blocks), bst, a);
      tk_end(g, bst, TK_BIN0 + b);
    }
  }
  if (fork) {
    HIP_OK(hipEventRecord(g->join_ev, side));
    HIP_OK(hipStreamWaitEvent(st, g->join_ev, 0));
  }
}

// snap_kernels: leading kernels of every step that read the initial labels
// (a run's first sweep in the asynchronous mode; the caller checks that the
// run starts from the initial labels and that the rows allow it).
void emit_sweep(lpa_graph *g, hipStream_t st, int mode, int prune, int late, int snap_kernels = 0) {
  // the deterministic mode's colour steps hold few hubs each: every partition
  // its own merge work item, merged in parallel (its steps are latency-bound)
  g->hub_gbits = mode == LPA_MODE_DETERMINISTIC ? 0 : HUB_PART_GROUP_BITS;
  g->hub_static_ok = mode == LPA_MODE_ASYNC;
  if (g->gate_active) {
    tk_begin(g, st);
    launch_gate_pass(g->ctl, g->gate_f, g->gate_z, g->cur_feat, g->F, g->gskip, g->n, g->cu_count,
                     g->ngraphs ? g->bgid : nullptr, g->ngraphs ? g->bgphase : nullptr, st);
    tk_end(g, st, TK_GATE);
  }
  if (mode == LPA_MODE_DETERMINISTIC) {
    // under capture, each colour step's bins form a branch beside its hub kernels
    const hipStream_t side = st == g->cap_stream ? g->side_stream : nullptr;
    // a colour step with little hub work decides and marks its hubs in one
    // kernel (every chunk re-reads its hub's partition maxima: at most
    // HUB_FUSED_READS of them in the step)
    for (int c = 0; c < g->ncol; ++c)
      emit_step(g, st, g->dlist, &g->dstart[(size_t)c * NBINS], g->fcount + (size_t)c * NBINS, prune,
                g->col_hub_chunks[c], g->col_hub_parts[c], 0, side, g->col_hub_reads[c] <= HUB_FUSED_READS, c);
  } else {
    const lpa_graph::AsyncSched &sc = async_sched(g, late);
    for (int ph = 0; ph < sc.nphase; ++ph)
      emit_step(g, st, sc.list, &sc.start[(size_t)ph * NBINS], g->fcount + (size_t)ph * NBINS, prune,
                sc.hub_chunks[ph], sc.hub_parts[ph], snap_kernels);
  }
  const int nfc = mode == LPA_MODE_DETERMINISTIC ? std::max(1, g->ncol) * NBINS : max_phases(g) * NBINS;
  tk_begin(g, st);
  if (g->ngraphs) launch_batch_end(g->ctl, batch_args(g), st);
  launch_end_sweep(g->ctl, g->fcount, nfc, g->host_done_dev, st);
  if (mode == LPA_MODE_ASYNC && prune) launch_dense_fill(g->ctl, g->off, g->F, g->n, st);
  tk_end(g, st, TK_END_SWEEP);
}

// One HIP graph holding `sweeps` consecutive sweeps (their kernels exit at
// once after the stop test holds), captured once per (mode, prune, sweeps).
// A graph of `sweeps` consecutive sweeps starting at sweep `first` (which
// selects the asynchronous schedule of each).
hipGraphExec_t sweep_graph(lpa_graph *g, int mode, int prune, int sweeps, int first, int verify = 0,
                           int snap = 0) {
  // captured kernels embed the feature arguments (trace switch, sweep cap)
  const int fcode = g->feat_on ? 1 + 2 * g->cur_feat.trace + 4 * g->gate_active + 8 * g->cur_feat.max_iters : 0;
  // only the early/late split of the covered sweeps matters
  const int fkey = mode == LPA_MODE_DETERMINISTIC ? 0
                   : verify                       ? 2
                   : sweeps == 1                  ? (first >= g->early_sweeps ? 1 : 0)
                                                  : 3 + std::min(first, g->early_sweeps);
  if (first != 0 || verify) snap = 0;
  auto key = std::make_tuple(mode, prune, sweeps, fcode,
                             fkey + (g->nonstrict ? 1000 : 0) + (g->hubs_last ? 2000 : 0) + 4000 * snap);
  auto it = g->graphs.find(key);
  if (it != g->graphs.end()) return it->second;
  hipGraph_t graph = nullptr;
  HIP_OK(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int s = 0; s < sweeps; ++s)
    emit_sweep(g, g->cap_stream, mode, prune, verify ? 2 : (first + s >= g->early_sweeps ? 1 : 0), s == 0 ? snap : 0);
  HIP_OK(hipStreamEndCapture(g->cap_stream, &graph));
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiateWithFlags(&exec, graph, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) throw Status{LPA_ERR_DEVICE};
  g->graphs[key] = exec;
  return exec;
}

void copy_in(lpa_graph *g, void *dst, const void *src, size_t bytes, unsigned flags) {
  HIP_OK(hipMemcpyAsync(dst, src, bytes, (flags & LPA_FLAG_DEVICE_PTRS) ? hipMemcpyDeviceToDevice
                                                                         : hipMemcpyHostToDevice, g->stream));
}

void copy_out(lpa_graph *g, void *dst, const void *src, size_t bytes, unsigned flags) {
  HIP_OK(hipMemcpyAsync(dst, src, bytes, (flags & LPA_FLAG_DEVICE_PTRS) ? hipMemcpyDeviceToDevice
                                                                         : hipMemcpyDeviceToHost, g->stream));
}

// Vertex arrays cross the boundary in vertex-id order; inside they are kept in
// storage order (position p holds vertex orig[p]).
int32_t *perm_stage(lpa_graph *g) {
  if (!g->perm_tmp) g->perm_tmp = dalloc_n<int32_t>(g, g->n);
  return g->perm_tmp;
}

template <class T>
void gather_dev(T *dst, const T *src, const int32_t *index, int64_t n, hipStream_t st) {
  if constexpr (sizeof(T) == 4) launch_gather_i32((int32_t *)dst, (const int32_t *)src, index, n, st);
  else launch_gather_u8((uint8_t *)dst, (const uint8_t *)src, index, n, st);
}

// dst[p] = src[orig[p]] (src: caller order, host or device per flags)
template <class T>
void vertex_in(lpa_graph *g, T *dst, const T *src, unsigned flags) {
  if (!g->orig) {
    copy_in(g, dst, src, sizeof(T) * g->n, flags);
    return;
  }
  const T *from = src;
  if (!(flags & LPA_FLAG_DEVICE_PTRS)) {
    T *stage = (T *)perm_stage(g);
    HIP_OK(hipMemcpyAsync(stage, src, sizeof(T) * g->n, hipMemcpyHostToDevice, g->stream));
    from = stage;
  }
  gather_dev<T>(dst, from, g->orig, g->n, g->stream);
}

// dst[v] = src[pos[v]] (dst: caller order, host or device per flags)
template <class T>
void vertex_out(lpa_graph *g, T *dst, const T *src, unsigned flags) {
  if (!g->orig) {
    copy_out(g, dst, src, sizeof(T) * g->n, flags);
    return;
  }
  if (flags & LPA_FLAG_DEVICE_PTRS) {
    gather_dev<T>(dst, src, g->pos, g->n, g->stream);
  } else {
    T *stage = (T *)perm_stage(g);
    gather_dev<T>(stage, src, g->pos, g->n, g->stream);
    HIP_OK(hipMemcpyAsync(dst, stage, sizeof(T) * g->n, hipMemcpyDeviceToHost, g->stream));
  }
}

template <class Fn>
int run_guarded(lpa_graph *g, Fn &&fn) {
  if (!g) return LPA_ERR_INVALID_ARG;
  try {
    HIP_OK(hipSetDevice(g->device));
    return fn();
  } catch (Status s) {
    return s.code;
  } catch (std::bad_alloc &) {
    return LPA_ERR_OUT_OF_MEMORY;
  }
}

}  // namespace

void gvelpa::note_hip_error(int err, const char *what, const char *file, int line) {
  const char *base = std::strrchr(file, '/');
  last_error = std::string(hipGetErrorString((hipError_t)err)) + " in " + what + " (" + (base ? base + 1 : file) +
               ":" + std::to_string(line) + ")";
}

// ======================================================================== ABI

extern "C" {

const char *lpa_last_error_detail(void) { return last_error.c_str(); }

const char *lpa_status_string(int status) {
  switch (status) {
    case LPA_OK: return "ok";
    case LPA_ERR_INVALID_ARG: return "invalid argument";
    case LPA_ERR_INVALID_CSR: return "invalid CSR (offsets or indices)";
    case LPA_ERR_WEIGHT_NOT_INTEGRAL: return "weights must be finite integers in [0, 2^24]";
    case LPA_ERR_TOO_LARGE: return "graph too large (n >= 2^31 or a weighted degree >= 2^32)";
    case LPA_ERR_OUT_OF_MEMORY: return "out of device memory";
    case LPA_ERR_DEVICE: return "no usable GPU or a HIP call failed";
    case LPA_ERR_NO_GATE: return "no gate network loaded";
    case LPA_ERR_INTERNAL: return "internal error reported by a kernel";
    default: return "unknown status";
  }
}

void lpa_destroy(lpa_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  drop_graphs(g);
  for (auto &p : g->ev_pool) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  for (auto &o : g->owned) (void)hipFree(o.first);
  if (g->host_done) (void)hipHostFree(g->host_done);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->side_stream) (void)hipStreamDestroy(g->side_stream);
  if (g->fork_ev) (void)hipEventDestroy(g->fork_ev);
  if (g->join_ev) (void)hipEventDestroy(g->join_ev);
  delete g;
}

// lpa_create, with the graph ranges of a batch (n_graphs = 0: one graph):
// the storage order keeps every graph's vertices inside its range.
static int create_graph(lpa_graph **out, int64_t n, int64_t m, const int64_t *offsets, const int32_t *indices,
                        const float *weights, int device, void *hip_stream, unsigned flags, int32_t n_graphs,
                        const int64_t *graph_vptr) {
  if (!out) return LPA_ERR_INVALID_ARG;
  *out = nullptr;
  if (n < 0 || m < 0 || !offsets || (m > 0 && !indices)) return LPA_ERR_INVALID_ARG;
  if (n >= ((int64_t)1 << 31)) return LPA_ERR_TOO_LARGE;
  const bool host_in = !(flags & LPA_FLAG_DEVICE_PTRS);
  uint32_t host_wmax = 0;
  bool host_not_ones = false;
  if (host_in) {
    // host arrays are validated before any device work
    int v = validate_host(n, m, offsets, indices, weights, flags & LPA_FLAG_CHECK_SYMMETRIC, &host_wmax,
                          &host_not_ones);
    if (v != LPA_OK) return v;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return LPA_ERR_DEVICE;
  }
  if (device < 0 || device >= ndev) return LPA_ERR_INVALID_ARG;
  lpa_graph *g = new (std::nothrow) lpa_graph();
  if (!g) return LPA_ERR_OUT_OF_MEMORY;
  g->device = device;
  g->stream = (hipStream_t)hip_stream;
  g->n = n;
  g->m = m;
  if (const char *b = std::getenv("GVELPA_DEVICE_BUDGET_BYTES")) g->budget = (size_t)std::strtoull(b, nullptr, 10);
  if (const char *c = std::getenv("GVELPA_HUB_PART_CAP"))  // testing: force the partition spill path
    g->hub_part_cap = (int32_t)std::max(1L, std::min((long)HUB_PART_CAP, std::strtol(c, nullptr, 10)));
  for (int b = 0; b < NBINS - 1; ++b) g->lim.maxdeg[b] = DEFAULT_BIN_MAXDEG[b];
  // asynchronous schedule: 16 colour-grouped steps for the first two sweeps,
  // 4 afterwards (late sweeps change few labels; fewer steps cost fewer launches)
  g->sched[0].nphase = 16;
  g->sched[1].nphase = 4;
  g->early_sweeps = 2;
  int rc = run_guarded(g, [&]() -> int {
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, device));
    g->cu_count = prop.multiProcessorCount;
    HIP_OK(hipDeviceGetAttribute(&g->wall_khz, hipDeviceAttributeWallClockRate, device));
    HIP_OK(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
    HIP_OK(hipStreamCreateWithFlags(&g->side_stream, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&g->join_ev, hipEventDisableTiming));
    HIP_OK(hipHostMalloc((void **)&g->host_done, sizeof(int32_t), hipHostMallocMapped));
    *g->host_done = 0;
    HIP_OK(hipHostGetDevicePointer((void **)&g->host_done_dev, g->host_done, 0));
    const bool dev = flags & LPA_FLAG_DEVICE_PTRS;
    // host copy of the offsets (schedule planning) and their basic checks
    g->h_off.resize((size_t)n + 1);
    if (dev) HIP_OK(hipMemcpy(g->h_off.data(), offsets, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    else std::memcpy(g->h_off.data(), offsets, sizeof(int64_t) * (n + 1));
    if (g->h_off[0] != 0 || g->h_off[n] != m) return LPA_ERR_INVALID_CSR;
    g->scratch_small = dalloc(g, 4096);
    CsrCheck *chk = (CsrCheck *)g->scratch_small;
    HIP_OK(hipMemsetAsync(chk, 0, 4096, g->stream));
    if (dev) {
      g->off = (int64_t *)offsets;
      g->idx = (int32_t *)indices;
    } else {
      g->off = dalloc_n<int64_t>(g, n + 1);
      g->idx = dalloc_n<int32_t>(g, m);
      HIP_OK(hipMemcpyAsync(g->off, offsets, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, g->stream));
      if (m) HIP_OK(hipMemcpyAsync(g->idx, indices, sizeof(int32_t) * m, hipMemcpyHostToDevice, g->stream));
    }
    const float *wdev = nullptr;
    float *wtmp = nullptr;
    if (weights) {
      if (dev) wdev = weights;
      else {
        wtmp = dalloc_n<float>(g, m);
        if (m) HIP_OK(hipMemcpyAsync(wtmp, weights, sizeof(float) * m, hipMemcpyHostToDevice, g->stream));
        wdev = wtmp;
      }
    }
    CsrCheck h{};
    if (dev) {
      launch_check_offsets(g->off, n, chk, g->stream);
      if (m) launch_check_edges(g->idx, wdev, m, n, chk, g->stream);
      HIP_OK(hipMemcpyAsync(&h, chk, sizeof(h), hipMemcpyDeviceToHost, g->stream));
      HIP_OK(hipStreamSynchronize(g->stream));
      if (h.bad_offsets || h.bad_index) return LPA_ERR_INVALID_CSR;
      if (h.bad_weight) return LPA_ERR_WEIGHT_NOT_INTEGRAL;
    } else {
      h.max_weight = host_wmax;
      h.not_all_ones = host_not_ones ? 1 : 0;
    }
    // internal weight format: none when every weight is 1, else uint8 or uint32
    g->wk = W_UNIT;
    if (weights && m && h.not_all_ones) g->wk = h.max_weight <= 255 ? W_U8 : W_U32;
    if (g->wk != W_UNIT) {
      g->w = dalloc(g, (size_t)m * (g->wk == W_U8 ? 1 : 4));
      launch_convert_weights(wdev, m, g->wk, g->w, g->stream);
    }
    if (wtmp) {
      HIP_OK(hipStreamSynchronize(g->stream));
      dfree(g, wtmp);
    }
    // storage order: decreasing degree (within each graph of a batch)
    if (!(flags & LPA_FLAG_NO_REORDER) && n > 1 && m > 0 && n < ((int64_t)1 << 31) - 1) {
      int32_t *gid = nullptr;
      int64_t *dvptr = nullptr;
      if (n_graphs > 0) {
        dvptr = dalloc_n<int64_t>(g, n_graphs + 1);
        gid = dalloc_n<int32_t>(g, n);
        HIP_OK(hipMemcpyAsync(dvptr, graph_vptr, sizeof(int64_t) * (n_graphs + 1), hipMemcpyHostToDevice,
                              g->stream));
        BatchArgs ba{};
        ba.ngraphs = n_graphs;
        ba.vptr = dvptr;
        ba.gid = gid;
        launch_batch_gid(ba, g->stream);
      }
      g->orig = dalloc_n<int32_t>(g, n);
      g->pos = dalloc_n<int32_t>(g, n);
      int64_t *noff = dalloc_n<int64_t>(g, n + 1);
      u64 *keys = dalloc_n<u64>(g, 2 * n + 1);
      const int64_t tb = order_temp_bytes(n);
      void *scr = dalloc(g, (size_t)std::max<int64_t>(tb, 1));
      HIP_OK(build_order(g->off, gid, n, g->orig, g->pos, noff, keys, scr, tb, g->stream));
      int32_t *nidx = dalloc_n<int32_t>(g, m);
      void *nw = g->wk == W_UNIT ? nullptr : dalloc(g, (size_t)m * (g->wk == W_U8 ? 1 : 4));
      launch_permute_rows(g->off, g->idx, g->w, g->wk, g->orig, g->pos, noff, nidx, nw, n, g->stream);
      HIP_OK(hipGetLastError());
      HIP_OK(hipStreamSynchronize(g->stream));
      dfree(g, scr);
      dfree(g, keys);
      dfree(g, gid);
      dfree(g, dvptr);
      if (!dev) {  // borrowed arrays stay with the caller
        dfree(g, g->off);
        dfree(g, g->idx);
      }
      dfree(g, g->w);
      g->off = noff;
      g->idx = nidx;
      g->w = nw;
      HIP_OK(hipMemcpy(g->h_off.data(), noff, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
      // every row sorted by neighbour position, in chunks of rows of at most CH entries
      const int64_t CH = std::min<int64_t>(m, (int64_t)1 << 28);
      const size_t wb = g->wk == W_U8 ? 1 : (g->wk == W_U32 ? 4 : 0);
      u64 *rkeys = dalloc_n<u64>(g, 2 * CH);
      int32_t *rperm = wb ? dalloc_n<int32_t>(g, 2 * CH) : nullptr;
      void *wcopy = wb ? dalloc(g, (size_t)CH * wb) : nullptr;
      const int64_t rtb = row_sort_temp_bytes(CH);
      void *rtmp = dalloc(g, (size_t)std::max<int64_t>(rtb, 1));
      for (int64_t r0 = 0; r0 < n;) {
        // rows [r0, r1) whose entries fit CH; a single longer row stays unsorted (the
        // order of a row's entries does not change any result)
        int64_t r1 = std::upper_bound(g->h_off.begin() + r0 + 1, g->h_off.end(), g->h_off[r0] + CH) -
                     g->h_off.begin() - 1;
        if (r1 <= r0) r1 = r0 + 1;
        const int64_t len = g->h_off[r1] - g->h_off[r0];
        if (len <= CH)
          HIP_OK(sort_rows_chunk(g->off, r0, r1, g->h_off[r0], len, g->idx, g->w, g->wk, rkeys, rperm, wcopy, rtmp,
                                 rtb, g->stream));
        r0 = r1;
      }
      HIP_OK(hipStreamSynchronize(g->stream));
      dfree(g, rtmp);
      dfree(g, wcopy);
      dfree(g, rperm);
      dfree(g, rkeys);
    }
    g->K = dalloc_n<uint32_t>(g, n);
    launch_weighted_degree(g->off, g->w, g->wk, n, g->K, chk, g->stream);
    if (n) launch_check_rows(g->off, g->idx, n, chk, g->stream);
    const bool dev_sym = dev && (flags & LPA_FLAG_CHECK_SYMMETRIC);
    if (dev_sym) launch_check_symmetric(g->off, g->idx, g->w, g->wk, n, chk, g->stream);
    u64 sums[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(&h, chk, sizeof(h), hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipMemcpyAsync(sums, (u64 *)(chk + 1), sizeof(sums), hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipStreamSynchronize(g->stream));
    if (h.big_degree) return LPA_ERR_TOO_LARGE;
    g->rows_strict = !h.rows_not_strict;
    if (dev_sym && sums[0] != sums[1]) return LPA_ERR_INVALID_CSR;
    int64_t act = 0;
    for (int64_t v = 0; v < n; ++v) act += g->h_off[v + 1] > g->h_off[v];
    g->n_active = act;
    g->C = dalloc_n<int32_t>(g, n);
    g->F = dalloc_n<uint8_t>(g, n);
    g->ctl = dalloc_n<Ctl>(g, 1);
    HIP_OK(hipMemsetAsync(g->ctl, 0, sizeof(Ctl), g->stream));
    launch_init_state(g->off, g->C, g->F, n, 1, 1, 0, g->orig, g->stream);
    HIP_OK(hipStreamSynchronize(g->stream));
    return LPA_OK;
  });
  if (rc != LPA_OK) {
    lpa_destroy(g);
    return rc;
  }
  *out = g;
  return LPA_OK;
}

int lpa_create(lpa_graph **out, int64_t n, int64_t m, const int64_t *offsets, const int32_t *indices,
               const float *weights, int device, void *hip_stream, unsigned flags) {
  return create_graph(out, n, m, offsets, indices, weights, device, hip_stream, flags, 0, nullptr);
}

int lpa_batch_create(lpa_graph **out, int32_t n_graphs, const int64_t *graph_vptr, int64_t n, int64_t m,
                     const int64_t *offsets, const int32_t *indices, const float *weights, int device,
                     void *hip_stream, unsigned flags) {
  if (!out) return LPA_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_graphs < 1 || !graph_vptr || graph_vptr[0] != 0 || graph_vptr[n_graphs] != n) return LPA_ERR_INVALID_ARG;
  int32_t live = 0;
  for (int32_t k = 0; k < n_graphs; ++k) {
    if (graph_vptr[k + 1] < graph_vptr[k]) return LPA_ERR_INVALID_ARG;
    live += graph_vptr[k + 1] > graph_vptr[k];
  }
  lpa_graph *g = nullptr;
  int rc = create_graph(&g, n, m, offsets, indices, weights, device, hip_stream, flags, n_graphs, graph_vptr);
  if (rc != LPA_OK) return rc;
  rc = run_guarded(g, [&]() -> int {
    // entries may not cross graphs (checked on the host offsets copy and the indices)
    g->ngraphs = n_graphs;
    g->nlive = live;
    g->bvptr = dalloc_n<int64_t>(g, n_graphs + 1);
    g->bgid = dalloc_n<int32_t>(g, n);
    g->bchg = dalloc_n<uint8_t>(g, n);
    g->bgdone = dalloc_n<int32_t>(g, n_graphs);
    g->bgiters = dalloc_n<int32_t>(g, n_graphs);
    g->bgconv = dalloc_n<int32_t>(g, n_graphs);
    g->bgphase = dalloc_n<int32_t>(g, n_graphs);
    g->bgcap = dalloc_n<int32_t>(g, n_graphs);
    g->bgverified = dalloc_n<int32_t>(g, n_graphs);
    g->bgvchanged = dalloc_n<int32_t>(g, n_graphs);
    HIP_OK(hipMemcpyAsync(g->bvptr, graph_vptr, sizeof(int64_t) * (n_graphs + 1), hipMemcpyHostToDevice,
                          g->stream));
    launch_batch_gid(batch_args(g), g->stream);
    int32_t *bad = (int32_t *)((char *)g->scratch_small + 2048);
    HIP_OK(hipMemsetAsync(bad, 0, sizeof(int32_t), g->stream));
    launch_check_block_diagonal(g->off, g->idx, g->bgid, g->n, bad, g->stream);
    int32_t hb = 0;
    HIP_OK(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipStreamSynchronize(g->stream));
    return hb ? LPA_ERR_INVALID_CSR : LPA_OK;
  });
  if (rc != LPA_OK) {
    lpa_destroy(g);
    return rc;
  }
  *out = g;
  return LPA_OK;
}

int lpa_batch_stats(const lpa_graph *gc, int32_t *iterations, int32_t *converged) {
  lpa_graph *g = const_cast<lpa_graph *>(gc);
  return run_guarded(g, [&]() -> int {
    if (!g->ngraphs) return LPA_ERR_INVALID_ARG;
    if (iterations)
      HIP_OK(hipMemcpy(iterations, g->bgiters, sizeof(int32_t) * g->ngraphs, hipMemcpyDeviceToHost));
    if (converged) HIP_OK(hipMemcpy(converged, g->bgconv, sizeof(int32_t) * g->ngraphs, hipMemcpyDeviceToHost));
    return LPA_OK;
  });
}

int lpa_batch_verify_stats(const lpa_graph *gc, int32_t *verified, int32_t *verify_changed) {
  lpa_graph *g = const_cast<lpa_graph *>(gc);
  return run_guarded(g, [&]() -> int {
    if (!g->ngraphs) return LPA_ERR_INVALID_ARG;
    if (verified)
      HIP_OK(hipMemcpy(verified, g->bgverified, sizeof(int32_t) * g->ngraphs, hipMemcpyDeviceToHost));
    if (verify_changed)
      HIP_OK(hipMemcpy(verify_changed, g->bgvchanged, sizeof(int32_t) * g->ngraphs, hipMemcpyDeviceToHost));
    return LPA_OK;
  });
}

int lpa_gate_load(lpa_graph *g, const float *params, float threshold) {
  return run_guarded(g, [&]() -> int {
    if (!params || !(threshold >= 0.0f) || !(threshold <= 1.0f)) return LPA_ERR_INVALID_ARG;
    float bf[GATE_PARAMS];
    for (int k = 0; k < GATE_PARAMS; ++k) {
      if (!std::isfinite(params[k])) return LPA_ERR_INVALID_ARG;
      uint32_t u;
      std::memcpy(&u, &params[k], 4);
      u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
      u &= 0xFFFF0000u;
      std::memcpy(&bf[k], &u, 4);
    }
    if (!g->gate_f) g->gate_f = dalloc_n<float>(g, GATE_PARAMS);
    HIP_OK(hipMemcpy(g->gate_f, bf, sizeof(bf), hipMemcpyHostToDevice));
    // p >= threshold  <=>  logit >= log(threshold / (1 - threshold))
    if (threshold <= 0.0f) g->gate_z = -INFINITY;
    else if (threshold >= 1.0f) g->gate_z = INFINITY;
    else g->gate_z = (float)std::log((double)threshold / (1.0 - (double)threshold));
    g->gate_loaded = true;
    drop_graphs(g);
    return LPA_OK;
  });
}

int lpa_set_trace(lpa_graph *g, int64_t capacity, double probability) {
  return run_guarded(g, [&]() -> int {
    if (capacity < 0 || !(probability >= 0.0) || !(probability <= 1.0)) return LPA_ERR_INVALID_ARG;
    dfree(g, g->tx);
    dfree(g, g->ty);
    dfree(g, g->tcount);
    g->tx = nullptr;
    g->ty = nullptr;
    g->tcount = nullptr;
    g->tcap = capacity;
    g->tthresh = probability >= 1.0 ? 0xFFFFFFFFu : (uint32_t)(probability * 4294967296.0);
    if (capacity > 0) {
      g->tx = dalloc_n<float>(g, capacity * NFEAT);
      g->ty = dalloc_n<uint8_t>(g, capacity);
      g->tcount = dalloc_n<u64>(g, 1);
      HIP_OK(hipMemsetAsync(g->tcount, 0, sizeof(u64), g->stream));
      HIP_OK(hipStreamSynchronize(g->stream));
    }
    drop_graphs(g);
    return LPA_OK;
  });
}

int lpa_gate_trace(const lpa_graph *gc, float *features, uint8_t *targets, int64_t capacity, int64_t *count,
                   unsigned flags) {
  lpa_graph *g = const_cast<lpa_graph *>(gc);
  return run_guarded(g, [&]() -> int {
    if (!count) return LPA_ERR_INVALID_ARG;
    u64 c = 0;
    if (g->tcount) HIP_OK(hipMemcpy(&c, g->tcount, sizeof(u64), hipMemcpyDeviceToHost));
    const int64_t have = std::min<int64_t>((int64_t)c, g->tcap);
    *count = have;
    if (!features) return LPA_OK;
    if (!targets || capacity < have) return LPA_ERR_INVALID_ARG;
    if (have) {
      copy_out(g, features, g->tx, sizeof(float) * NFEAT * have, flags);
      copy_out(g, targets, g->ty, have, flags);
      HIP_OK(hipStreamSynchronize(g->stream));
    }
    return LPA_OK;
  });
}

int lpa_set_bins(lpa_graph *g, const int32_t *max_degree, int32_t count) {
  return run_guarded(g, [&]() -> int {
    BinLimits lim{};
    if (!max_degree) {
      for (int b = 0; b < NBINS - 1; ++b) lim.maxdeg[b] = DEFAULT_BIN_MAXDEG[b];
    } else {
      if (count != NBINS - 1) return LPA_ERR_INVALID_ARG;
      for (int b = 0; b < NBINS - 1; ++b) {
        // a table must have room for every distinct label of its vertices
        if (max_degree[b] < 0 || max_degree[b] >= BIN_SLOTS[b]) return LPA_ERR_INVALID_ARG;
        if (b && max_degree[b] < max_degree[b - 1]) return LPA_ERR_INVALID_ARG;
        lim.maxdeg[b] = max_degree[b];
      }
    }
    if (std::memcmp(&lim, &g->lim, sizeof(lim)) != 0) {
      g->lim = lim;
      g->lists_ready = false;
      g->dlists_ready = false;
      drop_graphs(g);
    }
    return LPA_OK;
  });
}

int lpa_set_variants(lpa_graph *g, const int32_t *variant, int32_t count) {
  return run_guarded(g, [&]() -> int {
    int32_t v[NBINS - 1] = {0, 0, 0, 0, 0, 0};
    if (variant) {
      if (count != NBINS - 1) return LPA_ERR_INVALID_ARG;
      for (int b = 0; b < NBINS - 1; ++b) {
        if (variant[b] < 0 || variant[b] >= NVARIANTS) return LPA_ERR_INVALID_ARG;
        v[b] = variant[b];
      }
    }
    if (std::memcmp(v, g->variant, sizeof(v)) != 0) {
      std::memcpy(g->variant, v, sizeof(v));
      drop_graphs(g);
    }
    return LPA_OK;
  });
}

int lpa_autotune(lpa_graph *g, double tolerance, int max_iters, int mode, int32_t *variant_out, double *bin_ms_out,
                 int32_t *schedule_out, int32_t *bins_out) {
  if (!g || max_iters < 1 || max_iters > 1000 || (mode != LPA_MODE_ASYNC && mode != LPA_MODE_DETERMINISTIC))
    return LPA_ERR_INVALID_ARG;
  int rc = LPA_OK;
  // Every candidate of every step must keep the modularity of its runs
  // within 0.002 of q_ref: the asynchronous processing order (schedule, bin
  // limits, kernel shapes) changes which labels a sweep sees.  In the
  // deterministic mode results do not depend on these settings.
  double q_ref = 0.0;
  bool have_ref = false;
  auto quality_ok = [&](double q) { return !have_ref || q >= q_ref - 0.002; };
  // the reference runs: default bins, hubs first, labels read as the schedule delivers them
  rc = lpa_set_first_sweep(g, 0);
  if (rc == LPA_OK) rc = lpa_set_bins(g, nullptr, 0);
  if (rc == LPA_OK && mode == LPA_MODE_ASYNC) rc = lpa_set_bin_order(g, 0);
  if (rc != LPA_OK) return rc;
  // 1. Asynchronous schedule: the fastest candidate whose runs converge (for
  //    a batch: every graph) and whose modularity stays within 0.002 of the
  //    all-16-step schedule's.
  if (mode == LPA_MODE_ASYNC) {
    static const int32_t cand[][3] = {{16, 0, 16}, {16, 1, 4}, {16, 2, 4}, {16, 2, 8},
                                      {16, 3, 4},  {16, 3, 8}, {1, 0, 1}};
    double best_ms = 1e300;
    int best = 0;
    for (int c = 0; c < (int)(sizeof(cand) / sizeof(cand[0])); ++c) {
      rc = lpa_set_async_schedule(g, cand[c][0], cand[c][1], cand[c][2], g->async_by_colour ? 1 : 0);
      if (rc != LPA_OK) return rc;
      double ms = 1e300, q = 0.0;
      bool converged = true;
      for (int rep = 0; rep < 2; ++rep) {
        lpa_stats st;
        rc = lpa_run(g, tolerance, max_iters, mode, 1, 0, nullptr, nullptr, nullptr, &st);
        if (rc != LPA_OK) return rc;
        ms = std::min(ms, st.total_ms);
        converged = converged && st.converged;
      }
      rc = lpa_modularity(g, nullptr, 0, &q);
      if (rc != LPA_OK) return rc;
      if (c == 0) {
        q_ref = q;
        have_ref = true;
      }
      // a candidate must be clearly faster (3 %) to displace an earlier one
      if (converged && quality_ok(q) && ms < 0.97 * best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    rc = lpa_set_async_schedule(g, cand[best][0], cand[best][1], cand[best][2], g->async_by_colour ? 1 : 0);
    if (rc != LPA_OK) return rc;
    if (schedule_out) std::memcpy(schedule_out, cand[best], sizeof(cand[best]));
  } else if (schedule_out) {
    schedule_out[0] = g->sched[0].nphase;
    schedule_out[1] = g->early_sweeps;
    schedule_out[2] = g->sched[1].nphase;
  }
  // 2. Degree limits of the bins.  A bin's LDS table has a fixed size, so its
  //    limit sets how full the table can get: the candidates fill the tables
  //    to at most 1/2 (the default), 1/4, 3/4 or all of their slots.  A lower
  //    limit gives the bin's rows sparser tables (shorter probe chains) and
  //    sends more rows to the next, wider bin.  In the asynchronous mode the
  //    limits also set which vertices a kernel processes together, and so
  //    which labels they see; they are tuned together with the order of the
  //    bins inside a step - hubs first (the default) or last, after the other
  //    vertices have updated their labels (fewer distinct labels reach the
  //    hubs' partitions) - and, where the rows allow it, the snapshot first
  //    sweep (lpa_set_first_sweep: the first 1, 3 or all kernels of each step
  //    of the first sweep read the initial labels; cheap to read, but a sweep
  //    whose vertices all read them merges fewer labels, which can cost a
  //    sweep later on; 2 and 4 kernels are then tried around the best).  Every
  //    combination is timed in this order under the same acceptance rules.
  {
    static const int32_t lim_cand[][NBINS - 1] = {{4, 16, 64, 256, 1024, 4096},
                                                  {2, 8, 32, 128, 512, 2048},
                                                  {6, 24, 96, 384, 1536, 6144},
                                                  {7, 31, 127, 511, 2047, 8191}};
    const bool async = mode == LPA_MODE_ASYNC;
    static const int32_t snap_cand[] = {0, 1, 3, NBINS};
    const int n_snap = async && g->rows_strict ? (int)(sizeof(snap_cand) / sizeof(snap_cand[0])) : 1;
    const int n_order = async && g->n_hubs > 0 ? 2 : 1;
    double best_ms = 1e300;
    int best = 0, best_order = 0, best_snap = 0;
    // one configuration: converged (every graph of a batch) and within the
    // quality bar in the asynchronous mode; its faster run of two
    auto trial_lim = [&](const int32_t *lim, bool baseline, int order, int snap, double &ms) -> int {
      int r = lpa_set_bins(g, lim, NBINS - 1);
      if (r == LPA_OK && async) r = lpa_set_bin_order(g, order);
      if (r == LPA_OK && async) r = lpa_set_first_sweep(g, snap);
      if (r != LPA_OK) return r;
      ms = 1e300;
      bool converged = true;
      for (int rep = 0; rep < 2; ++rep) {
        lpa_stats st;
        r = lpa_run(g, tolerance, max_iters, mode, 1, 0, nullptr, nullptr, nullptr, &st);
        if (r != LPA_OK) return r;
        ms = std::min(ms, st.total_ms);
        converged = converged && st.converged;
      }
      double q = 0.0;
      if (async) {
        r = lpa_modularity(g, nullptr, 0, &q);
        if (r != LPA_OK) return r;
      }
      if (!(baseline || (converged && (!async || quality_ok(q))))) ms = 1e300;
      return LPA_OK;
    };
    auto trial = [&](int c, int order, int snap, double &ms) -> int {
      return trial_lim(lim_cand[c], c == 0 && order == 0 && snap == 0, order, snap, ms);
    };
    for (int c = 0; c < (int)(sizeof(lim_cand) / sizeof(lim_cand[0])); ++c)
      for (int order = 0; order < n_order; ++order)
        for (int k = 0; k < n_snap; ++k) {
          double ms = 0.0;
          rc = trial(c, order, snap_cand[k], ms);
          if (rc != LPA_OK) return rc;
          if (ms < 0.97 * best_ms) {
            best_ms = ms;
            best = c;
            best_order = order;
            best_snap = snap_cand[k];
          }
        }
    if (n_snap > 1)
      for (int32_t snap : {best_snap - 1, best_snap + 1}) {
        if (snap <= 0 || snap >= NBINS || snap == 1 || snap == 3) continue;  // 2 and 4 only
        double ms = 0.0;
        rc = trial(best, best_order, snap, ms);
        if (rc != LPA_OK) return rc;
        if (ms < 0.97 * best_ms) {
          best_ms = ms;
          best_snap = snap;
        }
      }
    // Then, in the asynchronous mode, each bin's limit on its own: the four
    // fill levels of its table with the other limits kept (limits stay
    // non-decreasing); a single bin moves less work, so 1.5 % faster suffices.
    int32_t lim[NBINS - 1];
    std::memcpy(lim, lim_cand[best], sizeof(lim));
    if (async)
      for (int b = 0; b < NBINS - 1; ++b)
        for (int c = 0; c < (int)(sizeof(lim_cand) / sizeof(lim_cand[0])); ++c) {
          int32_t cand[NBINS - 1];
          std::memcpy(cand, lim, sizeof(cand));
          cand[b] = lim_cand[c][b];
          if (cand[b] == lim[b] || (b > 0 && cand[b] < cand[b - 1]) || (b < NBINS - 2 && cand[b] > cand[b + 1]))
            continue;
          double ms = 0.0;
          rc = trial_lim(cand, false, best_order, best_snap, ms);
          if (rc != LPA_OK) return rc;
          if (ms < 0.985 * best_ms) {
            best_ms = ms;
            std::memcpy(lim, cand, sizeof(lim));
          }
        }
    rc = lpa_set_bins(g, lim, NBINS - 1);
    if (rc == LPA_OK && async) rc = lpa_set_bin_order(g, best_order);
    if (rc == LPA_OK && async) rc = lpa_set_first_sweep(g, best_snap);
    if (rc != LPA_OK) return rc;
    if (bins_out) std::memcpy(bins_out, lim, sizeof(lim));
  }
  // 3. Kernel shapes: every bin is its own kernel, so one run per variant
  //    times all bins at once; each run is repeated and the faster kept.
  double best_ms[NBINS - 1];
  int32_t best_v[NBINS - 1];
  for (int b = 0; b < NBINS - 1; ++b) {
    best_ms[b] = 1e300;
    best_v[b] = 0;
  }
  for (int v = 0; v < NVARIANTS; ++v) {
    int32_t all[NBINS - 1];
    for (int b = 0; b < NBINS - 1; ++b) all[b] = v;
    rc = lpa_set_variants(g, all, NBINS - 1);
    if (rc != LPA_OK) return rc;
    for (int rep = 0; rep < 2; ++rep) {
      lpa_stats st;
      rc = lpa_run(g, tolerance, max_iters, mode, 1, LPA_FLAG_KERNEL_TIMING, nullptr, nullptr, nullptr, &st);
      if (rc != LPA_OK) return rc;
      for (int b = 0; b < NBINS - 1; ++b) {
        if (!st.kernel_launches[TK_BIN0 + b]) continue;
        // the first variant timed sets the bar; later ones must beat it by 3 % (and the
        // repeat of the same variant by anything)
        const double bar = best_v[b] == v ? best_ms[b] : 0.97 * best_ms[b];
        if (st.kernel_ms[TK_BIN0 + b] < bar) {
          best_ms[b] = st.kernel_ms[TK_BIN0 + b];
          best_v[b] = v;
        }
      }
    }
  }
  rc = lpa_set_variants(g, best_v, NBINS - 1);
  if (rc != LPA_OK) return rc;
  if (mode == LPA_MODE_ASYNC) {
    // the mix of per-bin picks must converge and keep the quality; else every
    // bin goes back to its default shape
    bool converged = true;
    for (int rep = 0; rep < 2; ++rep) {
      lpa_stats st;
      rc = lpa_run(g, tolerance, max_iters, mode, 1, 0, nullptr, nullptr, nullptr, &st);
      if (rc != LPA_OK) return rc;
      converged = converged && st.converged;
    }
    double q = 0.0;
    rc = lpa_modularity(g, nullptr, 0, &q);
    if (rc != LPA_OK) return rc;
    if (!converged || !quality_ok(q)) {
      for (int b = 0; b < NBINS - 1; ++b) best_v[b] = 0;
      rc = lpa_set_variants(g, best_v, NBINS - 1);
      if (rc != LPA_OK) return rc;
    }
  }
  if (variant_out) std::memcpy(variant_out, best_v, sizeof(best_v));
  if (bin_ms_out)
    for (int b = 0; b < NBINS - 1; ++b) bin_ms_out[b] = best_ms[b] < 1e299 ? best_ms[b] : 0.0;
  return LPA_OK;
}

int lpa_set_async_schedule(lpa_graph *g, int32_t early_phases, int32_t early_sweeps, int32_t late_phases,
                           int32_t by_colour) {
  return run_guarded(g, [&]() -> int {
    if (early_phases < 1 || early_phases > 1024 || late_phases < 1 || late_phases > 1024 || early_sweeps < 0 ||
        early_sweeps > 1000)
      return LPA_ERR_INVALID_ARG;
    if (early_phases != g->sched[0].nphase || late_phases != g->sched[1].nphase ||
        (by_colour != 0) != g->async_by_colour) {
      g->sched[0].nphase = early_phases;
      g->sched[1].nphase = late_phases;
      g->async_by_colour = by_colour != 0;
      g->lists_ready = false;
      g->dlists_ready = false;
    }
    g->early_sweeps = early_sweeps;
    drop_graphs(g);
    return LPA_OK;
  });
}

int lpa_set_async_phases(lpa_graph *g, int32_t phases, int32_t by_colour) {
  return lpa_set_async_schedule(g, phases, 0, phases, by_colour);
}

int lpa_set_bin_order(lpa_graph *g, int32_t hubs_last) {
  return run_guarded(g, [&]() -> int {
    if (hubs_last != 0 && hubs_last != 1) return LPA_ERR_INVALID_ARG;
    if ((hubs_last != 0) != g->hubs_last) {
      g->hubs_last = hubs_last != 0;
      drop_graphs(g);
    }
    return LPA_OK;
  });
}

int lpa_set_first_sweep(lpa_graph *g, int32_t kernels) {
  return run_guarded(g, [&]() -> int {
    if (kernels < 0 || kernels > NBINS) return LPA_ERR_INVALID_ARG;
    g->snapshot_kernels = kernels;
    return LPA_OK;
  });
}

int lpa_get_schedule(const lpa_graph *gc, int32_t *out) {
  if (!gc || !out) return LPA_ERR_INVALID_ARG;
  out[0] = gc->sched[0].nphase;
  out[1] = gc->early_sweeps;
  out[2] = gc->sched[1].nphase;
  out[3] = gc->async_by_colour ? 1 : 0;
  out[4] = gc->hubs_last ? 1 : 0;
  out[5] = gc->snapshot_kernels;
  out[6] = gc->rows_strict ? 1 : 0;
  return LPA_OK;
}

int lpa_color(lpa_graph *g, uint32_t seed, int32_t *colors_out, unsigned flags, int32_t *num_colors) {
  return run_guarded(g, [&]() -> int {
    ensure_colored(g, seed);
    if (colors_out && g->n) {
      vertex_out<int32_t>(g, colors_out, g->color, flags);
      HIP_OK(hipStreamSynchronize(g->stream));
    }
    if (num_colors) *num_colors = g->ncol;
    return LPA_OK;
  });
}

int lpa_run(lpa_graph *g, double tolerance, int max_iters, int mode, int prune, unsigned flags,
            const int32_t *init_labels, const uint8_t *init_flags, int32_t *labels_out, lpa_stats *stats) {
  if (!g || max_iters < 0 || max_iters > 1000 || (mode != LPA_MODE_ASYNC && mode != LPA_MODE_DETERMINISTIC) ||
      !(tolerance == tolerance))
    return LPA_ERR_INVALID_ARG;
  if ((flags & LPA_FLAG_GATE) && !g->gate_loaded) return LPA_ERR_NO_GATE;
  return run_guarded(g, [&]() -> int {
    Events ev;
    hipEvent_t e0 = ev.e[0], e1 = ev.e[1], t0 = ev.e[2], t1 = ev.e[3];
    hipEvent_t lag[2] = {ev.e[4], ev.e[5]};
    const bool timing = flags & LPA_FLAG_KERNEL_TIMING;
    const bool use_graph = !(flags & (LPA_FLAG_NO_GRAPH | LPA_FLAG_KERNEL_TIMING));
    HIP_OK(hipEventRecord(e0, g->stream));
    // one-off setup of the schedule
    ensure_lists(g);
    if (mode == LPA_MODE_DETERMINISTIC) {
      ensure_colored(g, g->colored ? g->color_seed : 0u);
      ensure_dlists(g);
    }
    if (init_labels && g->n) {
      // labels must be vertex ids
      vertex_in<int32_t>(g, g->C, init_labels, flags);
      int32_t *bad = (int32_t *)((char *)g->scratch_small + 2048);
      HIP_OK(hipMemsetAsync(bad, 0, sizeof(int32_t), g->stream));
      launch_check_labels(g->C, g->n, bad, g->stream);
      int32_t hb = 0;
      HIP_OK(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
      HIP_OK(hipStreamSynchronize(g->stream));
      if (hb) return LPA_ERR_INVALID_ARG;
    }
    if (init_flags && g->n) vertex_in<uint8_t>(g, g->F, init_flags, flags);
    if (g->n)
      launch_init_state(g->off, g->C, g->F, g->n, init_labels ? 0 : 1, init_flags ? 0 : 1, max_iters > 0 ? 1 : 0,
                        g->orig,
                        g->stream);
    // A batched handle replays the whole run as one graph launch; otherwise
    // one sweep per launch, with the stop test polled one sweep behind.
    // (a single graph's run that ends with a verification sweep needs the
    // host between sweeps; a batch verifies every graph on the device, with
    // room for each graph's verification and fallback sweeps)
    const bool checked = flags & (LPA_FLAG_GATE | LPA_FLAG_VERIFY | LPA_FLAG_VERIFY_FULL);
    const int batch_mode = g->ngraphs && checked && max_iters > 0 ? ((flags & LPA_FLAG_VERIFY_FULL) ? 2 : 1) : 0;
    const int run_sweeps = batch_mode ? 2 * max_iters + 2 : max_iters;
    const bool one_launch = use_graph && (g->ngraphs > 0 || ((flags & LPA_FLAG_ONE_LAUNCH) && !checked));
    // gate features: written while the gate is used or training traces are recorded
    const bool gate = flags & LPA_FLAG_GATE;
    const bool trace = flags & LPA_FLAG_TRACE;
    g->nonstrict = flags & LPA_FLAG_NONSTRICT;
    g->feat_on = gate || trace;
    g->gate_active = gate;
    if (gate && !g->gskip) g->gskip = dalloc_n<uint8_t>(g, g->n);
    if (g->feat_on) {
      if (!g->feat) {
        g->feat = dalloc_n<float>(g, g->n * FEAT_STRIDE);
      }
      launch_feat_reset(g->feat, g->n, g->stream);
    }
    g->cur_feat = feat_args(g, max_iters, trace);
    // snapshot first sweep: asynchronous runs from the initial labels over
    // rows without repeated neighbours
    const int snap = mode == LPA_MODE_ASYNC && g->rows_strict && !init_labels ? g->snapshot_kernels : 0;
    // per-sweep graphs of the early and the late asynchronous schedule
    hipGraphExec_t exec = nullptr, exec_late = nullptr, exec_first = nullptr;
    if (use_graph && max_iters > 0) {
      exec = sweep_graph(g, mode, prune, one_launch ? run_sweeps : 1, 0, 0, one_launch ? snap : 0);
      exec_late = one_launch ? exec : sweep_graph(g, mode, prune, 1, g->early_sweeps);
      if (snap && !one_launch) exec_first = sweep_graph(g, mode, prune, 1, 0, 0, snap);
    }
    auto launch_sweep = [&](int s) {
      const int late = s >= g->early_sweeps;
      const bool first = snap && s == 0;
      if (exec) HIP_OK(hipGraphLaunch(first ? exec_first : late ? exec_late : exec, g->stream));
      else emit_sweep(g, g->stream, mode, prune, late ? 1 : 0, first ? snap : 0);
    };
    HIP_OK(hipEventRecord(e1, g->stream));
    HIP_OK(hipEventSynchronize(e1));
    float setup_ms = 0;
    HIP_OK(hipEventElapsedTime(&setup_ms, e0, e1));
    // the run
    g->timing = timing;
    g->ev_used = 0;
    HIP_OK(hipEventRecord(t0, g->stream));
    const int nfc = mode == LPA_MODE_DETERMINISTIC ? std::max(1, g->ncol) * NBINS : max_phases(g) * NBINS;
    const int dense = mode == LPA_MODE_ASYNC && prune && !(flags & LPA_FLAG_EXACT_MARKS);
    launch_run_begin(g->ctl, tolerance, run_sweeps, g->n, g->n_active, g->fcount, nfc, g->host_done_dev, dense,
                     !init_labels && !init_flags, gate ? 1 : 0, g->stream);
    if (g->ngraphs) launch_batch_begin(g->ctl, batch_args(g), g->n, g->nlive, batch_mode, max_iters, g->stream);
    // The stop test is read one sweep behind, so that the next sweep is queued
    // while the host waits; a deterministic sweep (thousands of colour-step
    // kernels) is long enough to wait for before queueing the next one, which
    // saves the sweep that would only find the run done.
    const int behind = mode == LPA_MODE_DETERMINISTIC ? 0 : 1;
    if (one_launch && exec) {
      HIP_OK(hipGraphLaunch(exec, g->stream));
    } else
    for (int s = 0; s < run_sweeps; ++s) {
      launch_sweep(s);
      HIP_OK(hipEventRecord(lag[s & 1], g->stream));
      if (s >= behind) {
        HIP_OK(hipEventSynchronize(lag[(s - behind) & 1]));
        if (__atomic_load_n(g->host_done, __ATOMIC_ACQUIRE)) break;
      }
    }
    // Verification: one full sweep after convergence; if it changes more than
    // tau * n labels the run goes on with plain pruning (gate off), then
    // verifies once more.
    auto sweep_loop = [&](int budget) {
      for (int s = 0; s < budget; ++s) {
        launch_sweep(max_iters + s);  // sweeps after a verification run in the late schedule
        HIP_OK(hipEventRecord(lag[s & 1], g->stream));
        if (s >= behind) {
          HIP_OK(hipEventSynchronize(lag[(s - behind) & 1]));
          if (__atomic_load_n(g->host_done, __ATOMIC_ACQUIRE)) break;
        }
      }
    };
    int verified = -1;
    if (checked && max_iters > 0 && !g->ngraphs) {
      // with the gate off no feature is read again: verification and any
      // fallback sweeps run the plain kernels (the plain late-sweep graph)
      g->feat_on = false;
      g->gate_active = false;
      hipGraphExec_t exec_verify = nullptr;
      if (use_graph) {
        exec_late = sweep_graph(g, mode, prune, 1, g->early_sweeps);
        exec_verify = sweep_graph(g, mode, prune, 1, g->early_sweeps, 1);
      }
      for (int attempt = 0; attempt < 2; ++attempt) {
        launch_set_phase(g->ctl, (flags & LPA_FLAG_VERIFY_FULL) ? 2 : 1, 0, 0, g->host_done_dev, g->stream);
        if (exec_verify) HIP_OK(hipGraphLaunch(exec_verify, g->stream));
        else emit_sweep(g, g->stream, mode, prune, 2);
        int32_t vflag = 0;
        HIP_OK(hipMemcpyAsync(&vflag, &g->ctl->verified, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
        HIP_OK(hipStreamSynchronize(g->stream));
        verified = vflag;
        if (vflag || attempt == 1) break;
        launch_set_phase(g->ctl, 0, 0, max_iters, g->host_done_dev, g->stream);
        sweep_loop(max_iters);
      }
    }
    HIP_OK(hipEventRecord(t1, g->stream));
    HIP_OK(hipStreamSynchronize(g->stream));
    g->timing = false;
    g->feat_on = false;
    g->gate_active = false;
    Ctl h;
    HIP_OK(hipMemcpy(&h, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    float run_ms = 0;
    HIP_OK(hipEventElapsedTime(&run_ms, t0, t1));
    g->has_labels = true;
    if (labels_out && g->n) {
      vertex_out<int32_t>(g, labels_out, g->C, flags);
      HIP_OK(hipStreamSynchronize(g->stream));
    }
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->iterations = h.iterations;
      stats->converged = h.converged;
      stats->verified = batch_mode ? h.batch_remaining == 0 && h.batch_unverified == 0 : verified > 0;
      stats->num_colors = mode == LPA_MODE_DETERMINISTIC ? g->ncol : 0;
      u64 prev = h.t_start;
      for (int s = 0; s < std::min(h.iterations, MAX_REC); ++s) {
        stats->changed[s] = (int64_t)h.st_changed[s];
        stats->frontier[s] = (int64_t)h.st_processed[s];
        stats->edges_scanned[s] = (int64_t)h.st_scanned[s];
        stats->gated_out[s] = (int64_t)h.st_gated[s];
        stats->ms[s] = (float)((double)(h.t_sweep[s] - prev) / (double)g->wall_khz);
        prev = h.t_sweep[s];
      }
      stats->total_changed = (int64_t)h.total_changed;
      stats->verify_changed = (int64_t)h.verify_changed;
      stats->verify_edges_scanned = (int64_t)h.verify_scanned;
      stats->total_ms = run_ms;
      stats->setup_ms = setup_ms;
      for (int b = 0; b < NBINS; ++b) {
        stats->bin_vertices[b] = (int64_t)h.bin_vertices[b];
        stats->bin_edges[b] = (int64_t)h.bin_edges[b];
        stats->bin_changed[b] = (int64_t)h.bin_changed[b];
        stats->bin_marks[b] = (int64_t)h.bin_marks[b];
      }
      stats->compact_listed = (int64_t)h.compact_listed;
      stats->compact_taken = (int64_t)h.compact_taken;
      stats->first_vertices = (int64_t)h.first_vertices;
      stats->first_edges = (int64_t)h.first_edges;
      stats->first_changed = (int64_t)h.first_changed;
      stats->first_marks = (int64_t)h.first_marks;
      stats->first_reads = (int64_t)h.first_reads;
      stats->weight_bytes = g->wk == W_UNIT ? 0 : (g->wk == W_U8 ? 1 : 4);
      if (timing) {
        for (size_t k = 0; k < g->ev_used; ++k) {
          float ms = 0;
          HIP_OK(hipEventElapsedTime(&ms, g->ev_pool[k].first, g->ev_pool[k].second));
          stats->kernel_ms[g->ev_kind[k]] += ms;
          stats->kernel_launches[g->ev_kind[k]] += 1;
        }
      }
    }
    if (h.error) {
      // leave the hub partitions empty for the next run
      if (g->hub_parts_total)
        HIP_OK(hipMemsetAsync(g->hub_pcnt, 0, sizeof(int32_t) * g->hub_parts_total, g->stream));
      HIP_OK(hipStreamSynchronize(g->stream));
      return LPA_ERR_INTERNAL;
    }
    return LPA_OK;
  });
}

int lpa_get_flags(const lpa_graph *gc, uint8_t *flags_out, unsigned flags) {
  lpa_graph *g = const_cast<lpa_graph *>(gc);
  return run_guarded(g, [&]() -> int {
    if (!flags_out) return LPA_ERR_INVALID_ARG;
    if (g->n) {
      vertex_out<uint8_t>(g, flags_out, g->F, flags);
      HIP_OK(hipStreamSynchronize(g->stream));
    }
    return LPA_OK;
  });
}

int lpa_modularity(const lpa_graph *gc, const int32_t *labels, unsigned flags, double *q_out) {
  lpa_graph *g = const_cast<lpa_graph *>(gc);
  return run_guarded(g, [&]() -> int {
    if (!q_out) return LPA_ERR_INVALID_ARG;
    if (g->n == 0 || g->m == 0) {
      *q_out = 0.0;
      return LPA_OK;
    }
    const int32_t *C = g->C;
    int32_t *tmp = nullptr;
    if (labels) {
      if ((flags & LPA_FLAG_DEVICE_PTRS) && !g->orig) C = labels;
      else {
        tmp = dalloc_n<int32_t>(g, g->n);
        vertex_in<int32_t>(g, tmp, labels, flags);
        C = tmp;
      }
    }
    char *sm = (char *)g->scratch_small;
    int32_t *bad = (int32_t *)(sm + 2048);
    ModAcc *acc = (ModAcc *)(sm + 2112);
    HIP_OK(hipMemsetAsync(bad, 0, sizeof(int32_t), g->stream));
    HIP_OK(hipMemsetAsync(acc, 0, sizeof(ModAcc), g->stream));
    launch_check_labels(C, g->n, bad, g->stream);
    u64 *tot = dalloc_n<u64>(g, g->n);
    const int nb = mod_square_blocks();
    u64 *part = dalloc_n<u64>(g, 2 * nb);
    HIP_OK(hipMemsetAsync(tot, 0, sizeof(u64) * g->n, g->stream));
    int32_t hb = 0;
    HIP_OK(hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipStreamSynchronize(g->stream));
    if (hb) {
      dfree(g, tot);
      dfree(g, part);
      dfree(g, tmp);
      return LPA_ERR_INVALID_ARG;
    }
    launch_mod_community_totals(C, g->K, g->n, tot, g->stream);
    launch_mod_inside(g->off, g->idx, g->w, g->wk, C, g->n, g->m, acc, g->stream);
    launch_mod_squares(tot, g->n, part, g->stream);
    ModAcc ha{};
    std::vector<u64> hp(2 * nb);
    HIP_OK(hipMemcpyAsync(&ha, acc, sizeof(ha), hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipMemcpyAsync(hp.data(), part, sizeof(u64) * 2 * nb, hipMemcpyDeviceToHost, g->stream));
    HIP_OK(hipStreamSynchronize(g->stream));
    dfree(g, tot);
    dfree(g, part);
    dfree(g, tmp);
    unsigned __int128 s2 = 0;
    for (int k = 0; k < nb; ++k) s2 += ((unsigned __int128)hp[2 * k + 1] << 64) | hp[2 * k];
    const unsigned __int128 two_m = ha.two_m;
    if (two_m == 0) {
      *q_out = 0.0;
      return LPA_OK;
    }
    const __int128 num = (__int128)((unsigned __int128)ha.s1 * two_m) - (__int128)s2;
    const unsigned __int128 den = two_m * two_m;
    *q_out = (double)num / (double)den;
    return LPA_OK;
  });
}

}  // extern "C"
