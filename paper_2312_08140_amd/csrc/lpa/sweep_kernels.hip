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
#include "tables.hpp"

namespace gvelpa {

// ---------------------------------------------------------------- run control

// Labels and flags before the first sweep.  A vertex without stored entries
// is processed in sweep 0 like any other (its flag is cleared, its label
// kept) and nothing can mark it again, so its flag is cleared here once a run
// has at least one sweep; such vertices are not in the work lists.
// Labels start as vertex ids (the id stored at position v: orig[v], or v).
__global__ void k_init_state(const int64_t *off, int32_t *C, uint8_t *F, int64_t n, int set_labels, int set_flags,
                             int clear_isolated, const int32_t *orig) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (set_labels) C[v] = orig ? orig[v] : (int32_t)v;
    if (set_flags) F[v] = 1;
    if (clear_isolated && off[v + 1] == off[v]) F[v] = 0;
  }
}

__global__ void k_run_begin(Ctl *ctl, double tau, int max_iters, int64_t n, int64_t n_active, int32_t *fcount,
                            int nfc, int32_t *host_done, int dense_enabled, int dense_first, int gate_on) {
  for (int k = threadIdx.x; k < nfc; k += blockDim.x) fcount[k] = 0;
  for (int k = threadIdx.x; k < NSHARD * NSLOT * 4; k += blockDim.x) ctl->shard[k / (NSLOT * 4)][(k >> 2) % NSLOT].c[k & 3] = 0;
  if (threadIdx.x == 0) {
    ctl->dense_enabled = dense_enabled;
    ctl->dense_cur = dense_enabled && dense_first;
    ctl->dense_prev = 0;
    ctl->dense_frac = 0.5;
    ctl->n_active = n_active;
    ctl->batch = 0;
    ctl->gate_on = gate_on;
    ctl->verified = 0;
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
    ctl->hub_chunks = ctl->hub_groups = 0;
    ctl->verify_changed = ctl->total_changed = ctl->verify_scanned = 0;
    for (int k = 0; k < MAX_REC; ++k)
      ctl->st_changed[k] = ctl->st_processed[k] = ctl->st_scanned[k] = ctl->st_gated[k] = ctl->t_sweep[k] = 0;
    for (int k = 0; k < NBINS; ++k)
      ctl->bin_vertices[k] = ctl->bin_edges[k] = ctl->bin_changed[k] = ctl->bin_marks[k] = 0;
    ctl->compact_listed = ctl->compact_taken = 0;
    ctl->first_vertices = ctl->first_edges = ctl->first_changed = ctl->first_marks = ctl->first_reads = 0;
    ctl->t_start = wall_clock64();
    if (host_done) {
      __atomic_store_n(host_done, ctl->done, __ATOMIC_RELAXED);
      __threadfence_system();
    }
  }
}

// Folds the sweep's counter shards into the sweep totals (ctl->changed,
// processed, scanned, gated) and the run totals per bin, clearing them.
__device__ void fold_shards(Ctl *ctl) {
  __shared__ u64 red[NSLOT][4];
  for (int k = threadIdx.x; k < NSLOT * 4; k += blockDim.x) red[k >> 2][k & 3] = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < NSHARD * NSLOT * 4; k += blockDim.x) {
    const int q = k & 3, slot = (k >> 2) % NSLOT, sh = k / (NSLOT * 4);
    const u64 x = ctl->shard[sh][slot].c[q];
    if (x) {
      atomicAdd(&red[slot][q], x);
      ctl->shard[sh][slot].c[q] = 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 changed = 0, scanned = 0;
    for (int b = 0; b < NBINS; ++b) {
      changed += red[b][0];
      scanned += red[b][1];
      ctl->bin_changed[b] += red[b][0];
      ctl->bin_edges[b] += red[b][1];
      ctl->bin_vertices[b] += red[b][2];
      ctl->bin_marks[b] += red[b][3];
    }
    changed += red[FIRST_SLOT][0];
    scanned += red[FIRST_SLOT][1];
    ctl->first_changed += red[FIRST_SLOT][0];
    ctl->first_edges += red[FIRST_SLOT][1];
    ctl->first_vertices += red[FIRST_SLOT][2];
    ctl->first_marks += red[FIRST_SLOT][3];
    ctl->first_reads += red[READS_SLOT][0];
    ctl->changed = changed;
    ctl->scanned = scanned;
    ctl->processed = red[NBINS][0];
    ctl->gated = red[NBINS][1];
    ctl->compact_taken += red[NBINS][0];
    ctl->compact_listed += red[NBINS][2];
  }
}

__global__ void k_end_sweep(Ctl *ctl, int32_t *fcount, int nfc, int32_t *host_done) {
  if (__atomic_load_n(&ctl->done, __ATOMIC_RELAXED)) return;
  for (int k = threadIdx.x; k < nfc; k += blockDim.x) fcount[k] = 0;
  fold_shards(ctl);
  if (threadIdx.x != 0) return;
  const int s = ctl->sweep;
  const u64 dn = ctl->changed;
  if (ctl->verify_phase) {
    // a verification sweep: one full sweep, judged by the same stop test
    ctl->verify_changed += dn;
    ctl->verify_scanned += ctl->scanned;
    ctl->total_changed += dn;
    ctl->verified = (double)dn / (double)(ctl->n > 0 ? ctl->n : 1) <= ctl->tau;
    ctl->sweep = s + 1;
    ctl->dense_prev = ctl->dense_cur;
    ctl->dense_cur = ctl->dense_enabled && (double)dn > ctl->dense_frac * (double)ctl->n_active;
    ctl->changed = ctl->processed = ctl->scanned = ctl->gated = 0;
    ctl->done = 1;
    if (host_done) {
      __atomic_store_n(host_done, 1, __ATOMIC_RELAXED);
      __threadfence_system();
    }
    return;
  }
  const int it = ctl->iterations;  // sweeps of the method so far (verification sweeps excluded)
  if (it < MAX_REC) {
    ctl->st_changed[it] = dn;
    ctl->st_processed[it] = ctl->processed;
    ctl->st_scanned[it] = ctl->scanned;
    ctl->st_gated[it] = ctl->gated;
    ctl->t_sweep[it] = wall_clock64();
  }
  ctl->total_changed += dn;
  ctl->dense_prev = ctl->dense_cur;
  // A gated sweep writes exact marks: its flags, with those the gate kept,
  // are all the verification sweep has to process (a dense sweep would flag
  // every vertex and turn the verification into a full sweep).
  // (likewise in a verified batch, where some graph may be verifying)
  ctl->dense_cur = ctl->dense_enabled && !ctl->gate_on && !(ctl->batch && ctl->batch_mode) &&
                   (double)dn > ctl->dense_frac * (double)ctl->n_active;
  ctl->iterations = it + 1;
  ctl->sweep = s + 1;
  if (ctl->batch) {
    // every graph has its own stop test (k_batch_end); the run ends with the last
    if (ctl->batch_remaining == 0 || s + 1 >= ctl->max_iters) {
      ctl->done = 1;
      ctl->converged = ctl->batch_remaining == 0 && ctl->batch_capped == 0;
    }
  } else {
    // Algorithm 1: stop when dN / N <= tau (evaluated in double).
    const bool conv = (double)dn / (double)(ctl->n > 0 ? ctl->n : 1) <= ctl->tau;
    if (conv) ctl->converged = 1;
    if (conv || s + 1 >= ctl->max_iters) ctl->done = 1;
  }
  ctl->changed = ctl->processed = ctl->scanned = ctl->gated = 0;
  if (host_done) {
    __atomic_store_n(host_done, ctl->done, __ATOMIC_RELAXED);
    __threadfence_system();
  }
}

// After a dense sweep every vertex with a stored entry is flagged.
__global__ void k_dense_fill(const Ctl *ctl, const int64_t *off, uint8_t *F, int64_t n) {
  if (!__atomic_load_n(&ctl->dense_prev, __ATOMIC_RELAXED)) return;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (off[v + 1] > off[v]) F[v] = 1;
}

// ---------------------------------------------------------------- batched runs

__global__ void k_batch_gid(BatchArgs b) {
  for (int g = blockIdx.x; g < b.ngraphs; g += gridDim.x)
    for (int64_t v = b.vptr[g] + threadIdx.x; v < b.vptr[g + 1]; v += blockDim.x) b.gid[v] = g;
}

__global__ void k_batch_begin(Ctl *ctl, BatchArgs b, int64_t n, int32_t live, int mode, int iters) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    b.chg[v] = 0;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < b.ngraphs; g += gridDim.x * blockDim.x) {
    const bool empty = b.vptr[g + 1] == b.vptr[g];  // an empty graph has nothing to do
    b.gdone[g] = empty;
    b.giters[g] = 0;
    b.gconv[g] = empty;
    b.gphase[g] = empty ? BPH_DONE : BPH_MAIN;
    b.gcap[g] = iters;
    b.gverified[g] = empty;
    b.gvchanged[g] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->batch = 1;
    ctl->batch_remaining = live;
    ctl->batch_capped = 0;
    ctl->batch_mode = mode;
    ctl->batch_iters = iters;
    ctl->batch_unverified = 0;
  }
}

// Per-graph stop test of the sweep just finished (Algorithm 1 applied to
// every graph separately): dN_g counts the graph's changed vertices.  In a
// verified run every graph then goes through its own verification sweep
// (gate off) and, if that changes more than tau * N_g labels, through plain
// sweeps (at least one, at most `iters`, ending once the graph's sweeps,
// verification included, reach 2 * iters) and a last verification sweep.
// The batch therefore needs at most 2 * iters + 2 sweeps.  Sweep counts of a graph equal
// the batch's, as every graph starts at sweep 0 and takes part in each sweep
// until it is done.
__global__ __launch_bounds__(256) void k_batch_end(Ctl *ctl, BatchArgs b) {
  if (__atomic_load_n(&ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ int s_sum[4];
  __shared__ int s_flag_all;
  const int s = ctl->sweep;
  const int mode = ctl->batch_mode, iters = ctl->batch_iters;
  for (int g = blockIdx.x; g < b.ngraphs; g += gridDim.x) {
    const int64_t v0 = b.vptr[g], v1 = b.vptr[g + 1];
    int c = 0;
    for (int64_t v = v0 + threadIdx.x; v < v1; v += 256) {
      c += b.chg[v];
      b.chg[v] = 0;
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = c;
    if (threadIdx.x == 0) s_flag_all = 0;
    __syncthreads();
    if (threadIdx.x == 0 && !b.gdone[g]) {
      const int64_t dn = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
      const bool small = (double)dn / (double)(v1 - v0) <= ctl->tau;
      const int ph = b.gphase[g];
      int next = ph;
      bool finish = false;
      if (ph == BPH_MAIN || ph == BPH_FALLBACK) {
        b.giters[g] += 1;
        if (small) b.gconv[g] = 1;
        if (small || s + 1 >= (ph == BPH_MAIN ? iters : b.gcap[g])) {
          if (mode == 0) finish = true;
          else next = ph + 1;
        }
      } else {
        b.gvchanged[g] += (int32_t)dn;
        atomicAdd((unsigned long long *)&ctl->verify_changed, (unsigned long long)dn);
        b.gverified[g] = small;
        if (small || ph == BPH_VERIFY2) {
          finish = true;
        } else {
          next = BPH_FALLBACK;
          b.gcap[g] = min(2 * iters, s + 1 + iters);
        }
      }
      if (finish) {
        b.gdone[g] = 1;
        b.gphase[g] = BPH_DONE;
        atomicSub(&ctl->batch_remaining, 1);
        if (!b.gconv[g]) atomicAdd(&ctl->batch_capped, 1);
        if (mode && !b.gverified[g]) atomicAdd(&ctl->batch_unverified, 1);
      } else {
        b.gphase[g] = next;
        // a full verification processes every vertex of the graph that has entries
        if (mode == 2 && next != ph && (next == BPH_VERIFY || next == BPH_VERIFY2)) s_flag_all = 1;
      }
    }
    __syncthreads();
    if (s_flag_all)
      for (int64_t v = v0 + threadIdx.x; v < v1; v += 256)
        if (b.off[v + 1] > b.off[v]) b.F[v] = 1;
    __syncthreads();
  }
}

void launch_batch_gid(const BatchArgs &b, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_gid, dim3(std::max(1, std::min(b.ngraphs, 8192))), dim3(256), 0, st, b);
}

void launch_batch_begin(Ctl *ctl, const BatchArgs &b, int64_t n, int32_t live, int mode, int iters,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_batch_begin, dim3(4096), dim3(256), 0, st, ctl, b, n, live, mode, iters);
}

void launch_batch_end(Ctl *ctl, const BatchArgs &b, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_end, dim3(std::max(1, std::min(b.ngraphs, 8192))), dim3(256), 0, st, ctl, b);
}

// ---------------------------------------------------------------- compaction

// Tiles of 256 * CU entries per block; flagged vertices get their slot in the
// bin's frontier from an LDS counter, then one global atomic per (tile, bin)
// reserves the tile's range.
constexpr int CU = 8;

// Logit of the gate network (parameters already in LDS as fp32 values of
// their bf16 rounding; W1[32][8], b1, W2[32][32], b2, W3[32], b3).
__device__ __forceinline__ float gate_logit(const float *P, const float *x) {
  const float *W1 = P, *b1 = P + 256, *W2 = P + 288, *b2 = P + 1312, *W3 = P + 1344;
  float h1[32];
#pragma unroll
  for (int o = 0; o < 32; ++o) {
    float acc = b1[o];
#pragma unroll
    for (int q = 0; q < NFEAT; ++q) acc = fmaf(W1[o * 8 + q], x[q], acc);
    h1[o] = acc > 0.0f ? acc : 0.0f;
  }
  float z = P[1376];
  for (int o = 0; o < 32; ++o) {
    float acc = b2[o];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc = fmaf(W2[o * 32 + q], h1[q], acc);
    z = fmaf(W3[o], acc > 0.0f ? acc : 0.0f, z);
  }
  return z;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Gate decisions of a sweep, taken once at its start for every vertex that is
// flagged then and has been processed before: skip[v] = 1 when the network's
// logit is below z (the vertex keeps its flag and waits).  Vertices flagged
// later in the sweep are not gated in it.
// The same network with its parameters (fp32 values of their bf16 rounding)
// read at wave-uniform addresses, so they arrive through scalar loads and
// feed the FMAs as scalar operands; same order of operations as gate_logit.
__device__ __forceinline__ float gate_logit_uniform(const float *__restrict__ P, const float *x) {
  float h1[32];
#pragma unroll
  for (int o = 0; o < 32; ++o) {
    float acc = P[256 + o];
#pragma unroll
    for (int q = 0; q < NFEAT; ++q) acc = fmaf(P[o * 8 + q], x[q], acc);
    h1[o] = acc > 0.0f ? acc : 0.0f;
  }
  float z = P[1376];
#pragma unroll 2
  for (int o = 0; o < 32; ++o) {
    float acc = P[1312 + o];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc = fmaf(P[288 + o * 32 + q], h1[q], acc);
    z = fmaf(P[1344 + o], acc > 0.0f ? acc : 0.0f, z);
  }
  return z;
}

__global__ __launch_bounds__(256) void k_gate_pass(const Ctl *ctl, const float *__restrict__ gate, float z, FeatArgs f,
                                                   const uint8_t *F, uint8_t *skip, int64_t n,
                                                   const int32_t *gid, const int32_t *gphase) {
  if (__atomic_load_n(&ctl->done, __ATOMIC_RELAXED)) return;
  const int sweep = ctl->sweep;
  if (!ctl->gate_on || ctl->verify_phase || sweep < 1) return;
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v - threadIdx.x < n; v += (int64_t)gridDim.x * 256) {
    const float *rec = f.feat + v * FEAT_STRIDE;
    // a batched graph past its gated sweeps (verifying, falling back, done) is not gated
    const bool in_gate = v < n && F[v] && (!gphase || gphase[gid[v]] == BPH_MAIN);
    const int lp = in_gate ? record_lastp(rec) : -1;
    float x[NFEAT] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (lp >= 0) decision_features(rec, lp, sweep, f.max_iters, x);
    float logit = 0.0f;
    if (__ballot(lp >= 0)) logit = gate_logit_uniform(gate, x);  // whole waves skip the network
    if (v < n) skip[v] = lp >= 0 && logit < z ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void k_compact(CompactArgs a) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  __shared__ int lcount[NBINS];
  __shared__ int lbase[NBINS];
  __shared__ int s_taken[4], s_gated[4];
  // a full verification sweep takes every vertex (a pruned one, the flagged
  // vertices with the gate off); the gate acts from sweep 1 on
  const bool take_all = a.ctl->verify_phase == 2;
  const int sweep = a.ctl->sweep;
  const bool gate = a.gskip && a.ctl->gate_on && !a.ctl->verify_phase && sweep >= 1;
  int taken_total = 0, gated_total = 0;
  if (a.ovf_count && blockIdx.x == 0 && threadIdx.x == 0) *a.ovf_count = 0;  // the step's hub spills start empty
  for (int64_t tile = (int64_t)blockIdx.x * 256 * CU; tile < a.len; tile += (int64_t)gridDim.x * 256 * CU) {
    if (threadIdx.x < NBINS) lcount[threadIdx.x] = 0;
    int v[CU];
    uint8_t f[CU];
#pragma unroll
    for (int r = 0; r < CU; ++r) {
      const int64_t p = tile + r * 256 + threadIdx.x;
      v[r] = p < a.len ? a.list[p] : -1;
    }
#pragma unroll
    for (int r = 0; r < CU; ++r)
      f[r] = v[r] >= 0 ? ((a.prune && !take_all) ? a.F[v[r]] : (uint8_t)1) : (uint8_t)0;
    if (a.gdone) {  // batched: a graph that has stopped keeps its state
#pragma unroll
      for (int r = 0; r < CU; ++r)
        if (f[r] && a.gdone[a.gid[v[r]]]) f[r] = 0;
    }
    if (gate) {  // a flagged vertex the network expects to keep its label stays flagged, unprocessed
#pragma unroll
      for (int r = 0; r < CU; ++r)
        if (f[r] && a.gskip[v[r]]) {
          f[r] = 0;
          ++gated_total;
        }
    }
    __syncthreads();
    int bin[CU], slot[CU];
#pragma unroll
    for (int r = 0; r < CU; ++r) {
      const int64_t p = tile + r * 256 + threadIdx.x;
      bin[r] = 0;
#pragma unroll
      for (int k = 1; k < NBINS; ++k)
        if (p >= a.bounds[k]) bin[r] = k;
      slot[r] = 0;
      if (f[r]) {
        a.F[v[r]] = 0;  // marked processed before its scan
        slot[r] = atomicAdd(&lcount[bin[r]], 1);
        ++taken_total;
      }
      if (a.hub_taken && v[r] >= 0 && bin[r] == HUB_BIN) a.hub_taken[p - a.bounds[HUB_BIN]] = f[r];
    }
    __syncthreads();
    if (threadIdx.x < NBINS && lcount[threadIdx.x] > 0)
      lbase[threadIdx.x] = atomicAdd(&a.fcount[threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < CU; ++r)
      if (f[r]) a.front[a.bounds[bin[r]] + lbase[bin[r]] + slot[r]] = v[r];
    __syncthreads();
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    taken_total += __shfl_xor(taken_total, m, 64);
    gated_total += __shfl_xor(gated_total, m, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_taken[threadIdx.x >> 6] = taken_total;
    s_gated[threadIdx.x >> 6] = gated_total;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = s_taken[0] + s_taken[1] + s_taken[2] + s_taken[3];
    const int gt = s_gated[0] + s_gated[1] + s_gated[2] + s_gated[3];
    Shard &sh = a.ctl->shard[blockIdx.x & (NSHARD - 1)][NBINS];
    if (t) atomicAdd(&sh.c[0], (u64)t);
    if (gt) atomicAdd(&sh.c[1], (u64)gt);
    int64_t listed = 0;
    for (int64_t tile = (int64_t)blockIdx.x * 256 * CU; tile < a.len; tile += (int64_t)gridDim.x * 256 * CU)
      listed += min((int64_t)256 * CU, a.len - tile);
    if (listed) atomicAdd(&sh.c[2], (u64)listed);
  }
}

// ---------------------------------------------------------------- low / mid degree
//
// Both scan kernels run a three-stage software pipeline per group of lanes:
// while vertex A's labels are merged in the LDS table, the row entries of the
// next vertex B and the row offsets of the one after (C) are in flight, so a
// vertex costs about one memory latency instead of four.  The first GROUP * U
// entries of a row travel in registers (and serve the neighbour marks); the
// bins' default degree limits keep every row within that first pass.

template <int GROUP, int U, int WK, bool FEAT = false>
struct RowStage {
  int v;
  int64_t b, e;
  int32_t cur;
  uint32_t K;  // FEAT: weighted degree and sweep of the last processing
  int lp;
  int j[U];
  uint32_t w[U];
  uint32_t lbl[U];

  __device__ __forceinline__ void load_head(const ScanArgs &a, int vv) {
    v = vv;
    if (v >= 0) {
      b = a.off[v];
      e = a.off[v + 1];
      cur = a.C[v];
      if constexpr (FEAT) {
        K = a.f.K[v];
        lp = record_lastp(a.f.feat + (int64_t)v * FEAT_STRIDE);
      }
    }
  }
  __device__ __forceinline__ void load_row(const ScanArgs &a, int lane) {
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t k = b + lane + (int64_t)r * GROUP;
      const bool ok = v >= 0 && k < e;
      j[r] = ok ? a.idx[k] : -1;
      w[r] = ok ? load_w<WK>(a.w, k) : 0u;
    }
  }
  __device__ __forceinline__ void gather(const ScanArgs &a) {
#pragma unroll
    for (int r = 0; r < U; ++r) lbl[r] = (j[r] >= 0 && j[r] != v) ? (uint32_t)a.C[j[r]] : 0xFFFFFFFFu;
  }
  // Flags the neighbours held in registers; a flag already set is not
  // written again (read first: redundant byte stores to random lines are what
  // the marks would otherwise cost in write-back traffic).
  __device__ __forceinline__ u64 mark(const ScanArgs &a) const {
    uint8_t f[U];
#pragma unroll
    for (int r = 0; r < U; ++r) f[r] = (j[r] >= 0 && j[r] != v) ? a.F[j[r]] : (uint8_t)1;
    u64 n = 0;
#pragma unroll
    for (int r = 0; r < U; ++r) {
      n += (j[r] >= 0 && j[r] != v) ? 1 : 0;
      if (!f[r]) a.F[j[r]] = 1;
    }
    return n;
  }
};

// GROUP lanes of one wave per vertex (64 / GROUP vertices per wave).  For
// GROUP <= 2 the tables of a workgroup's GPB groups are interleaved (slot s of
// group g at tab[s * GPB + g], so the lanes of a wave - mostly different
// groups - hit different LDS banks); larger groups keep their table
// contiguous (the lanes of one group then spread over the banks by hash).
// REG: one thread per vertex with its table in registers (rows of at most
// SLOTS - 1 <= U entries, all loaded at once).
template <int GROUP, int SLOTS, int U, int WK, bool FEAT, bool REG = false>
__global__ __launch_bounds__(256) void k_scan_group(ScanArgs a) {
  static_assert(GROUP <= 64 && (GROUP & (GROUP - 1)) == 0, "a group lives inside one wave");
  static_assert(!REG || (GROUP == 1 && U >= SLOTS - 1), "a register table holds the bin's longest row");
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  constexpr int GPB = 256 / GROUP;
  constexpr int BITS = __builtin_ctz(SLOTS);
  constexpr int TS = GROUP <= 2 ? GPB : 1;  // table stride
  __shared__ u64 tab[REG ? 1 : GPB * SLOTS];
  const int lane = threadIdx.x % GROUP;
  const int grp = threadIdx.x / GROUP;
  u64 *T = TS == 1 ? tab + grp * SLOTS : tab + grp;
  const int count = *a.fcount;
  if ((int)blockIdx.x * GPB >= count) return;  // grids are sized for the whole list; most of a sparse step idles
  const int stride = gridDim.x * GPB;
  const bool mark_now = a.prune && !__atomic_load_n(&a.ctl->dense_cur, __ATOMIC_RELAXED);
  const int sweep = FEAT ? a.ctl->sweep : 0;
  u64 n_changed = 0, n_scanned = 0, n_vert = 0, n_marks = 0;
  int overflow = 0;
  int i = blockIdx.x * GPB + grp;
  RowStage<GROUP, U, WK, FEAT> A, B;
  A.load_head(a, i < count ? a.front[i] : -1);
  B.load_head(a, i + stride < count ? a.front[i + stride] : -1);
  A.load_row(a, lane);
  A.gather(a);
  for (; A.v >= 0; i += stride) {
    B.load_row(a, lane);
    const int vc = i + 2 * stride < count ? a.front[i + 2 * stride] : -1;
    const bool one_pass = A.e - A.b <= (int64_t)GROUP * U;
    const TieRule tr = tie_rule_of(a, A.v);
    TabStats ts{0u, 0u, 0};
    u64 best = 0;
    uint32_t own = 0;  // FEAT: summed weight of the vertex's own label
    if constexpr (REG) {
      // the label sums of the row in registers: an entry whose label occurs
      // first at it adds the weights of the later entries with that label
      overflow |= !one_pass;  // never expected: the bin limit keeps rows within the registers
#pragma unroll
      for (int r = 0; r < U; ++r) {
        if (A.lbl[r] == 0xFFFFFFFFu) continue;
        bool first = true;
        uint32_t sum = A.w[r];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          if (q == r || A.lbl[q] != A.lbl[r]) continue;
          if (q < r) first = false;
          else sum += A.w[q];
        }
        if (!first) continue;
        const u64 kk = entry_key(((u64)A.lbl[r] << 32) | sum, tr);
        best = kk > best ? kk : best;
        if constexpr (FEAT) {
          if (A.lbl[r] == (uint32_t)A.cur) own = sum;
          ++ts.nd;
          if (sum > ts.w1) {
            ts.w2 = ts.w1;
            ts.w1 = sum;
          } else if (sum > ts.w2) {
            ts.w2 = sum;
          }
        }
      }
    } else {
      // merge A
#pragma unroll
      for (int s = lane; s < SLOTS; s += GROUP) T[s * TS] = EMPTY;
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < U; ++r)
        if (A.lbl[r] != 0xFFFFFFFFu) overflow |= !lds_insert<BITS, TS>(T, A.lbl[r], A.w[r]);
      if (!one_pass)
        overflow |=
            scan_row_strided<GROUP, U, BITS, TS, WK>(a.idx, a.w, a.C, A.b + (int64_t)GROUP * U, A.e, A.v, lane, T);
      wave_lds_sync();
      u64 lbest;
      if constexpr (FEAT) lbest = table_best_stats<GROUP, SLOTS, TS>(T, lane, ts, tr);
      else lbest = table_best<GROUP, SLOTS, TS>(T, lane, tr);
      best = group_max<GROUP>(lbest);
      if constexpr (FEAT) own = table_lookup<BITS, TS>(T, (uint32_t)A.cur);
    }
    bool changed = false;
    if (best != 0) {
      const int32_t cs = (int32_t)key_label(best, tr);
      if (cs != A.cur) {
        changed = true;
        if (lane == 0) {
          a.C[A.v] = cs;
          ++n_changed;
          if (a.chg) a.chg[A.v] = 1;
        }
        if (mark_now) {
          n_marks += A.mark(a);
          if (!one_pass) n_marks += mark_row<GROUP, U>(a.idx, a.F, A.b + (int64_t)GROUP * U, A.e, A.v, lane);
        }
      }
    }
    if constexpr (FEAT) {
      const TabStats t = group_stats<GROUP>(ts);
      if (lane == 0) write_features(a.f, A.v, sweep, A.e - A.b, t, own, changed, A.K, A.lp);
    }
    if (lane == 0) {
      n_scanned += (u64)(A.e - A.b);
      ++n_vert;
    }
    wave_lds_sync();
    B.gather(a);
    A = B;
    B.load_head(a, vc);
  }
  block_accum<256>(n_changed, n_scanned, n_vert, n_marks, overflow, a.ctl, a.bin);
}

// One workgroup of BLOCK threads per vertex.
template <int BLOCK, int SLOTS, int U, int WK, bool FEAT>
__global__ __launch_bounds__(BLOCK) void k_scan_block(ScanArgs a) {
  if (__atomic_load_n(&a.ctl->done, __ATOMIC_RELAXED)) return;
  constexpr int BITS = __builtin_ctz(SLOTS);
  __shared__ u64 T[SLOTS];
  __shared__ u64 red[BLOCK / 64];
  __shared__ TabStats tred[FEAT ? BLOCK / 64 : 1];
  const int count = *a.fcount;
  if ((int)blockIdx.x >= count) return;
  const int stride = gridDim.x;
  const bool mark_now = a.prune && !__atomic_load_n(&a.ctl->dense_cur, __ATOMIC_RELAXED);
  const int sweep = FEAT ? a.ctl->sweep : 0;
  u64 n_changed = 0, n_scanned = 0, n_vert = 0, n_marks = 0;
  int overflow = 0;
  int i = blockIdx.x;
  RowStage<BLOCK, U, WK, FEAT> A, B;
  A.load_head(a, i < count ? a.front[i] : -1);
  B.load_head(a, i + stride < count ? a.front[i + stride] : -1);
  A.load_row(a, threadIdx.x);
  A.gather(a);
  for (; A.v >= 0; i += stride) {
    B.load_row(a, threadIdx.x);
    const int vc = i + 2 * stride < count ? a.front[i + 2 * stride] : -1;
    for (int s = threadIdx.x; s < SLOTS; s += BLOCK) T[s] = EMPTY;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < U; ++r)
      if (A.lbl[r] != 0xFFFFFFFFu) overflow |= !lds_insert<BITS>(T, A.lbl[r], A.w[r]);
    const bool one_pass = A.e - A.b <= (int64_t)BLOCK * U;
    if (!one_pass)
      overflow |= scan_row<BLOCK, U, BITS, WK>(a.idx, a.w, a.C, A.b + (int64_t)BLOCK * U, A.e, A.v, threadIdx.x, T);
    __syncthreads();
    TabStats ts{0u, 0u, 0};
    u64 lbest;
    const TieRule tr = tie_rule_of(a, A.v);
    if constexpr (FEAT) lbest = table_best_stats<BLOCK, SLOTS>(T, threadIdx.x, ts, tr);
    else lbest = table_best<BLOCK, SLOTS>(T, threadIdx.x, tr);
    const u64 best = block_max<BLOCK>(lbest, red);
    bool changed = false;
    if (best != 0) {
      const int32_t cs = (int32_t)key_label(best, tr);
      if (cs != A.cur) {
        changed = true;
        if (threadIdx.x == 0) {
          a.C[A.v] = cs;
          ++n_changed;
          if (a.chg) a.chg[A.v] = 1;
        }
        if (mark_now) {
          n_marks += A.mark(a);
          if (!one_pass) n_marks += mark_row<BLOCK, U>(a.idx, a.F, A.b + (int64_t)BLOCK * U, A.e, A.v, threadIdx.x);
        }
      }
    }
    if constexpr (FEAT) {
      const TabStats t = group_stats<64>(ts);
      if ((threadIdx.x & 63) == 0) tred[threadIdx.x >> 6] = t;
      __syncthreads();
      if (threadIdx.x == 0) {
        TabStats m = tred[0];
        for (int k = 1; k < BLOCK / 64; ++k) m = merge_stats(m, tred[k]);
        write_features(a.f, A.v, sweep, A.e - A.b, m, table_lookup<BITS>(T, (uint32_t)A.cur), changed, A.K, A.lp);
      }
    }
    if (threadIdx.x == 0) {
      n_scanned += (u64)(A.e - A.b);
      ++n_vert;
    }
    __syncthreads();
    B.gather(a);
    A = B;
    B.load_head(a, vc);
  }
  block_accum<BLOCK>(n_changed, n_scanned, n_vert, n_marks, overflow, a.ctl, a.bin);
}

// ---------------------------------------------------------------- launchers

template <int B, int V, int WK, bool FEAT>
static void launch_shape(dim3 grid, hipStream_t st, const ScanArgs &a) {
  constexpr BinShape sh = BIN_SHAPES[B][V];
  static_assert(sh.slots == BIN_SLOTS[B], "a bin's variants share its table size");
  if constexpr (B <= 3) {
    static_assert(sh.group <= 64, "group bins keep a vertex inside one wave");
    hipLaunchKernelGGL((k_scan_group<sh.group, sh.slots, sh.unroll, WK, FEAT, sh.reg != 0>), grid, dim3(256), 0, st,
                       a);
  } else {
    hipLaunchKernelGGL((k_scan_block<sh.group, sh.slots, sh.unroll, WK, FEAT>), grid, dim3(sh.group), 0, st, a);
  }
}

template <int B, int WK, bool FEAT>
static void launch_bin_v(int variant, dim3 grid, hipStream_t st, const ScanArgs &a) {
  switch (variant) {
    case 1: launch_shape<B, 1, WK, FEAT>(grid, st, a); break;
    case 2: launch_shape<B, 2, WK, FEAT>(grid, st, a); break;
    default: launch_shape<B, 0, WK, FEAT>(grid, st, a); break;
  }
}

template <int WK, bool FEAT>
static void launch_bin_wk(int bin, int variant, dim3 grid, hipStream_t st, const ScanArgs &a) {
  switch (bin) {
    case 0: launch_bin_v<0, WK, FEAT>(variant, grid, st, a); break;
    case 1: launch_bin_v<1, WK, FEAT>(variant, grid, st, a); break;
    case 2: launch_bin_v<2, WK, FEAT>(variant, grid, st, a); break;
    case 3: launch_bin_v<3, WK, FEAT>(variant, grid, st, a); break;
    case 4: launch_bin_v<4, WK, FEAT>(variant, grid, st, a); break;
    case 5: launch_bin_v<5, WK, FEAT>(variant, grid, st, a); break;
    default: break;
  }
}

int bin_vertices_per_block(int bin, int variant) {
  const BinShape sh = BIN_SHAPES[bin][variant];
  return bin <= 3 ? 256 / sh.group : 1;
}

void launch_scan_bin(int bin, int variant, int wk, bool feat, int blocks, hipStream_t st, const ScanArgs &a) {
  if (feat) {
    if (wk == W_UNIT) launch_bin_wk<W_UNIT, true>(bin, variant, dim3(blocks), st, a);
    else if (wk == W_U8) launch_bin_wk<W_U8, true>(bin, variant, dim3(blocks), st, a);
    else launch_bin_wk<W_U32, true>(bin, variant, dim3(blocks), st, a);
  } else {
    if (wk == W_UNIT) launch_bin_wk<W_UNIT, false>(bin, variant, dim3(blocks), st, a);
    else if (wk == W_U8) launch_bin_wk<W_U8, false>(bin, variant, dim3(blocks), st, a);
    else launch_bin_wk<W_U32, false>(bin, variant, dim3(blocks), st, a);
  }
}

void launch_gate_pass(const Ctl *ctl, const float *gate, float z, const FeatArgs &f, const uint8_t *F,
                      uint8_t *skip, int64_t n, int cu_count, const int32_t *gid, const int32_t *gphase,
                      hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)cu_count * 16));
  hipLaunchKernelGGL(k_gate_pass, dim3((unsigned)blocks), dim3(256), 0, st, ctl, gate, z, f, F, skip, n, gid,
                     gphase);
}

void launch_compact(const CompactArgs &a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_compact, dim3(blocks), dim3(256), 0, st, a);
}

void launch_init_state(const int64_t *off, int32_t *C, uint8_t *F, int64_t n, int set_labels, int set_flags,
                       int clear_isolated, const int32_t *orig, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, st, off, C, F, n, set_labels, set_flags,
                     clear_isolated, orig);
}

void launch_run_begin(Ctl *ctl, double tau, int max_iters, int64_t n, int64_t n_active, int32_t *fcount, int nfc,
                      int32_t *host_done, int dense_enabled, int dense_first, int gate_on, hipStream_t st) {
  hipLaunchKernelGGL(k_run_begin, dim3(1), dim3(256), 0, st, ctl, tau, max_iters, n, n_active, fcount, nfc, host_done,
                     dense_enabled, dense_first, gate_on);
}

__global__ void k_set_phase(Ctl *ctl, int verify, int gate_on, int extra_iters, int32_t *host_done) {
  ctl->verify_phase = verify;
  ctl->gate_on = gate_on;
  ctl->max_iters += extra_iters;
  ctl->done = 0;
  if (host_done) {
    __atomic_store_n(host_done, 0, __ATOMIC_RELAXED);
    __threadfence_system();
  }
}

void launch_set_phase(Ctl *ctl, int verify, int gate_on, int extra_iters, int32_t *host_done, hipStream_t st) {
  hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(1), 0, st, ctl, verify, gate_on, extra_iters, host_done);
}

// every vertex record: never processed
__global__ void k_feat_reset(float *feat, int64_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    feat[v * FEAT_STRIDE + FEAT_LASTP] = __int_as_float(-1);
}

void launch_feat_reset(float *feat, int64_t n, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_feat_reset, dim3(blocks < 1 ? 1 : blocks), dim3(256), 0, st, feat, n);
}

void launch_dense_fill(const Ctl *ctl, const int64_t *off, uint8_t *F, int64_t n, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_dense_fill, dim3(blocks), dim3(256), 0, st, ctl, off, F, n);
}

void launch_end_sweep(Ctl *ctl, int32_t *fcount, int nfc, int32_t *host_done, hipStream_t st) {
  hipLaunchKernelGGL(k_end_sweep, dim3(1), dim3(256), 0, st, ctl, fcount, nfc, host_done);
}

}  // namespace gvelpa
