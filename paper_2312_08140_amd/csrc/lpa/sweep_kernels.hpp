// Host-visible launchers of the gfx950 kernels.
#pragma once
#include "common.hpp"

namespace gvelpa {

// records the failing HIP call for lpa_last_error_detail (engine.hip)
void note_hip_error(int err, const char *what, const char *file, int line);

// Arguments of one frontier compaction (one step: the whole graph in async
// mode, one colour class in deterministic mode).  Entries [bounds[b],
// bounds[b+1]) of `list` are the step's vertices of bin b; the flagged ones
// are written to the same range of `front`, counted in fcount[b].
struct CompactArgs {
  const int32_t *list;
  int64_t len;
  int32_t bounds[NBINS + 1];
  uint8_t *F;
  int32_t *front;
  int32_t *fcount;
  Ctl *ctl;
  int prune;
  const int32_t *gid;    // batched runs: graph of every vertex (NULL otherwise)
  const int32_t *gdone;  // batched runs: 1 for a graph that has stopped
  const uint8_t *gskip;  // gate decisions of the sweep (k_gate_pass; NULL: no gate)
  FeatArgs f;
  // static hub plan: taken[p - bounds[HUB_BIN]] = 1 for each hub-bin entry
  // taken in this step, 0 for the others; the spill counter is cleared
  uint8_t *hub_taken;
  u64 *ovf_count;
};

void launch_compact(const CompactArgs &a, int blocks, hipStream_t st);
// gid, gphase: batched runs (NULL otherwise); only graphs in their gated sweeps (phase 0) pass the gate
void launch_gate_pass(const Ctl *ctl, const float *gate, float z, const FeatArgs &f, const uint8_t *F,
                      uint8_t *skip, int64_t n, int cu_count, const int32_t *gid, const int32_t *gphase,
                      hipStream_t st);
void launch_scan_bin(int bin, int variant, int wk, bool feat, int blocks, hipStream_t st, const ScanArgs &a);
int bin_vertices_per_block(int bin, int variant);
// max_hubs: most flagged hubs the step can have (its hub-bin segment)
void launch_hub_plan(const ScanArgs &a, const HubArgs &h, int64_t max_hubs, int blocks, int tile_blocks,
                     hipStream_t st);
int hub_plan_tiles(int64_t entries);  // tiles of the hub plan for that many frontier hubs
void launch_hub_chunk(int wk, int blocks, hipStream_t st, const ScanArgs &a, const HubArgs &h);
// snapshot first sweep (first_sweep.hip)
void launch_first_bin(int bin, int variant, int wk, bool feat, int blocks, hipStream_t st, const ScanArgs &a);
void launch_hub_first_chunk(int wk, int blocks, hipStream_t st, const ScanArgs &a, const HubArgs &h);
void launch_hub_part(int blocks, bool feat, hipStream_t st, const ScanArgs &a, const HubArgs &h);
// the hub decision and neighbour marks: k_hub_decide + k_hub_mark, or (fused)
// k_hub_finish, whose every chunk re-reads the hub's partition maxima
void launch_hub_finish(int hub_blocks, int chunk_blocks, int prune, bool feat, bool fused, hipStream_t st,
                       const ScanArgs &a, const HubArgs &h);
void launch_init_state(const int64_t *off, int32_t *C, uint8_t *F, int64_t n, int set_labels, int set_flags,
                       int clear_isolated, const int32_t *orig, hipStream_t st);
void launch_run_begin(Ctl *ctl, double tau, int max_iters, int64_t n, int64_t n_active, int32_t *fcount, int nfc,
                      int32_t *host_done, int dense_enabled, int dense_first, int gate_on, hipStream_t st);
void launch_dense_fill(const Ctl *ctl, const int64_t *off, uint8_t *F, int64_t n, hipStream_t st);
void launch_set_phase(Ctl *ctl, int verify, int gate_on, int extra_iters, int32_t *host_done, hipStream_t st);
void launch_feat_reset(float *feat, int64_t n, hipStream_t st);

// batched runs (graph g owns vertices [vptr[g], vptr[g+1]))
// Phases of a graph in a verified run: BPH_MAIN (the method's sweeps, gated
// when the gate is on), BPH_VERIFY (verification sweep), BPH_FALLBACK (plain
// sweeps after a failed verification), BPH_VERIFY2 (the last verification),
// BPH_DONE.
enum { BPH_MAIN = 0, BPH_VERIFY = 1, BPH_FALLBACK = 2, BPH_VERIFY2 = 3, BPH_DONE = 4 };
struct BatchArgs {
  int32_t ngraphs;
  const int64_t *vptr;
  int32_t *gid;
  uint8_t *chg;
  int32_t *gdone, *giters, *gconv;
  int32_t *gphase, *gcap, *gverified, *gvchanged;  // verified runs (phase, fallback cap, outcome)
  const int64_t *off;                               // full verification: flags every vertex with entries
  uint8_t *F;
};
void launch_batch_gid(const BatchArgs &b, hipStream_t st);
// mode: verification mode (0 none, 1 flagged vertices, 2 all); iters: sweep cap of the method per graph
void launch_batch_begin(Ctl *ctl, const BatchArgs &b, int64_t n, int32_t live, int mode, int iters,
                        hipStream_t st);
void launch_batch_end(Ctl *ctl, const BatchArgs &b, hipStream_t st);
void launch_check_block_diagonal(const int64_t *off, const int32_t *idx, const int32_t *gid, int64_t n, int32_t *bad,
                                 hipStream_t st);
void launch_end_sweep(Ctl *ctl, int32_t *fcount, int nfc, int32_t *host_done, hipStream_t st);

// setup_kernels.hip
struct CsrCheck {
  int32_t bad_index;      // an index outside [0, n)
  int32_t bad_weight;     // negative, non-integral, non-finite or > 2^24
  int32_t bad_offsets;    // decreasing offsets
  int32_t big_degree;     // weighted degree >= 2^32
  uint32_t max_weight;
  int32_t not_all_ones;
  int32_t asym;           // LPA_FLAG_CHECK_SYMMETRIC: a missing or different reverse entry
  int32_t rows_not_strict;  // a row whose neighbours are not strictly increasing (unsorted or repeated)
};
void launch_check_offsets(const int64_t *off, int64_t n, CsrCheck *chk, hipStream_t st);
void launch_check_edges(const int32_t *idx, const float *w, int64_t m, int64_t n, CsrCheck *chk, hipStream_t st);
void launch_check_rows(const int64_t *off, const int32_t *idx, int64_t n, CsrCheck *chk, hipStream_t st);
void launch_convert_weights(const float *w, int64_t m, int wk, void *out, hipStream_t st);
void launch_weighted_degree(const int64_t *off, const void *w, int wk, int64_t n, uint32_t *K, CsrCheck *chk,
                            hipStream_t st);
void launch_check_symmetric(const int64_t *off, const int32_t *idx, const void *w, int wk, int64_t n,
                            CsrCheck *chk, hipStream_t st);
void launch_bin_hist(const int64_t *off, int64_t n, const int32_t *color, const int32_t *cmap, int nphase,
                     const BinLimits &lim, int32_t *hist, int nkeys, hipStream_t st);
void launch_bin_scatter(const int64_t *off, int64_t n, const int32_t *color, const int32_t *cmap, int nphase,
                        const BinLimits &lim, int32_t *cursor, int32_t *list, int nkeys, hipStream_t st);
uint32_t phase_seed();
void launch_color_init(const int64_t *off, const int32_t *idx, int32_t *color, u64 *pk, int32_t *pending,
                       int32_t *front, int32_t *count, int64_t n, uint32_t seed, const int32_t *orig,
                       hipStream_t st);
void launch_color_round(const int64_t *off, const int32_t *idx, int32_t *color, const u64 *pk, int32_t *pending,
                        const int32_t *work_in, int32_t *work_out, int32_t *counts, int r, int blocks,
                        const int32_t *orig, hipStream_t st);

// metrics_kernels.hip
struct ModAcc {
  u64 two_m;
  u64 s1;
};
void launch_mod_community_totals(const int32_t *C, const uint32_t *K, int64_t n, u64 *tot, hipStream_t st);
void launch_mod_inside(const int64_t *off, const int32_t *idx, const void *w, int wk, const int32_t *C, int64_t n,
                       int64_t m, ModAcc *acc, hipStream_t st);
int mod_square_blocks();
void launch_mod_squares(const u64 *tot, int64_t n, u64 *partials /* 2 per block */, hipStream_t st);
void launch_check_labels(const int32_t *C, int64_t n, int32_t *bad, hipStream_t st);

// reorder.hip: vertices stored in decreasing degree order (labels keep their
// values, the original ids); order[p] = vertex at position p, pos[v] its position.
int64_t order_temp_bytes(int64_t n);
hipError_t build_order(const int64_t *off, const int32_t *gid, int64_t n, int32_t *order, int32_t *pos,
                       int64_t *noff, u64 *keys, void *temp, int64_t temp_bytes, hipStream_t st);
void launch_permute_rows(const int64_t *off, const int32_t *idx, const void *w, int wk, const int32_t *order,
                         const int32_t *pos, const int64_t *noff, int32_t *nidx, void *nw, int64_t n,
                         hipStream_t st);
int64_t row_sort_temp_bytes(int64_t chunk);
hipError_t sort_rows_chunk(const int64_t *off, int64_t r0, int64_t r1, int64_t e0, int64_t len, int32_t *idx,
                           void *w, int wk, u64 *keys, int32_t *perm, void *wcopy, void *temp, int64_t temp_bytes,
                           hipStream_t st);
void launch_gather_i32(int32_t *dst, const int32_t *src, const int32_t *index, int64_t n, hipStream_t st);
// out[c] = idx[at[c]] (64-bit positions)
void launch_gather_at(const int32_t *idx, const int64_t *at, int64_t count, int32_t *out, hipStream_t st);
void launch_gather_u8(uint8_t *dst, const uint8_t *src, const int32_t *index, int64_t n, hipStream_t st);

// gate_kernels.hip: the gate network's forward pass, gradient of the weighted
// BCE (per-workgroup partials of GATE_PARAMS + 1 floats, the last the loss,
// summed into grad) and the Adam update of the FP32 master parameters.
void launch_gate_forward(const float *master, const float *X, int64_t count, float *p, hipStream_t st);
int gate_grad_blocks(int64_t nb);
void launch_gate_grad(const float *master, const float *X, const uint8_t *Y, const int64_t *sel, int64_t base,
                      int64_t nb, float pw, float denom, float *partial, float *grad, hipStream_t st);
void launch_adam(float *theta, const float *grad, float *m, float *v, int t, float lr, float b1, float b2, float eps,
                 float *loss_acc, float loss_scale, hipStream_t st);
void launch_check_index(const int64_t *sel, int64_t len, int64_t limit, int32_t *bad, hipStream_t st);
void launch_select_pos(const float *p, const uint8_t *Y, int64_t count, float *out, unsigned long long *npos,
                       hipStream_t st);

}  // namespace gvelpa
