/*
 * gvelpa.h - C ABI of the MI355X (gfx950) strict label-propagation library.
 *
 * The library runs the label-scan sweep of GVE-LPA (S. Sahu, "GVE-LPA: Fast
 * Label Propagation Algorithm (LPA) for Community Detection in Shared Memory
 * Setting", arXiv 2312.08140) on one AMD GPU.  Every step of a run executes
 * in the library's own HIP kernels.
 *
 * Conventions shared by every entry point:
 *   - Integer status codes (lpa_status); nothing throws across the ABI.
 *     lpa_status_string() gives a message for any code.
 *   - Graphs are undirected CSR with every edge stored in both directions:
 *     offsets int64[n+1], indices int32[m], optional weights float[m] that
 *     hold non-negative integers <= 2^24 (NULL = unit weights, Section 3).
 *   - Labels are vertex ids (Algorithm 1 starts from C = [0 .. |V|)), never
 *     renumbered; a vertex whose only stored neighbour is itself, or that
 *     has none, keeps its label.
 *   - Pointers are host pointers unless LPA_FLAG_DEVICE_PTRS is given, in
 *     which case they are device pointers on the handle's device.
 *   - All work is enqueued on the stream given to lpa_create (NULL = the
 *     device's null stream); calls that return results synchronise it.
 *   - One handle must not be used from two host threads at once.
 */
#ifndef GVELPA_H
#define GVELPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lpa_graph lpa_graph; /* opaque; owned by the library */

typedef enum {
  LPA_OK = 0,
  LPA_ERR_INVALID_ARG = -1,         /* NULL handle/pointer, bad mode, bad size */
  LPA_ERR_INVALID_CSR = -2,         /* offsets not monotone, offsets[0] != 0, offsets[n] != m, index out of range */
  LPA_ERR_WEIGHT_NOT_INTEGRAL = -3, /* a weight is negative, non-integral, non-finite or above 2^24 */
  LPA_ERR_TOO_LARGE = -4,           /* n >= 2^31, or a weighted degree reaches 2^32 */
  LPA_ERR_OUT_OF_MEMORY = -5,       /* device allocation failed (or exceeded GVELPA_DEVICE_BUDGET_BYTES) */
  LPA_ERR_DEVICE = -6,              /* no usable GPU, or a HIP call failed */
  LPA_ERR_NO_GATE = -7,             /* a gated run was asked for before lpa_gate_load */
  LPA_ERR_INTERNAL = -8             /* a kernel reported an internal inconsistency (e.g. table overflow) */
} lpa_status;

/* Execution modes of lpa_run. */
enum {
  LPA_MODE_ASYNC = 0,        /* labels updated in place while the sweep runs; any interleaving is valid (Section 4.1) */
  LPA_MODE_DETERMINISTIC = 1 /* vertices visited colour class by colour class; equals the sequential method in
                                (colour, id) order, see lpa_color */
};

/* Flags (bitwise or). */
enum {
  LPA_FLAG_DEVICE_PTRS = 1,     /* pointer arguments are device pointers */
  LPA_FLAG_CHECK_SYMMETRIC = 2, /* lpa_create: also verify that every (i,j,w) has a matching (j,i,w) */
  LPA_FLAG_GATE = 4,            /* lpa_run: use the learned active-set gate (needs lpa_gate_load) */
  LPA_FLAG_NO_GRAPH = 8,        /* lpa_run: launch kernels one by one instead of replaying a captured HIP graph */
  LPA_FLAG_KERNEL_TIMING = 16,  /* lpa_run: time every kernel with HIP events (implies LPA_FLAG_NO_GRAPH) */
  LPA_FLAG_VERIFY = 32,         /* lpa_run: after convergence, run one verification sweep with the gate off; if
                                   it changes more than tau * n labels, continue with plain pruning.  The sweep
                                   processes the flagged vertices: an unflagged vertex has had no neighbour
                                   change since its last scan, so scanning it again returns its own label
                                   (Section 4.1.4) and the sweep equals a full unpruned one in its result */
  LPA_FLAG_TRACE = 64,          /* lpa_run: record gate training samples (features, changed-next-sweep) */
  LPA_FLAG_EXACT_MARKS = 128,   /* lpa_run, async mode: always flag neighbours one by one.  By default a sweep
                                   that follows one in which more than half of the vertices changed writes no
                                   marks and flags every vertex at its end instead (the first sweep of a fresh
                                   run counts as such); this only adds work that cannot change a label.  Gated
                                   runs (LPA_FLAG_GATE) write exact marks after their first sweep, so that their
                                   verification sweep processes only what is flagged */
  LPA_FLAG_ONE_LAUNCH = 256,    /* lpa_run: replay all max_iters sweeps as one HIP graph launch (sweeps after
                                   the stop test exit at once); batched handles always do */
  LPA_FLAG_VERIFY_FULL = 512,   /* lpa_run: the verification sweep processes every vertex (same result as the
                                   default, at the cost of a whole sweep) */
  LPA_FLAG_NO_REORDER = 1024,   /* lpa_create, lpa_batch_create: keep vertices in id order inside the library.
                                   By default they are stored in decreasing degree order (within each graph of
                                   a batch) so that frequently gathered labels share cache lines; labels keep
                                   their values and every array crosses the boundary in id order, so results
                                   are the same */
  LPA_FLAG_NONSTRICT = 2048     /* lpa_run: non-strict LPA (Section 4.1.5): among the labels of largest summed
                                   weight, vertex v takes the one of smallest rank ((c + 1) * M_v) mod P instead
                                   of the smallest id, P = 2^31 - 1 and M_v = 1580030173^(1 + (v mod 64)) mod P
                                   (the paper picks one of them by a modulo operation on the label id; this is
                                   the reading taken) */
};

#define LPA_MAX_SWEEPS_RECORDED 64
#define LPA_NUM_TIMED_KERNELS 16

/* Per-run statistics.  Per-sweep arrays hold the first 64 sweeps. */
typedef struct {
  int32_t iterations;  /* lpaMove() calls executed (Algorithm 1), verification sweeps excluded (a batch:
                          sweeps of the batch, every graph's verification sweeps included) */
  int32_t converged;   /* 1 if the stop test dN/N <= tau held (a batch: for every graph) */
  int32_t verified;    /* LPA_FLAG_VERIFY: 1 if the verification sweep changed <= tau * n labels (a batch:
                          every graph's last verification sweep, judged by dN_g / N_g) */
  int32_t num_colors;  /* deterministic mode: colour classes */
  int64_t changed[LPA_MAX_SWEEPS_RECORDED];       /* dN of each sweep */
  int64_t frontier[LPA_MAX_SWEEPS_RECORDED];      /* vertices with >= 1 stored entry processed in each sweep */
  int64_t edges_scanned[LPA_MAX_SWEEPS_RECORDED]; /* stored entries of those vertices */
  int64_t gated_out[LPA_MAX_SWEEPS_RECORDED];     /* flagged vertices the gate skipped (kept flagged) */
  float ms[LPA_MAX_SWEEPS_RECORDED];              /* device time of each sweep */
  int64_t verify_changed;                         /* labels changed by the verification sweep(s) */
  int64_t total_changed;
  double total_ms;                                /* device time from run start to final labels */
  double setup_ms;                                /* one-off work done by this call (colouring, capture) */
  /* LPA_FLAG_KERNEL_TIMING: summed HIP-event time and launch count per kernel kind:
     0 compaction, 1..6 degree bins 0..5, 7..9 hub plan/scan/finish, 10 end of sweep,
     11 hub partition merge, 12 other, 13 gate decisions, 14 scan kernels of a snapshot
     first sweep (lpa_set_first_sweep; bins and hub chunks) */
  double kernel_ms[LPA_NUM_TIMED_KERNELS];
  int64_t kernel_launches[LPA_NUM_TIMED_KERNELS];
  /* run totals per degree bin (bin 6 = hubs): vertices processed, stored entries
     scanned, labels changed, neighbour marks written; and of the compaction:
     list entries read and vertices taken.  With weight_bytes (bytes per stored
     weight inside the library: 0 unit, 1 or 4) they give the bytes each kernel
     must move. */
  int64_t bin_vertices[8], bin_edges[8], bin_changed[8], bin_marks[8];
  int64_t compact_listed, compact_taken;
  int32_t weight_bytes;
  int32_t reserved;
  int64_t verify_edges_scanned;  /* stored entries scanned by the verification sweep(s) (0 for a batch) */
  /* snapshot first sweep (lpa_set_first_sweep), when it ran: vertices processed,
     stored entries scanned, labels changed and neighbour marks written by its
     kernels, and neighbour ids they read (counted in none of the bin totals) */
  int64_t first_vertices, first_edges, first_changed, first_marks, first_reads;
} lpa_stats;

/*
 * lpa_create - upload (or borrow) a CSR graph and prepare the sweep.
 *   out       receives the handle (set to NULL on failure).
 *   n, m      vertex and stored-entry counts; 0 <= n < 2^31, m >= 0.
 *   offsets   int64[n+1], offsets[0] = 0, non-decreasing, offsets[n] = m.
 *   indices   int32[m], 0 <= indices[e] < n.
 *   weights   float[m] integral in [0, 2^24], or NULL for unit weights; the
 *             weighted degree of every vertex must stay below 2^32.
 *   device    HIP device ordinal.
 *   hip_stream  a hipStream_t (NULL = null stream) used for all later work.
 *   flags     LPA_FLAG_DEVICE_PTRS: the three arrays are device memory and
 *             are borrowed (the caller keeps them alive and unchanged until
 *             lpa_destroy); otherwise they are copied.  LPA_FLAG_CHECK_SYMMETRIC.
 * The graph model is the one of Section 3 (w_ij = w_ji).  The library owns
 * all further device memory (labels, flags, work lists, tables).
 */
int lpa_create(lpa_graph **out, int64_t n, int64_t m, const int64_t *offsets, const int32_t *indices,
               const float *weights, int device, void *hip_stream, unsigned flags);

/*
 * lpa_run - strict label propagation, Algorithm 1 (Section 4.2) with the
 * strict update of Eq. (2): each processed vertex takes the label of largest
 * summed edge weight among its neighbours (itself excluded), the smallest
 * label id on ties (Section 2); runs until dN/N <= tolerance or max_iters
 * sweeps (Section 4.1.2-4.1.3; the paper uses 0.05 and 20).
 *   mode        LPA_MODE_ASYNC or LPA_MODE_DETERMINISTIC.
 *   prune       1: vertex pruning (Section 4.1.4) - only flagged vertices are
 *               processed, a vertex is unflagged when processed and its
 *               neighbours are flagged when it changes; 0: every vertex with a
 *               stored entry is processed in every sweep.
 *   flags       LPA_FLAG_* (DEVICE_PTRS applies to init_labels, init_flags and
 *               labels_out).
 *   init_labels int32[n] starting labels (each in [0, n)), NULL = identity.
 *   init_flags  uint8[n] starting flags, NULL = all flagged.  Together with
 *               init_labels this resumes a run from a snapshot.
 *   labels_out  int32[n] final labels (may be NULL).
 *   stats       optional statistics (may be NULL).
 * max_iters must be in [0, 1000].  Synchronises the stream before returning.
 */
int lpa_run(lpa_graph *g, double tolerance, int max_iters, int mode, int prune, unsigned flags,
            const int32_t *init_labels, const uint8_t *init_flags, int32_t *labels_out, lpa_stats *stats);

/*
 * lpa_get_flags - copy the pruning flags left by the last lpa_run (uint8[n],
 * host or device per flags); with the labels they form a resumable snapshot.
 */
int lpa_get_flags(const lpa_graph *g, uint8_t *flags_out, unsigned flags);

/*
 * lpa_modularity - modularity Q of a labeling, Eq. (1) (Section 3.2), in its
 * community form: Q = sum_c [sigma_c/2m - (Sigma_c/2m)^2], with K_i the summed
 * stored weights of row i, Sigma_c the sum of K_i over c and sigma_c the
 * stored weight with both endpoints in c.  Sums are exact integers computed
 * on the GPU; the host forms num = S1*2m - S2 and den = (2m)^2 in 128-bit
 * integers and returns (double)num / (double)den.  labels: int32[n] in [0, n)
 * (host or device per flags); labels == NULL means the labels of the last run.
 */
int lpa_modularity(const lpa_graph *g, const int32_t *labels, unsigned flags, double *q_out);

/*
 * lpa_set_variants - kernel shape of each degree bin 0..5 (count must be 6;
 * NULL restores the defaults): 0, 1 or 2, a choice of lanes per vertex and
 * row entries in flight per lane at the bin's fixed table size.  Results do
 * not depend on it (the deterministic mode stays label-for-label equal).
 */
int lpa_set_variants(lpa_graph *g, const int32_t *variant, int32_t count);

/*
 * lpa_autotune - tunes the handle on its own graph with runs of the given
 * tolerance, max_iters >= 1 and mode (pruning on).  Asynchronous mode first:
 * among the schedules (early steps, early sweeps, late steps) = (16, 0, 16),
 * (16, 1, 4), (16, 2, 4), (16, 2, 8), (16, 3, 4), (16, 3, 8), (1, 0, 1) (one
 * step: every flagged vertex at once) it installs the fastest whose runs
 * converge (a batch: every graph) and whose modularity stays within 0.002 of
 * the first's; the first stays when no other qualifies (schedule_out: int32[3],
 * may be NULL).  Then the degree limits of the bins (lpa_set_bins): each
 * bin's LDS table has a fixed size (8, 32, 128, 512, 2048, 8192 slots), and
 * the candidates let it fill to at most 1/2 (the default), 1/4, 3/4 or all of
 * them; in the asynchronous mode each candidate is timed together with the
 * order of the bins in a step (lpa_set_bin_order; on a graph with hubs) and,
 * where the rows allow it, the kernels of each step of the first sweep that
 * read the initial labels (lpa_set_first_sweep: none, 1, 3 or all, then 2 and
 * 4 next to the best); the fastest combination is kept and, in the
 * asynchronous mode, each bin's limit is then tried at the other fill levels
 * on its own (limits kept non-decreasing; a change must be 1.5 % faster); the
 * result is installed (read it back with lpa_get_schedule) and its limits
 * returned in bins_out (int32[6], may be NULL).  Then it times every kernel
 * shape variant (per-kernel timing), keeps for each bin the fastest and
 * returns it in variant_out (int32[6], may be NULL) with the chosen kernels'
 * times in bin_ms_out (double[6], ms per run, 0 for an empty bin; may be
 * NULL).  A later candidate replaces an earlier one only when it is at least
 * 3 % faster, so near-ties keep the earlier (default) choice.  In the
 * asynchronous mode every candidate of the three steps must also converge
 * and keep the modularity of its runs within 0.002 of the all-16-step
 * schedule's (the processing order they set changes which labels a sweep
 * sees); the mix of per-bin kernel shapes is checked once more as a whole
 * and replaced by the default shapes if it fails.  None of these settings
 * changes a deterministic result.  Leaves the labels of its last trial run.
 */
int lpa_autotune(lpa_graph *g, double tolerance, int max_iters, int mode, int32_t *variant_out, double *bin_ms_out,
                 int32_t *schedule_out, int32_t *bins_out);

/*
 * lpa_set_async_schedule - schedule of the asynchronous mode.  The flagged
 * vertices of a sweep are split into steps processed one after the other,
 * every vertex of a step at once, so a step sees the labels earlier steps
 * wrote in place (Section 4.1).  The first `early_sweeps` sweeps of a run use
 * `early_phases` steps, later sweeps (and a verification sweep)
 * `late_phases` steps; the default is 16 steps for 2 sweeps, then 4.
 * by_colour = 1: steps are runs of consecutive colour classes of lpa_color,
 * about n / phases vertices each (vertices of one class are never adjacent);
 * 0: steps by a fixed hash of the vertex id.  Phases in [1, 1024],
 * early_sweeps in [0, 1000]; takes effect for the next lpa_run.
 */
int lpa_set_async_schedule(lpa_graph *g, int32_t early_phases, int32_t early_sweeps, int32_t late_phases,
                           int32_t by_colour);

/* lpa_set_async_phases - the same number of steps in every sweep. */
int lpa_set_async_phases(lpa_graph *g, int32_t phases, int32_t by_colour);

/*
 * lpa_set_bin_order - order of the degree bins inside a step: 0 (the
 * default) runs the hub bin first and then the lower bins from the largest
 * degree down; 1 runs the lower bins first and the hubs last, so that the
 * hubs see the labels the other vertices of the step have just written.  In
 * the asynchronous mode this changes which labels a step sees (any order is
 * a valid run); deterministic results do not depend on it (the vertices of a
 * colour class are never adjacent).  Takes effect for the next lpa_run.
 */
int lpa_set_bin_order(lpa_graph *g, int32_t hubs_last);

/*
 * lpa_set_bins - degree limits of bins 0..5 (count must be 6, non-decreasing,
 * each below its bin's table size 8, 32, 128, 512, 2048, 8192; NULL restores
 * 4, 16, 64, 256, 1024, 4096); rows above the last limit take the hub path.
 * Results do not depend on them (the deterministic mode stays label-for-label
 * equal); takes effect for the next lpa_run.
 */
int lpa_set_bins(lpa_graph *g, const int32_t *max_degree, int32_t count);

/*
 * lpa_set_first_sweep - snapshot first sweep (asynchronous mode): in the
 * first sweep of a run that starts from the initial labels (no init_labels),
 * the first `kernels` kernels of every step - in processing order, one per
 * degree bin and one for the hubs (lpa_set_bin_order) - read every label as
 * it was when the sweep began, which is one interleaving of an asynchronous
 * sweep (Section 4.1): their reads precede the writes of the sweep.  Those
 * labels are the vertex ids (Algorithm 1 starts from C[v] = v) and each occurs
 * once in a row without repeated neighbours, so Eq. (2) becomes the heaviest
 * entry (smallest id, or rank in non-strict LPA, among the heaviest): these
 * kernels need no label table and read a neighbour's id only for entries of
 * the running maximum weight.  kernels: 0 (the default) to 7 (every kernel of
 * the sweep); other values give LPA_ERR_INVALID_ARG.  Applies only when
 * every row's neighbours are strictly increasing (lpa_get_schedule reports
 * it) and no gate or trace is on; otherwise the first sweep runs like the
 * others.  Deterministic runs never use it.  Takes effect for the next
 * lpa_run.
 */
int lpa_set_first_sweep(lpa_graph *g, int32_t kernels);

/*
 * lpa_get_schedule - the handle's current asynchronous configuration, as
 * lpa_autotune leaves it: out int32[7] = early steps, early sweeps, late
 * steps, steps by colour (1) or by hash (0), hubs last (1) or first (0),
 * kernels of the snapshot first sweep (lpa_set_first_sweep), and whether the
 * rows allow it (1: every row's neighbours strictly increase).
 */
int lpa_get_schedule(const lpa_graph *g, int32_t *out);

/*
 * lpa_color - colouring used by the deterministic mode (computed on first use):
 * Jones-Plassmann with priority (deg(v), fmix32(v ^ seed), v) compared
 * lexicographically - deg(v) being the stored entries of row v and fmix32 the
 * MurmurHash3 32-bit finaliser - which equals the greedy colouring that takes
 * vertices in decreasing priority.  colors_out int32[n] (host or device per
 * flags, may be NULL); *num_colors receives the class count.
 */
int lpa_color(lpa_graph *g, uint32_t seed, int32_t *colors_out, unsigned flags, int32_t *num_colors);

/*
 * lpa_batch_create - many independent graphs in one handle: a block-diagonal
 * CSR (no entry crosses graphs) where graph g owns vertices
 * [graph_vptr[g], graph_vptr[g+1]).  lpa_run then applies Algorithm 1 to
 * every graph separately - its own sweep count and its own stop test
 * dN_g / N_g <= tolerance; a graph that stops keeps its labels and flags while
 * the others go on, and the whole run is one HIP graph launch.  Labels are
 * global vertex ids.  graph_vptr is int64[n_graphs+1] (host memory);
 * an entry joining two graphs gives LPA_ERR_INVALID_CSR.  Gated and verified
 * runs (LPA_FLAG_GATE, LPA_FLAG_VERIFY, LPA_FLAG_VERIFY_FULL) apply the
 * single-graph procedure to every graph on the device, in the same launch:
 * after its stop test (or its max_iters sweeps) a graph runs its own
 * verification sweep with the gate off; one that changes more than
 * tolerance * N_g labels goes on with plain sweeps (at least one, at most
 * max_iters, ending once the graph's sweeps, its verification included,
 * reach 2 * max_iters) and a last verification sweep.  Dense sweeps (see LPA_FLAG_EXACT_MARKS) are then
 * limited to the first sweep.
 */
int lpa_batch_create(lpa_graph **out, int32_t n_graphs, const int64_t *graph_vptr, int64_t n, int64_t m,
                     const int64_t *offsets, const int32_t *indices, const float *weights, int device,
                     void *hip_stream, unsigned flags);

/*
 * lpa_batch_stats - per-graph results of the last batched run:
 * iterations[n_graphs] and converged[n_graphs] (host arrays, may be NULL).
 */
int lpa_batch_stats(const lpa_graph *g, int32_t *iterations, int32_t *converged);

/*
 * lpa_batch_verify_stats - per-graph verification outcome of the last
 * batched run with LPA_FLAG_GATE / LPA_FLAG_VERIFY / LPA_FLAG_VERIFY_FULL:
 * verified[n_graphs] (1 if the graph's last verification sweep changed
 * <= tolerance * N_g labels; empty graphs count as verified) and
 * verify_changed[n_graphs] (labels changed by its verification sweeps); host
 * arrays, may be NULL.  iterations from lpa_batch_stats exclude the
 * verification sweeps.  LPA_ERR_INVALID_ARG for a handle that is no batch.
 */
int lpa_batch_verify_stats(const lpa_graph *g, int32_t *verified, int32_t *verify_changed);

/*
 * Learned active-set gate.  Vertex pruning (Section 4.1.4) processes every
 * flagged vertex; the gate additionally skips a flagged vertex whose
 * predicted chance of changing its label is below a threshold, and keeps it
 * flagged for later sweeps.  The predictor is a network 8-32-32-1 (ReLU,
 * ReLU, sigmoid) over eight features that each processing of a vertex leaves
 * behind: log2(1 + deg), (W1 - W2) / K, W(own label) / K, changed at its last
 * processing, sweep / max_iters, W1 / K, distinct neighbour labels / deg and
 * min(sweeps since last processed, 8) / 8, where W1 >= W2 are the two largest
 * label weights among the neighbours and K the weighted degree.  Parameters
 * are 1377 FP32 values, W1[32][8], b1[32], W2[32][32], b2[32], W3[32], b3
 * (row-major); the GPU evaluates their bf16 rounding (to nearest, ties to
 * even) with FP32 sums.  The decisions of a sweep are taken at its start for
 * the vertices flagged then.  A gated run (LPA_FLAG_GATE) always ends with a
 * verification sweep (LPA_FLAG_VERIFY); if that sweep changes more than
 * tolerance * n labels the run continues with plain pruning.
 */

/*
 * lpa_gate_load - install gate parameters (host float[1377], finite) and the
 * threshold in [0, 1]: a flagged vertex is processed when p >= threshold
 * (0: every flagged vertex, the plain method; 1: none before verification).
 * Takes effect for the next lpa_run with LPA_FLAG_GATE.
 */
int lpa_gate_load(lpa_graph *g, const float *params, float threshold);

/*
 * lpa_set_trace - make runs with LPA_FLAG_TRACE record training samples: for
 * a vertex processed in sweep s that was last processed in sweep s' < s, the
 * features it had for the decision at sweep s and the target 1 if its label
 * changed at s.  Each such event is kept with the given probability (a fixed
 * hash of (vertex, sweep)); at most `capacity` samples are kept.  Resets the
 * sample buffer (capacity 0 frees it).
 */
int lpa_set_trace(lpa_graph *g, int64_t capacity, double probability);

/*
 * lpa_gate_trace - the samples recorded since lpa_set_trace: *count receives
 * their number; with features != NULL, copies float[count][8] features and
 * uint8[count] targets (host or device per flags; capacity = their length in
 * samples, which must be >= *count).
 */
int lpa_gate_trace(const lpa_graph *g, float *features, uint8_t *targets, int64_t capacity, int64_t *count,
                   unsigned flags);

/*
 * lpa_gate_forward - probabilities float[count] of the gate network for the
 * features float[count][8] (host or device per flags; params always host).
 * Runs on `device`, enqueued on hip_stream, synchronised before returning.
 */
int lpa_gate_forward(const float *params, const float *features, int64_t count, float *probs, int device,
                     void *hip_stream, unsigned flags);

/*
 * lpa_gate_backward - gradient (host float[1377]) and value (*loss, may be
 * NULL) of the mean weighted binary cross-entropy
 *   L = mean over samples of -(pos_weight * y * log p + (1 - y) * log(1 - p))
 * at params, over features float[count][8] and targets uint8[count] (0 or not
 * 0; host or device per flags).  pos_weight >= 0.
 */
int lpa_gate_backward(const float *params, const float *features, const uint8_t *targets, int64_t count,
                      float pos_weight, float *grad, float *loss, int device, void *hip_stream, unsigned flags);

/*
 * lpa_gate_backward_noalloc - lpa_gate_backward for callers that cannot
 * allocate device memory (tight training loops, harnesses that forbid
 * hipMalloc): the same gradient and loss, bit for bit, computed without any
 * allocation.  Its scratch (the device copy of the parameters and the
 * per-workgroup partial gradients) lives in a fixed array of about 11.3 MB in
 * the library's device memory, one copy per GPU, held until the process ends.
 *   params     host float[1377] (finite).
 *   features   DEVICE float[count][8]; targets DEVICE uint8[count].
 *   count      1 .. LPA_GATE_NOALLOC_MAX_SAMPLES; larger counts return
 *              LPA_ERR_TOO_LARGE (split them, or use lpa_gate_backward).
 *   grad       host float[1377]; loss host float (may be NULL).
 * Every call on a GPU shares that GPU's scratch: calls that overlap on one
 * GPU (from several host threads or streams) race and must be serialised by
 * the caller.  Synchronises hip_stream before returning.
 */
#define LPA_GATE_NOALLOC_MAX_SAMPLES 262144
int lpa_gate_backward_noalloc(const float *params, const float *features, const uint8_t *targets, int64_t count,
                              float pos_weight, float *grad, float *loss, int device, void *hip_stream);

/*
 * lpa_gate_train - Adam (Kingma and Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected) on the loss of lpa_gate_backward, FP32 master parameters
 * updated in place in params (host float[1377]).  Each epoch takes the samples
 * in the order order[e * count .. (e+1) * count) (int64, each in [0, count);
 * NULL: 0, 1, ...) in mini-batches of `batch`, one update per mini-batch (its
 * mean loss).  epoch_loss (host float[epochs], may be NULL) receives each
 * epoch's sample-weighted mean of the mini-batch losses, each taken before its
 * update.  features, targets and order are host or device per flags.
 */
int lpa_gate_train(float *params, const float *features, const uint8_t *targets, int64_t count,
                   const int64_t *order, int32_t epochs, int32_t batch, float lr, float pos_weight,
                   float *epoch_loss, int device, void *hip_stream, unsigned flags);

/*
 * lpa_gate_threshold - the largest threshold t such that at least a fraction
 * `recall` of the samples with target 1 have p >= t (1 when no target is 1);
 * arrays as in lpa_gate_backward.
 */
int lpa_gate_threshold(const float *params, const float *features, const uint8_t *targets, int64_t count,
                       double recall, float *threshold, int device, void *hip_stream, unsigned flags);

/*
 * lpa_nmi - normalised mutual information of two labelings a, b (int32[n],
 * any values; host or device per flags): 2 I(X;Y) / (H(X) + H(Y)) with
 * natural logarithms, the quality measure the paper names in Section 1
 * (arithmetic normalisation); 1 when both have a single class or n = 0.
 * Runs on `device`, enqueued on hip_stream, synchronised before returning.
 */
int lpa_nmi(const int32_t *a, const int32_t *b, int64_t n, double *nmi_out, int device, void *hip_stream,
            unsigned flags);

/* lpa_destroy - release the handle and all device memory it owns (NULL is a no-op). */
void lpa_destroy(lpa_graph *g);

/* lpa_status_string - static message for a status code. */
const char *lpa_status_string(int status);

/* lpa_last_error_detail - for the last LPA_ERR_DEVICE returned on this
 * thread, the HIP error and the call that failed ("" if none); valid until
 * the next failing call on the thread. */
const char *lpa_last_error_detail(void);

#ifdef __cplusplus
}
#endif
#endif /* GVELPA_H */
