/*
 * gvelpa_cpu.h - multicore CPU label propagation in the paper's own design.
 *
 * A host-only comparator for the GPU library: the parallel GVE-LPA of the
 * paper (Sections 4.1-4.2, Algorithm 1) on shared-memory CPU threads, written
 * from its description.  It is a separate library (libgvelpa_cpu.so); the GPU
 * path never calls it.
 *
 *   - OpenMP threads over the vertices with a dynamic schedule of chunk 2048
 *     (Section 4.1.1);
 *   - asynchronous, in-place label updates: a thread sees the labels other
 *     threads have already written in this sweep (Section 4.1);
 *   - vertex pruning with 8-bit flags: a vertex is unflagged when processed
 *     and its neighbours are flagged when its label changes (Section 4.1.4);
 *   - per-thread "Far-KV" hashtables: a keys list plus a values array indexed
 *     by label with one slot per vertex, separately allocated per thread so
 *     threads never share cache lines (Section 4.1.6);
 *   - changed-label count by a parallel reduction, stop when dN/N <= tolerance
 *     or after max_iters sweeps (Sections 4.1.2-4.1.3);
 *   - strict tie rule (smallest label id) or the non-strict one of
 *     gvelpa.h's LPA_FLAG_NONSTRICT (Section 4.1.5).
 * With one thread the run is the sequential method in id order.
 */
#ifndef GVELPA_CPU_H
#define GVELPA_CPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * gvcpu_lpa - label propagation on a host CSR graph (the conventions of
 * gvelpa.h: undirected, both directions stored, weights NULL or integral
 * floats in [0, 2^24], weighted degrees below 2^32).
 *   tolerance, max_iters (0 .. 1000), prune (0/1), nonstrict (0/1).
 *   threads    OpenMP threads (<= 0: the OpenMP default).
 *   labels     out: int32[n] final labels (vertex ids).
 *   changed, processed, scanned   out (may be NULL): int64[max(max_iters, 1)]
 *              per sweep: labels changed, flagged vertices with a stored entry
 *              processed, and their stored entries.
 *   iterations, converged        out (may be NULL).
 *   seconds    out (may be NULL): wall time of the sweeps (tables allocated
 *              before the clock starts).
 * Returns 0, -1 for invalid arguments (bad CSR, weights or sizes), -2 when
 * memory runs out.
 */
int gvcpu_lpa(int64_t n, const int64_t *offsets, const int32_t *indices, const float *weights, double tolerance,
              int max_iters, int prune, int nonstrict, int threads, int32_t *labels, int64_t *changed,
              int64_t *processed, int64_t *scanned, int32_t *iterations, int32_t *converged, double *seconds);

/* gvcpu_max_threads - the OpenMP default thread count. */
int gvcpu_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif /* GVELPA_CPU_H */
