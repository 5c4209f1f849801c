/*
 * gvelpa_gen.h - seeded synthetic graphs assembled on the GPU.
 *
 * The paper runs on graphs whose reverse edges are added (Section 5.1,
 * Table 1: |E| counts both directions) and treats them as undirected with
 * symmetric weights (Section 3).  These entry points build such inputs
 * directly in device memory.  They are input generators only: they hold none
 * of the label-propagation arithmetic, and the CSR they produce is
 * bit-identical to the one the host generator of the Python package
 * (graphgen.rmat) returns for the same parameters, so a graph made here can
 * be checked against the host-generated copy entry by entry.
 *
 * Output CSR: undirected, every edge stored in both directions, no
 * self-loops, no duplicate entries, rows sorted by neighbour id; int64
 * offsets[n+1], int32 indices[m], optional fp32 weights[m] holding integers.
 */
#ifndef GVELPA_GEN_H
#define GVELPA_GEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Allocator of the output arrays, called on the calling host thread with
 * the device current: kind 0 = offsets (int64, count = n + 1), 1 = indices
 * (int32, count = m), 2 = weights (float, count = m).  It returns device
 * memory of at least max(count, 1) elements, owned by the caller, or NULL
 * (the generator then fails with GVGEN_ERR_OUT_OF_MEMORY). */
typedef void *(*gvgen_alloc_fn)(int kind, int64_t count);

enum {
  GVGEN_OK = 0,
  GVGEN_ERR_INVALID_ARG = -1,    /* parameters out of range */
  GVGEN_ERR_OUT_OF_MEMORY = -2,  /* a device allocation (own scratch or the caller's) failed */
  GVGEN_ERR_DEVICE = -3          /* a HIP call failed */
};

/*
 * gvgen_rmat - R-MAT graph (Chakrabarti, Zhan and Faloutsos, SDM 2004)
 * without noise and without vertex permutation: 2^scale vertices and
 * edge_factor * 2^scale generated edges; edge e descends `scale` levels of
 * the quadrant recursion with probabilities (a, b, c, 1 - a - b - c), two
 * levels per 64-bit counter-based draw (SplitMix64 output function of
 * key + (counter + 1) * 0x9E3779B97F4A7C15).  Self-loops are dropped, both
 * directions stored, duplicates removed.
 *   scale       1..30; edge_factor >= 1; a, b, c >= 0 with a + b + c <= 1.
 *   seed        the graph is a pure function of the parameters and the seed.
 *   weighted    1: weight 1 + (hash of the unordered pair & 7), symmetric;
 *               0: all weights 1.0; -1: no weight array (unit weights).
 *   device, hip_stream  where the work runs (NULL = null stream); the call
 *               synchronises the stream before returning.
 *   alloc       allocator of the three output arrays (above).
 *   n_out, m_out  vertex and stored-entry counts.
 * Scratch memory of about 4 bytes per generated edge direction plus 8 bytes
 * per vertex (plus a sort buffer of at most 4 GiB) is allocated and freed by
 * the call.  Returns GVGEN_OK or a negative code.
 */
int gvgen_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed, int weighted, int device,
               void *hip_stream, gvgen_alloc_fn alloc, int64_t *n_out, int64_t *m_out);

/* gvgen_status_string - static message for a status code. */
const char *gvgen_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* GVELPA_GEN_H */
