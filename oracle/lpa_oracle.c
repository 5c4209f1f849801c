/*
 * Sequential CPU oracle for strict label propagation (GVE-LPA, arXiv 2312.08140).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can check the GPU library against a plain,
 * obviously correct implementation.  It shares no code with the GPU path.
 *
 * Everything here is plain C99, sequential, in place and unoptimised.
 *
 *   oracle_lpa         Algorithm 1 (Section 4.2): lpa() with lpaMove() and
 *                      scanCommunities(), executed one vertex at a time in an
 *                      explicit order pi; the update rule is Eq. (2) (the
 *                      label-propagation argmax, Section 3.3) in its strict
 *                      form (Section 4.1.5, and the smallest-id tie rule
 *                      stated in Section 2) or, on request, the non-strict
 *                      form of Section 4.1.5 (tie_rank below).
 *   oracle_color       greedy colouring in decreasing (degree, hash, id)
 *                      priority; defines the vertex order of the
 *                      deterministic GPU mode.
 *   oracle_modularity  Eq. (1) (Section 3.2), community form, in exact integers with one
 *                      final FP64 division.
 *
 * Readings of points the paper leaves open:
 *   - ties go to the smallest label id; the current label gets no preference;
 *   - a vertex with no neighbour other than itself keeps its label and does
 *     not count as changed;
 *   - the stop test is (double)dN / (double)N <= tau, with tau fixed;
 *   - a vertex's flag is cleared before its scan; marks are in place, so a
 *     vertex marked before its turn in the current sweep is processed in it;
 *   - re-marking skips the vertex itself (self-loops are not neighbours);
 *   - weights are integers (given as fp32) and sums are exact (uint64).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_STATS 64

/* Non-strict tie rule (Section 4.1.5 names it: among the labels of maximum
 * weight one is picked by a modulo operation on the label id instead of the
 * smallest id).  Reading taken here: vertex v ranks the dominant labels by
 *   r_v(c) = ((c + 1) * A^(1 + (v mod 64))) mod P,  P = 2^31 - 1 (prime),
 * A = TIE_A, and takes the label of smallest rank.  For a fixed v, distinct
 * labels get distinct ranks (P is prime and neither factor is 0 mod P), so
 * the pick is unique; it changes with v mod 64 like a random pick would. */
#define TIE_P 2147483647ull
#define TIE_A 1580030173ull

/* A^(1 + (v mod 64)) mod P, by repeated multiplication */
static uint64_t tie_mult(int64_t v) {
  uint64_t m = 1;
  for (int64_t k = 0; k <= v % 64; ++k) m = m * TIE_A % TIE_P;
  return m;
}

static uint64_t tie_rank(int32_t c, uint64_t mult) { return ((uint64_t)c + 1) % TIE_P * mult % TIE_P; }

/* MurmurHash3 32-bit finaliser (Appleby, public domain). */
static uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

static int weights_ok(int64_t m, const float *w) {
  if (!w) return 1;
  for (int64_t e = 0; e < m; ++e) {
    float x = w[e];
    if (!(x >= 0.0f) || x > 16777216.0f || (float)(uint32_t)x != x) return 0;
  }
  return 1;
}

/*
 * oracle_lpa: strict LPA in the vertex order `order` (NULL = 0..n-1).
 *
 * init_labels / init_flags (NULL = identity labels / all flagged) allow a run
 * to resume from a snapshot.  Outputs: labels[n], flags[n] (final flags; may
 * be NULL), and per sweep s < ORACLE_MAX_STATS: changed[s] (dN), processed[s]
 * (flagged vertices visited that have at least one stored entry) and
 * scanned[s] (stored entries of those vertices).  *iterations = number of
 * lpaMove calls executed; *converged = 1 when the stop test held.
 * nonstrict = 0: ties go to the smallest label id (strict LPA); 1: to the
 * smallest rank r_v (non-strict LPA, above).
 * Returns 0, or -1 for invalid arguments, -3 for non-integral weights.
 */
int oracle_lpa(int64_t n, const int64_t *off, const int32_t *idx, const float *w, const int32_t *order,
               double tau, int max_iters, int prune, const int32_t *init_labels, const uint8_t *init_flags,
               int32_t *labels, uint8_t *flags_out, int64_t *changed, int64_t *processed, int64_t *scanned,
               int32_t *iterations, int32_t *converged, int nonstrict) {
  if (n < 0 || !off || (off[n] > 0 && !idx) || !labels || max_iters < 0) return -1;
  const int64_t m = off[n];
  if (!weights_ok(m, w)) return -3;

  int32_t *C = labels;
  uint8_t *F = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  uint64_t *acc = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  uint8_t *seen = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
  int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!F || !acc || !seen || !touched) {
    free(F); free(acc); free(seen); free(touched);
    return -1;
  }
  /* C <- [0 .. |V|); every vertex starts unprocessed (flagged). */
  for (int64_t v = 0; v < n; ++v) {
    C[v] = init_labels ? init_labels[v] : (int32_t)v;
    F[v] = init_flags ? (init_flags[v] != 0) : 1;
  }
  int32_t it_done = 0, conv = 0;
  for (int it = 0; it < max_iters; ++it) {
    int64_t dN = 0, nproc = 0, nscan = 0;
    /* lpaMove: visit vertices in order; sequential and in place. */
    for (int64_t p = 0; p < n; ++p) {
      const int64_t v = order ? order[p] : p;
      if (prune && !F[v]) continue;
      F[v] = 0; /* mark v processed before its scan */
      const int64_t b = off[v], e = off[v + 1];
      if (e > b) {
        nproc += 1;
        nscan += e - b;
      }
      /* scanCommunities: total weight of every neighbour label, self excluded. */
      int64_t nt = 0;
      for (int64_t k = b; k < e; ++k) {
        const int32_t j = idx[k];
        if (j == v) continue;
        const int32_t c = C[j];
        if (!seen[c]) {
          seen[c] = 1;
          acc[c] = 0;
          touched[nt++] = c;
        }
        acc[c] += w ? (uint64_t)w[k] : 1u;
      }
      if (nt == 0) continue; /* no neighbour other than itself: keep the label */
      /* most weighted label; among equals the smallest id (strict) or rank */
      const uint64_t mult = nonstrict ? tie_mult(v) : 0;
      int32_t best = touched[0];
      for (int64_t t = 1; t < nt; ++t) {
        const int32_t c = touched[t];
        const int smaller = nonstrict ? tie_rank(c, mult) < tie_rank(best, mult) : c < best;
        if (acc[c] > acc[best] || (acc[c] == acc[best] && smaller)) best = c;
      }
      for (int64_t t = 0; t < nt; ++t) seen[touched[t]] = 0;
      if (best == C[v]) continue;
      C[v] = best;
      dN += 1;
      if (prune) /* mark the neighbours of v (not v itself) for processing */
        for (int64_t k = b; k < e; ++k)
          if (idx[k] != v) F[idx[k]] = 1;
    }
    if (it < ORACLE_MAX_STATS) {
      if (changed) changed[it] = dN;
      if (processed) processed[it] = nproc;
      if (scanned) scanned[it] = nscan;
    }
    it_done = it + 1;
    if ((double)dN / (double)(n > 0 ? n : 1) <= tau) {
      conv = 1;
      break;
    }
  }
  if (flags_out) memcpy(flags_out, F, (size_t)n);
  if (iterations) *iterations = it_done;
  if (converged) *converged = conv;
  free(F); free(acc); free(seen); free(touched);
  return 0;
}

/* Priority of v: (deg(v), fmix32(v ^ seed), v) compared lexicographically,
 * deg(v) = stored entries of row v; larger is coloured first. */
typedef struct {
  uint64_t key; /* deg << 32 | fmix32(v ^ seed) */
  uint32_t v;
} prio_t;

static int cmp_desc(const void *a, const void *b) {
  const prio_t *x = (const prio_t *)a, *y = (const prio_t *)b;
  if (x->key != y->key) return x->key < y->key ? 1 : -1;
  return x->v < y->v ? 1 : (x->v > y->v ? -1 : 0);
}

/*
 * oracle_color: greedy colouring; vertices taken in decreasing priority, each
 * gets the smallest colour not used by an already coloured neighbour.
 * Self-loops are ignored.  Writes colors[n]; returns the number of colours,
 * or -1 on allocation failure.
 */
int64_t oracle_color(int64_t n, const int64_t *off, const int32_t *idx, uint32_t seed, int32_t *colors) {
  prio_t *keys = (prio_t *)malloc(sizeof(prio_t) * (size_t)(n > 0 ? n : 1));
  int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 2));
  if (!keys || !stamp) {
    free(keys); free(stamp);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) {
    const uint64_t deg = (uint64_t)(off[v + 1] - off[v]);
    keys[v].key = (deg << 32) | fmix32((uint32_t)v ^ seed);
    keys[v].v = (uint32_t)v;
    colors[v] = -1;
  }
  for (int64_t c = 0; c < n + 2; ++c) stamp[c] = -1;
  qsort(keys, (size_t)n, sizeof(prio_t), cmp_desc);
  int64_t ncol = 0;
  for (int64_t p = 0; p < n; ++p) {
    const int64_t v = (int64_t)keys[p].v;
    for (int64_t k = off[v]; k < off[v + 1]; ++k) {
      const int32_t j = idx[k];
      if (j != v && colors[j] >= 0) stamp[colors[j]] = v;
    }
    int32_t c = 0;
    while (stamp[c] == v) ++c;
    colors[v] = c;
    if (c + 1 > ncol) ncol = c + 1;
  }
  free(keys); free(stamp);
  return ncol;
}

/* Vertex order sorted by (colour, id): the order the deterministic mode follows. */
int oracle_color_order(int64_t n, const int32_t *colors, int64_t ncol, int32_t *order) {
  int64_t *start = (int64_t *)calloc((size_t)(ncol + 1), sizeof(int64_t));
  if (!start) return -1;
  for (int64_t v = 0; v < n; ++v) start[colors[v] + 1] += 1;
  for (int64_t c = 0; c < ncol; ++c) start[c + 1] += start[c];
  for (int64_t v = 0; v < n; ++v) order[start[colors[v]]++] = (int32_t)v;
  free(start);
  return 0;
}

/*
 * oracle_modularity: Eq. (1), community form (Section 3.2).  With K_i the sum of the stored
 * weights of row i (self-loop entries included, counted once), 2m = sum_i K_i,
 * sigma_c = stored weight with both ends in c, Sigma_c = sum_{i in c} K_i:
 *   Q = (S1 * 2m - S2) / (2m)^2,  S1 = sum_c sigma_c,  S2 = sum_c Sigma_c^2,
 * all in exact integers; numerator and denominator are each rounded to double
 * once and divided once.  Labels must lie in [0, n).  Returns 0, -1 on bad
 * labels, -3 on non-integral weights.  An edgeless graph gives Q = 0.
 */
int oracle_modularity(int64_t n, const int64_t *off, const int32_t *idx, const float *w, const int32_t *labels,
                      double *q_out) {
  const int64_t m = off[n];
  if (!weights_ok(m, w)) return -3;
  for (int64_t v = 0; v < n; ++v)
    if (labels[v] < 0 || labels[v] >= n) return -1;
  unsigned __int128 *tot = (unsigned __int128 *)calloc((size_t)(n > 0 ? n : 1), sizeof(unsigned __int128));
  if (!tot) return -1;
  unsigned __int128 two_m = 0, s1 = 0, s2 = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = off[i]; k < off[i + 1]; ++k) {
      const uint64_t x = w ? (uint64_t)w[k] : 1u;
      two_m += x;
      tot[labels[i]] += x;
      if (labels[idx[k]] == labels[i]) s1 += x;
    }
  }
  for (int64_t c = 0; c < n; ++c) s2 += tot[c] * tot[c];
  free(tot);
  if (two_m == 0) {
    *q_out = 0.0;
    return 0;
  }
  const __int128 num = (__int128)(s1 * two_m) - (__int128)s2;
  const unsigned __int128 den = two_m * two_m;
  *q_out = (double)num / (double)den;
  return 0;
}
