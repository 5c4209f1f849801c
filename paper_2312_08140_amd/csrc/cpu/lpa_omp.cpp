// Multicore CPU label propagation in the paper's own design (host only; the
// comparator the GPU library is measured against).  See include/gvelpa_cpu.h.
//
// Algorithm 1 (Section 4.2) on OpenMP threads: a dynamic schedule of chunk
// 2048 over the vertices (Section 4.1.1), asynchronous in-place labels
// (Section 4.1), 8-bit pruning flags (Section 4.1.4), per-thread Far-KV
// tables (Section 4.1.6), a reduction for dN and the dN/N <= tau stop test
// (Sections 4.1.2-4.1.3).  Labels and flags are shared between threads and
// read/written with relaxed atomics: any interleaving is a valid
// asynchronous run.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gvelpa_cpu.h"

namespace {

// Non-strict tie rule (gvelpa.h, LPA_FLAG_NONSTRICT): among the heaviest
// labels vertex v takes the smallest ((c + 1) * A^(1 + v mod 64)) mod P.
constexpr uint64_t TIE_P = 2147483647ull;
constexpr uint64_t TIE_A = 1580030173ull;

// Far-KV table of one thread: values indexed by label (one slot per vertex;
// a slot holds 1 + the summed weight while its label is in use) and the list
// of labels in use.  Allocated by its own thread, apart from the others.
struct FarKV {
  uint64_t *val = nullptr;
  int32_t *keys = nullptr;
};

inline int32_t load_i32(const int32_t *p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
inline void store_i32(int32_t *p, int32_t x) { __atomic_store_n(p, x, __ATOMIC_RELAXED); }
inline uint8_t load_u8(const uint8_t *p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }
inline void store_u8(uint8_t *p, uint8_t x) { __atomic_store_n(p, x, __ATOMIC_RELAXED); }

bool valid_csr(int64_t n, const int64_t *off, const int32_t *idx, const float *w) {
  if (off[0] != 0) return false;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t v = 0; v < n; ++v) {
    if (off[v + 1] < off[v]) {
      bad = 1;
      continue;
    }
    uint64_t deg = 0;
    for (int64_t k = off[v]; k < off[v + 1]; ++k) {
      if (idx[k] < 0 || (int64_t)idx[k] >= n) bad = 1;
      if (w) {
        const float x = w[k];
        if (!(x >= 0.0f) || x > 16777216.0f || std::floor(x) != x) bad = 1;
        else deg += (uint64_t)x;
      } else {
        deg += 1;
      }
    }
    if (deg >= (1ull << 32)) bad = 1;
  }
  return !bad;
}

}  // namespace

extern "C" {

int gvcpu_max_threads(void) { return omp_get_max_threads(); }

int gvcpu_lpa(int64_t n, const int64_t *off, const int32_t *idx, const float *w, double tau, int max_iters,
              int prune, int nonstrict, int threads, int32_t *labels, int64_t *changed, int64_t *processed,
              int64_t *scanned, int32_t *iterations, int32_t *converged, double *seconds) {
  if (n < 0 || n >= ((int64_t)1 << 31) || !off || !labels || max_iters < 0 || max_iters > 1000 ||
      (off[n] > 0 && !idx) || tau != tau)
    return -1;
  if (!valid_csr(n, off, idx, w)) return -1;
  const int nt = threads > 0 ? threads : omp_get_max_threads();
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) maxdeg = std::max<int64_t>(maxdeg, off[v + 1] - off[v]);
  uint64_t mult[64];
  {
    uint64_t m = 1;
    for (int k = 0; k < 64; ++k) mult[k] = m = m * TIE_A % TIE_P;
  }
  std::vector<uint8_t> flags((size_t)std::max<int64_t>(n, 1), 1);
  uint8_t *F = flags.data();
  int32_t *C = labels;
  for (int64_t v = 0; v < n; ++v) C[v] = (int32_t)v;
  // one Far-KV table per thread, allocated (and first touched) by that thread
  std::vector<FarKV> tab((size_t)nt);
  int oom = 0;
#pragma omp parallel num_threads(nt) reduction(| : oom)
  {
    FarKV &h = tab[(size_t)omp_get_thread_num()];
    h.val = (uint64_t *)std::calloc((size_t)std::max<int64_t>(n, 1), sizeof(uint64_t));
    h.keys = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(maxdeg, 1));
    if (!h.val || !h.keys) oom = 1;
  }
  for (FarKV &h : tab)  // a thread the first region did not get
    if (!h.val && !oom) {
      h.val = (uint64_t *)std::calloc((size_t)std::max<int64_t>(n, 1), sizeof(uint64_t));
      h.keys = (int32_t *)std::malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(maxdeg, 1));
      if (!h.val || !h.keys) oom = 1;
    }
  auto release = [&]() {
    for (FarKV &h : tab) {
      std::free(h.val);
      std::free(h.keys);
    }
  };
  if (oom) {
    release();
    return -2;
  }
  const double t0 = omp_get_wtime();
  int32_t done = 0, conv = 0;
  for (int it = 0; it < max_iters; ++it) {
    int64_t dn = 0, np = 0, ns = 0;
#pragma omp parallel num_threads(nt) reduction(+ : dn, np, ns)
    {
      FarKV &h = tab[(size_t)omp_get_thread_num()];
#pragma omp for schedule(dynamic, 2048)
      for (int64_t v = 0; v < n; ++v) {
        if (prune && !load_u8(&F[v])) continue;
        store_u8(&F[v], 0);  // processed before its scan
        const int64_t b = off[v], e = off[v + 1];
        if (e > b) {
          np += 1;
          ns += e - b;
        }
        // scanCommunities: summed weight per neighbour label, the vertex itself skipped
        int64_t nk = 0;
        for (int64_t k = b; k < e; ++k) {
          const int32_t j = idx[k];
          if (j == v) continue;
          const int32_t c = load_i32(&C[j]);
          if (!h.val[c]) {
            h.keys[nk++] = c;
            h.val[c] = 1;
          }
          h.val[c] += w ? (uint64_t)w[k] : 1u;
        }
        if (!nk) continue;  // no neighbour besides itself: the label stays
        int32_t best = h.keys[0];
        const uint64_t mv = mult[v & 63];
        for (int64_t t = 1; t < nk; ++t) {
          const int32_t c = h.keys[t];
          bool better = h.val[c] > h.val[best];
          if (!better && h.val[c] == h.val[best])
            better = nonstrict ? ((uint64_t)c + 1) % TIE_P * mv % TIE_P < ((uint64_t)best + 1) % TIE_P * mv % TIE_P
                               : c < best;
          if (better) best = c;
        }
        for (int64_t t = 0; t < nk; ++t) h.val[h.keys[t]] = 0;
        if (best == load_i32(&C[v])) continue;
        store_i32(&C[v], best);
        dn += 1;
        if (prune)
          for (int64_t k = b; k < e; ++k)
            if (idx[k] != v) store_u8(&F[idx[k]], 1);
      }
    }
    if (changed) changed[it] = dn;
    if (processed) processed[it] = np;
    if (scanned) scanned[it] = ns;
    done = it + 1;
    if ((double)dn / (double)(n > 0 ? n : 1) <= tau) {
      conv = 1;
      break;
    }
  }
  if (seconds) *seconds = omp_get_wtime() - t0;
  if (iterations) *iterations = done;
  if (converged) *converged = conv;
  release();
  return 0;
}

}  // extern "C"
