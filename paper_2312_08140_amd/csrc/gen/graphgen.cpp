// Seeded synthetic graph generators: R-MAT, stochastic block model (SBM), a
// batch of uneven SBMs laid out block-diagonally, and a sparse road-like
// lattice (low average degree).
//
// This module only builds inputs.  It holds none of the label-propagation
// arithmetic, and both the sequential oracle and the GPU library consume the
// CSR arrays it produces.  Every random draw is counter based, so a graph is a
// pure function of its parameters and seed, independent of the thread count.
//
// Random numbers: the SplitMix64 output function (Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
// key + (counter + 1) * 0x9E3779B97F4A7C15.
//
// Output CSR: undirected, every edge stored in both directions, no self-loops,
// no duplicate entries, rows sorted by neighbour id; int64 offsets, int32
// indices, fp32 weights holding small integers.  Arrays are obtained through a
// caller-supplied allocator so that the caller (numpy) owns them.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline uint64_t draw(uint64_t key, uint64_t ctr) { return mix64(key + (ctr + 1) * kGamma); }
inline double unit_double(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
inline uint64_t stream_key(uint64_t seed, uint64_t stream) { return mix64(seed * kGamma + stream * 0xD1B54A32D192ED03ull); }

// Symmetric edge weight in 1..8 from the unordered pair.
inline float pair_weight(uint64_t wkey, uint32_t u, uint32_t v) {
  uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
  return (float)(1 + (mix64(wkey ^ (((uint64_t)lo << 32) | hi)) & 7));
}

typedef void *(*alloc_fn)(int kind, int64_t count);  // kind: 0 offsets i64, 1 indices i32, 2 weights f32

// Edge source: a callable emit(e, u, v) producing directed pair (u, v) for edge e
// (returns false when the edge is dropped).  Builds the symmetrised CSR in
// four passes: count, scatter, per-row sort+dedupe, compact.
template <class Src>
int build_csr(int64_t n, int64_t n_edges, Src src, int weighted, uint64_t wkey, alloc_fn alloc,
              int64_t *m_out) {
  // builds of over 2^30 edges report each pass on stderr (they take minutes)
  const bool verbose = n_edges > ((int64_t)1 << 30);
  auto pass_done = [&](const char *what) {
    if (verbose) std::fprintf(stderr, "graphgen: %s done (%lld edges)\n", what, (long long)n_edges);
  };
  std::vector<int64_t> deg(n + 1, 0);
  // pass 1: degree count (each kept edge contributes to both endpoints)
#pragma omp parallel for schedule(static, 1 << 16)
  for (int64_t e = 0; e < n_edges; ++e) {
    uint32_t u, v;
    if (!src(e, u, v)) continue;
    __atomic_fetch_add(&deg[u], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&deg[v], 1, __ATOMIC_RELAXED);
  }
  pass_done("degree count");
  std::vector<int64_t> off0(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) off0[i + 1] = off0[i] + deg[i];
  int64_t total = off0[n];
  std::vector<int32_t> scratch((size_t)total);
  std::fill(deg.begin(), deg.end(), 0);
  // pass 2: scatter both directions
#pragma omp parallel for schedule(static, 1 << 16)
  for (int64_t e = 0; e < n_edges; ++e) {
    uint32_t u, v;
    if (!src(e, u, v)) continue;
    int64_t pu = off0[u] + __atomic_fetch_add(&deg[u], 1, __ATOMIC_RELAXED);
    int64_t pv = off0[v] + __atomic_fetch_add(&deg[v], 1, __ATOMIC_RELAXED);
    scratch[pu] = (int32_t)v;
    scratch[pv] = (int32_t)u;
  }
  pass_done("scatter");
  // pass 3: sort and dedupe every row in place
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    int32_t *b = scratch.data() + off0[i], *e = scratch.data() + off0[i + 1];
    std::sort(b, e);
    deg[i] = std::unique(b, e) - b;
  }
  pass_done("row sort and dedupe");
  int64_t *off = (int64_t *)alloc(0, n + 1);
  if (!off) return -1;
  off[0] = 0;
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg[i];
  int64_t m = off[n];
  int32_t *idx = (int32_t *)alloc(1, m);
  if (!idx && m) return -1;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i)
    if (deg[i]) std::memcpy(idx + off[i], scratch.data() + off0[i], sizeof(int32_t) * deg[i]);
  std::vector<int32_t>().swap(scratch);
  if (weighted >= 0) {
    float *w = (float *)alloc(2, m);
    if (!w && m) return -1;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = off[i]; e < off[i + 1]; ++e)
        w[e] = weighted ? pair_weight(wkey, (uint32_t)i, (uint32_t)idx[e]) : 1.0f;
  }
  *m_out = m;
  return 0;
}

// SBM block layout: contiguous id ranges, sizes as equal as possible.
struct Blocks {
  int64_t n, k;
  int64_t size(int64_t b) const { return n / k + (b < n % k ? 1 : 0); }
  int64_t start(int64_t b) const { return b * (n / k) + std::min(b, n % k); }
};

// Enumerate the edges of one SBM on vertex ids [base, base + n) into `out`.
// direct = 1: one Bernoulli draw per candidate pair (exact, integer threshold).
// direct = 0: geometric skipping over candidate pairs (Batagelj and Brandes,
// "Efficient generation of large random networks", Phys. Rev. E 71, 2005).
void sbm_edges(int64_t n, int64_t k, double p_in, double p_out, uint64_t seed, int direct, uint32_t base,
               std::vector<uint64_t> &out) {
  Blocks B{n, k};
  for (int64_t bi = 0; bi < k; ++bi) {
    for (int64_t bj = bi; bj < k; ++bj) {
      const double p = (bi == bj) ? p_in : p_out;
      if (p <= 0.0) continue;
      const int64_t si = B.size(bi), sj = B.size(bj), oi = B.start(bi), oj = B.start(bj);
      const int64_t cand = (bi == bj) ? si * (si - 1) / 2 : si * sj;
      if (cand == 0) continue;
      const uint64_t key = stream_key(seed, (uint64_t)bi * (uint64_t)k + (uint64_t)bj + 1);
      auto decode = [&](int64_t t, uint32_t &u, uint32_t &v) {
        if (bi != bj) {
          u = (uint32_t)(oi + t / sj);
          v = (uint32_t)(oj + t % sj);
        } else {  // t indexes pairs (r, c), r < c, row-major over the upper triangle
          int64_t r = (int64_t)((2.0 * si - 1 - std::sqrt((2.0 * si - 1) * (2.0 * si - 1) - 8.0 * (double)t)) / 2);
          if (r < 0) r = 0;
          auto row_start = [&](int64_t rr) { return rr * (2 * si - rr - 1) / 2; };
          while (r > 0 && row_start(r) > t) --r;
          while (row_start(r + 1) <= t) ++r;
          int64_t c = r + 1 + (t - row_start(r));
          u = (uint32_t)(oi + r);
          v = (uint32_t)(oi + c);
        }
      };
      if (direct || p >= 1.0) {
        const uint64_t thr = p >= 1.0 ? (1ull << 32) : (uint64_t)std::llround(p * 4294967296.0);
        for (int64_t t = 0; t < cand; ++t) {
          if ((draw(key, (uint64_t)t) >> 32) < thr) {
            uint32_t u, v;
            decode(t, u, v);
            out.push_back(((uint64_t)(u + base) << 32) | (uint64_t)(v + base));
          }
        }
      } else {
        const double lq = std::log1p(-p);
        int64_t t = -1;
        uint64_t ctr = 0;
        for (;;) {
          double r = unit_double(draw(key, ctr++));
          double skip = std::floor(std::log1p(-r) / lq);
          if (!(skip < (double)cand)) break;
          t += 1 + (int64_t)skip;
          if (t >= cand) break;
          uint32_t u, v;
          decode(t, u, v);
          out.push_back(((uint64_t)(u + base) << 32) | (uint64_t)(v + base));
        }
      }
    }
  }
}

}  // namespace

extern "C" {

// R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004) without noise and without
// vertex permutation: 2^scale vertices, edge_factor * 2^scale generated edges,
// two recursion levels per 64-bit draw (32-bit uniforms per level).
int gg_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed, int weighted,
            alloc_fn alloc, int64_t *n_out, int64_t *m_out) {
  if (scale < 1 || scale > 30 || edge_factor < 1 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -2;
  const int64_t n = (int64_t)1 << scale;
  const int64_t n_edges = (int64_t)edge_factor << scale;
  const uint64_t ta = (uint64_t)std::llround(a * 4294967296.0);
  const uint64_t tb = (uint64_t)std::llround((a + b) * 4294967296.0);
  const uint64_t tc = (uint64_t)std::llround((a + b + c) * 4294967296.0);
  const uint64_t key = stream_key(seed, 0x524D4154ull);
  const int draws_per_edge = (scale + 1) / 2;
  auto src = [&](int64_t e, uint32_t &u, uint32_t &v) -> bool {
    uint32_t su = 0, sv = 0;
    uint64_t x = 0;
    for (int l = 0; l < scale; ++l) {
      if ((l & 1) == 0) x = draw(key, (uint64_t)e * draws_per_edge + (l >> 1));
      uint64_t r = (l & 1) ? (x & 0xFFFFFFFFull) : (x >> 32);
      uint32_t bit = 1u << (scale - 1 - l);
      if (r < ta) {
      } else if (r < tb) {
        sv |= bit;
      } else if (r < tc) {
        su |= bit;
      } else {
        su |= bit;
        sv |= bit;
      }
    }
    u = su;
    v = sv;
    return u != v;
  };
  *n_out = n;
  return build_csr(n, n_edges, src, weighted, stream_key(seed, 0x57454947ull), alloc, m_out);
}

// Planted-partition SBM on n vertices in k contiguous blocks.
int gg_sbm(int64_t n, int64_t k, double p_in, double p_out, uint64_t seed, int weighted, int direct, alloc_fn alloc,
           int64_t *m_out) {
  if (n < 1 || n >= ((int64_t)1 << 31) || k < 1 || k > n || p_in < 0 || p_in > 1 || p_out < 0 || p_out > 1) return -2;
  std::vector<uint64_t> edges;
  sbm_edges(n, k, p_in, p_out, seed, direct, 0, edges);
  auto src = [&](int64_t e, uint32_t &u, uint32_t &v) -> bool {
    u = (uint32_t)(edges[e] >> 32);
    v = (uint32_t)edges[e];
    return true;
  };
  return build_csr(n, (int64_t)edges.size(), src, weighted, stream_key(seed, 0x57454947ull), alloc, m_out);
}

// Per-graph parameters of the uneven SBM batch, drawn from the master seed:
// n_g = round(exp(U[ln n_lo, ln n_hi])), k_g = max(1, floor(n_g / 100)),
// d_g ~ U[d_lo, d_hi], mu_g ~ U[mu_lo, mu_hi], s = n_g / k_g,
// p_in = d (1 - mu) / (s - 1), p_out = d mu / (n - s)  (both clipped to [0, 1]).
int gg_sbm_batch_params(int32_t count, uint64_t master_seed, double n_lo, double n_hi, double d_lo, double d_hi,
                        double mu_lo, double mu_hi, int64_t *n_g, int64_t *k_g, double *p_in, double *p_out) {
  if (count < 1 || n_lo < 2 || n_hi < n_lo) return -2;
  const uint64_t key = stream_key(master_seed, 0x42415443ull);
  for (int32_t g = 0; g < count; ++g) {
    double u0 = unit_double(draw(key, 3 * (uint64_t)g + 0));
    double u1 = unit_double(draw(key, 3 * (uint64_t)g + 1));
    double u2 = unit_double(draw(key, 3 * (uint64_t)g + 2));
    int64_t n = (int64_t)std::llround(std::exp(std::log(n_lo) + u0 * (std::log(n_hi) - std::log(n_lo))));
    int64_t k = std::max<int64_t>(1, n / 100);
    double d = d_lo + u1 * (d_hi - d_lo);
    double mu = mu_lo + u2 * (mu_hi - mu_lo);
    double s = (double)n / (double)k;
    double pi = s > 1 ? d * (1 - mu) / (s - 1) : 0.0;
    double po = (n - s) > 0 ? d * mu / ((double)n - s) : 0.0;
    n_g[g] = n;
    k_g[g] = k;
    p_in[g] = std::min(1.0, std::max(0.0, pi));
    p_out[g] = std::min(1.0, std::max(0.0, po));
  }
  return 0;
}

// Block-diagonal union of `count` SBMs (graph g uses seed seed_base + g);
// graph_vptr[g] is the first global vertex id of graph g, graph_vptr[count] = N.
int gg_sbm_batch(int32_t count, const int64_t *n_g, const int64_t *k_g, const double *p_in, const double *p_out,
                 uint64_t seed_base, int weighted, alloc_fn alloc, int64_t *graph_vptr, int64_t *n_out,
                 int64_t *m_out) {
  graph_vptr[0] = 0;
  for (int32_t g = 0; g < count; ++g) graph_vptr[g + 1] = graph_vptr[g] + n_g[g];
  const int64_t n = graph_vptr[count];
  if (n >= ((int64_t)1 << 31)) return -2;
  std::vector<std::vector<uint64_t>> per(count);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t g = 0; g < count; ++g)
    sbm_edges(n_g[g], k_g[g], p_in[g], p_out[g], seed_base + (uint64_t)g, 0, (uint32_t)graph_vptr[g], per[g]);
  std::vector<int64_t> eoff(count + 1, 0);
  for (int32_t g = 0; g < count; ++g) eoff[g + 1] = eoff[g] + (int64_t)per[g].size();
  std::vector<uint64_t> edges((size_t)eoff[count]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t g = 0; g < count; ++g) {
    std::copy(per[g].begin(), per[g].end(), edges.begin() + eoff[g]);
    std::vector<uint64_t>().swap(per[g]);
  }
  auto src = [&](int64_t e, uint32_t &u, uint32_t &v) -> bool {
    u = (uint32_t)(edges[e] >> 32);
    v = (uint32_t)edges[e];
    return true;
  };
  *n_out = n;
  return build_csr(n, (int64_t)edges.size(), src, weighted, stream_key(seed_base, 0x57454947ull), alloc, m_out);
}

// Low-degree, road-like graph: the 4-neighbour lattice of rows x cols
// vertices (row-major ids), each lattice edge kept with probability p_keep
// (one counter-based draw per candidate edge: horizontal ones first, then
// vertical).  With p_keep = 0.55 the average degree is about 2.2, the order
// of the road and k-mer graphs of the paper's dataset.
int gg_grid(int64_t rows, int64_t cols, double p_keep, uint64_t seed, int weighted, alloc_fn alloc, int64_t *n_out,
            int64_t *m_out) {
  if (rows < 1 || cols < 1 || rows * cols >= ((int64_t)1 << 31) || !(p_keep >= 0.0) || p_keep > 1.0) return -2;
  const int64_t n = rows * cols;
  const int64_t nh = rows * (cols - 1), nv = (rows - 1) * cols;
  const uint64_t thr = p_keep >= 1.0 ? (1ull << 32) : (uint64_t)std::llround(p_keep * 4294967296.0);
  const uint64_t key = stream_key(seed, 0x47524944ull);
  auto src = [&](int64_t e, uint32_t &u, uint32_t &v) -> bool {
    if ((draw(key, (uint64_t)e) >> 32) >= thr) return false;
    if (e < nh) {
      const int64_t r = e / (cols - 1), c = e % (cols - 1);
      u = (uint32_t)(r * cols + c);
      v = u + 1;
    } else {
      const int64_t f = e - nh;
      u = (uint32_t)f;
      v = (uint32_t)(f + cols);
    }
    return true;
  };
  *n_out = n;
  return build_csr(n, nh + nv, src, weighted, stream_key(seed, 0x57454947ull), alloc, m_out);
}

int gg_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
