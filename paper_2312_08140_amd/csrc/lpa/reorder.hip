// Storage order of the vertices.  The library keeps vertices in decreasing
// degree order (within each graph of a batch), so that the labels gathered
// most often - those of high-degree vertices - share cache lines.  Labels keep
// their values (original vertex ids), so the method's results do not change;
// only positions do: position p holds original vertex order[p], and original
// vertex v sits at position pos[v].
#include <hipcub/hipcub.hpp>

#include "sweep_kernels.hpp"

namespace gvelpa {

// key = graph << 32 | (0xFFFFFFFF - degree): ascending key = by graph, then by
// decreasing degree; the radix sort is stable, so ties keep id order.
__global__ void k_order_keys(const int64_t *off, const int32_t *gid, int64_t n, u64 *key, int32_t *val) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const u64 deg = (u64)(off[v + 1] - off[v]);
    const u64 g = gid ? (u64)(uint32_t)gid[v] : 0ull;
    key[v] = (g << 32) | (0xFFFFFFFFull - (deg < 0xFFFFFFFFull ? deg : 0xFFFFFFFFull));
    val[v] = (int32_t)v;
  }
}

__global__ void k_inverse(const int32_t *order, int64_t n, int32_t *pos, int64_t *ndeg, const int64_t *off) {
  if (blockIdx.x == 0 && threadIdx.x == 0) ndeg[n] = 0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = order[p];
    pos[v] = (int32_t)p;
    ndeg[p] = off[v + 1] - off[v];
  }
}

// New row p = old row order[p], neighbours renamed to positions; one wave per row.
template <int WK>
__global__ __launch_bounds__(256) void k_permute_rows(const int64_t *off, const int32_t *idx, const void *w,
                                                      const int32_t *order, const int32_t *pos, const int64_t *noff,
                                                      int32_t *nidx, void *nw, int64_t n) {
  const int lane = threadIdx.x & 63;
  for (int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < n; p += (int64_t)gridDim.x * 4) {
    const int32_t v = order[p];
    const int64_t b = off[v], e = off[v + 1], nb = noff[p];
    for (int64_t k = b + lane; k < e; k += 64) {
      nidx[nb + (k - b)] = pos[idx[k]];
      if constexpr (WK == W_U8) ((uint8_t *)nw)[nb + (k - b)] = ((const uint8_t *)w)[k];
      if constexpr (WK == W_U32) ((uint32_t *)nw)[nb + (k - b)] = ((const uint32_t *)w)[k];
    }
  }
}

template <class T>
__global__ void k_gather(T *dst, const T *src, const int32_t *index, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[index[i]];
}

static int grid(int64_t n, int per, int cap = 16384) {
  int64_t b = (n + per - 1) / per;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// bytes of temporary storage the sort and the scan of build_order need
int64_t order_temp_bytes(int64_t n) {
  size_t sort_bytes = 0, scan_bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (u64 *)nullptr, (u64 *)nullptr, (int32_t *)nullptr,
                                           (int32_t *)nullptr, (int)n, 0, 64);
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int64_t *)nullptr, (int64_t *)nullptr, (int)(n + 1));
  return (int64_t)std::max(sort_bytes, scan_bytes);
}

// keys: 2n + 1 u64 of scratch (sort keys in; sort keys out, later the
// permuted degrees); temp: order_temp_bytes(n) bytes (separately allocated,
// so it has the alignment of an allocation)
hipError_t build_order(const int64_t *off, const int32_t *gid, int64_t n, int32_t *order, int32_t *pos,
                       int64_t *noff, u64 *keys, void *temp, int64_t temp_bytes, hipStream_t st) {
  u64 *kin = keys, *kout = keys + n;
  int64_t *deg = (int64_t *)kout;  // reused once the sorted keys are no longer needed
  int32_t *vin = pos;              // pos is written only after the sort
  size_t tb = (size_t)temp_bytes;
  hipLaunchKernelGGL(k_order_keys, dim3(grid(n, 256)), dim3(256), 0, st, off, gid, n, kin, vin);
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, tb, kin, kout, vin, order, (int)n, 0, 64, st);
  if (e != hipSuccess) return e;
  // noff[0 .. n] = exclusive prefix sum of the permuted degrees (noff[n] = m)
  hipLaunchKernelGGL(k_inverse, dim3(grid(n, 256)), dim3(256), 0, st, order, n, pos, deg, off);
  tb = (size_t)temp_bytes;
  return hipcub::DeviceScan::ExclusiveSum(temp, tb, deg, noff, (int)(n + 1), st);
}

void launch_permute_rows(const int64_t *off, const int32_t *idx, const void *w, int wk, const int32_t *order,
                         const int32_t *pos, const int64_t *noff, int32_t *nidx, void *nw, int64_t n,
                         hipStream_t st) {
  const dim3 g(grid(n, 4)), b(256);
  if (wk == W_U8) hipLaunchKernelGGL(k_permute_rows<W_U8>, g, b, 0, st, off, idx, w, order, pos, noff, nidx, nw, n);
  else if (wk == W_U32)
    hipLaunchKernelGGL(k_permute_rows<W_U32>, g, b, 0, st, off, idx, w, order, pos, noff, nidx, nw, n);
  else hipLaunchKernelGGL(k_permute_rows<W_UNIT>, g, b, 0, st, off, idx, w, order, pos, noff, nidx, nw, n);
}

// ---------------------------------------------------------------- sorted rows
//
// After the renaming, the entries of a row are sorted by neighbour position
// (with their weights), so a row's gathers walk the label array in order and
// neighbours that share a cache line are read together.  Rows [r0, r1) with
// their entries [off[r0], off[r1)) are sorted at once by the key
// (row - r0) << 32 | neighbour, in chunks of at most 2^30 entries.

__global__ void k_row_keys(const int64_t *off, const int32_t *idx, int64_t r0, int64_t r1, u64 *key) {
  const int lane = threadIdx.x & 63;
  const int64_t base = off[r0];
  for (int64_t r = r0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < r1; r += (int64_t)gridDim.x * 4)
    for (int64_t k = off[r] + lane; k < off[r + 1]; k += 64)
      key[k - base] = ((u64)(r - r0) << 32) | (uint32_t)idx[k];
}

__global__ void k_iota(int32_t *v, int64_t len) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (int32_t)i;
}

// idx[base + i] = low half of key[i]; weights follow their entries (perm[i] = old slot)
template <int WK>
__global__ void k_row_store(const u64 *key, const int32_t *perm, int64_t len, int64_t base, int32_t *idx,
                            const void *wsrc, void *w) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    idx[base + i] = (int32_t)(uint32_t)key[i];
    if constexpr (WK == W_U8) ((uint8_t *)w)[base + i] = ((const uint8_t *)wsrc)[perm[i]];
    if constexpr (WK == W_U32) ((uint32_t *)w)[base + i] = ((const uint32_t *)wsrc)[perm[i]];
  }
}

int64_t row_sort_temp_bytes(int64_t chunk) {
  size_t b1 = 0, b2 = 0;
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, b1, (u64 *)nullptr, (u64 *)nullptr, (int)chunk, 0, 64);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b2, (u64 *)nullptr, (u64 *)nullptr, (int32_t *)nullptr,
                                           (int32_t *)nullptr, (int)chunk, 0, 64);
  return (int64_t)std::max(b1, b2);
}

// Sorts the rows [r0, r1) (their entries fit a chunk).  keys: 2 * len u64;
// perm: 2 * len int32 (weighted rows only); wcopy: the chunk's weights (weighted only).
hipError_t sort_rows_chunk(const int64_t *off, int64_t r0, int64_t r1, int64_t e0, int64_t len, int32_t *idx,
                           void *w, int wk, u64 *keys, int32_t *perm, void *wcopy, void *temp, int64_t temp_bytes,
                           hipStream_t st) {
  if (len <= 0) return hipSuccess;
  u64 *kin = keys, *kout = keys + len;
  const int bits = 32 + std::max(1, 64 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, r1 - r0)));
  hipLaunchKernelGGL(k_row_keys, dim3(grid(r1 - r0, 4)), dim3(256), 0, st, off, idx, r0, r1, kin);
  size_t tb = (size_t)temp_bytes;
  hipError_t e;
  if (wk == W_UNIT) {
    e = hipcub::DeviceRadixSort::SortKeys(temp, tb, kin, kout, (int)len, 0, bits, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_store<W_UNIT>, dim3(grid(len, 256)), dim3(256), 0, st, kout, (const int32_t *)nullptr,
                       len, e0, idx, (const void *)nullptr, (void *)nullptr);
    return hipGetLastError();
  }
  int32_t *pin = perm, *pout = perm + len;
  hipLaunchKernelGGL(k_iota, dim3(grid(len, 256)), dim3(256), 0, st, pin, len);
  e = hipcub::DeviceRadixSort::SortPairs(temp, tb, kin, kout, pin, pout, (int)len, 0, bits, st);
  if (e != hipSuccess) return e;
  const size_t wb = wk == W_U8 ? 1 : 4;
  e = hipMemcpyAsync(wcopy, (char *)w + e0 * wb, len * wb, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  if (wk == W_U8)
    hipLaunchKernelGGL(k_row_store<W_U8>, dim3(grid(len, 256)), dim3(256), 0, st, kout, pout, len, e0, idx,
                       (const void *)wcopy, w);
  else
    hipLaunchKernelGGL(k_row_store<W_U32>, dim3(grid(len, 256)), dim3(256), 0, st, kout, pout, len, e0, idx,
                       (const void *)wcopy, w);
  return hipGetLastError();
}

void launch_gather_i32(int32_t *dst, const int32_t *src, const int32_t *index, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_gather<int32_t>, dim3(grid(n, 256)), dim3(256), 0, st, dst, src, index, n);
}

void launch_gather_u8(uint8_t *dst, const uint8_t *src, const int32_t *index, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_gather<uint8_t>, dim3(grid(n, 256)), dim3(256), 0, st, dst, src, index, n);
}

}  // namespace gvelpa
