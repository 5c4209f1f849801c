// Normalised mutual information of two labelings on the GPU:
//   NMI = 2 I(X;Y) / (H(X) + H(Y)), natural logarithm (arithmetic normalisation).
// With n_a, n_b, n_ab the sizes of the classes and of their intersections and
// S_a = sum n_a ln n_a (likewise S_b, S_ab):
//   H(X) = ln n - S_a / n,  H(Y) = ln n - S_b / n,
//   I(X;Y) = ln n + (S_ab - S_a - S_b) / n.
// Class sizes come from radix-sorting the labels (and the label pairs) and
// run-length encoding the sorted keys; the x ln x sums are reduced in double
// in a fixed order.  Two single-class labelings give 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <hipcub/hipcub.hpp>
#include <vector>

#include "gvelpa.h"
#include "sweep_kernels.hpp"

namespace {

struct Fail {
  int code;
};

#define NMI_HIP(expr)                                        \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) {                                  \
      gvelpa::note_hip_error(_e, #expr, __FILE__, __LINE__); \
      throw Fail{LPA_ERR_DEVICE};                            \
    }                                                        \
  } while (0)

constexpr int RED_BLOCKS = 1024;

__global__ void k_pack_keys(const int32_t *a, const int32_t *b, int64_t n, uint64_t *ka, uint64_t *kb,
                            uint64_t *kab) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t x = (uint32_t)a[i], y = (uint32_t)b[i];
    ka[i] = x;
    kb[i] = y;
    kab[i] = ((uint64_t)x << 32) | y;
  }
}

// partial[block] = sum over runs r of this block's stride of c_r ln c_r
__global__ __launch_bounds__(256) void k_xlogx(const uint32_t *counts, const int64_t *nruns, double *partial) {
  __shared__ double red[256];
  const int64_t m = *nruns;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    const double c = (double)counts[i];
    s += c * log(c);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

struct Buf {
  hipStream_t st = nullptr;
  std::vector<void *> mem;
  ~Buf() {
    (void)hipStreamSynchronize(st);  // nothing is freed while a kernel may still use it
    for (void *p : mem) (void)hipFree(p);
  }
  template <class T>
  T *alloc(size_t count) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{LPA_ERR_OUT_OF_MEMORY};
    }
    mem.push_back(p);
    return (T *)p;
  }
};

// sum of c ln c over the class sizes of the keys; *classes receives their number
double sum_xlogx(Buf &buf, uint64_t *keys, uint64_t *sorted, int64_t n, int bits, hipStream_t st,
                 int64_t *classes) {
  size_t t1 = 0, t2 = 0;
  NMI_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, t1, keys, sorted, (int)n, 0, bits, st));
  uint64_t *uniq = keys;  // the unsorted keys are no longer needed
  uint32_t *counts = buf.alloc<uint32_t>(n);
  int64_t *nruns = buf.alloc<int64_t>(1);
  NMI_HIP(hipcub::DeviceRunLengthEncode::Encode(nullptr, t2, sorted, uniq, counts, nruns, (int)n, st));
  void *tmp = buf.alloc<char>(std::max(t1, t2));
  NMI_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, t1, keys, sorted, (int)n, 0, bits, st));
  NMI_HIP(hipcub::DeviceRunLengthEncode::Encode(tmp, t2, sorted, uniq, counts, nruns, (int)n, st));
  double *partial = buf.alloc<double>(RED_BLOCKS);
  hipLaunchKernelGGL(k_xlogx, dim3(RED_BLOCKS), dim3(256), 0, st, counts, nruns, partial);
  NMI_HIP(hipGetLastError());
  std::vector<double> h(RED_BLOCKS);
  NMI_HIP(hipMemcpyAsync(h.data(), partial, sizeof(double) * RED_BLOCKS, hipMemcpyDeviceToHost, st));
  NMI_HIP(hipMemcpyAsync(classes, nruns, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  NMI_HIP(hipStreamSynchronize(st));
  double s = 0.0;
  for (double x : h) s += x;
  return s;
}

}  // namespace

extern "C" int lpa_nmi(const int32_t *a, const int32_t *b, int64_t n, double *nmi_out, int device, void *hip_stream,
                       unsigned flags) {
  if (!nmi_out || n < 0 || (n > 0 && (!a || !b))) return LPA_ERR_INVALID_ARG;
  if (n >= ((int64_t)1 << 31)) return LPA_ERR_TOO_LARGE;
  if (n == 0) {
    *nmi_out = 1.0;
    return LPA_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return LPA_ERR_DEVICE;
  }
  if (device < 0 || device >= ndev) return LPA_ERR_INVALID_ARG;
  try {
    NMI_HIP(hipSetDevice(device));
    hipStream_t st = (hipStream_t)hip_stream;
    Buf buf;
    buf.st = st;
    const int32_t *da = a, *db = b;
    if (!(flags & LPA_FLAG_DEVICE_PTRS)) {
      int32_t *ca = buf.alloc<int32_t>(n), *cb = buf.alloc<int32_t>(n);
      NMI_HIP(hipMemcpyAsync(ca, a, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
      NMI_HIP(hipMemcpyAsync(cb, b, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
      da = ca;
      db = cb;
    }
    uint64_t *ka = buf.alloc<uint64_t>(n), *kb = buf.alloc<uint64_t>(n), *kab = buf.alloc<uint64_t>(n);
    uint64_t *sorted = buf.alloc<uint64_t>(n);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_pack_keys, dim3(blocks), dim3(256), 0, st, da, db, n, ka, kb, kab);
    NMI_HIP(hipGetLastError());
    int64_t classes_a = 0, classes_b = 0, classes_ab = 0;
    const double sa = sum_xlogx(buf, ka, sorted, n, 32, st, &classes_a);
    const double sb = sum_xlogx(buf, kb, sorted, n, 32, st, &classes_b);
    const double sab = sum_xlogx(buf, kab, sorted, n, 64, st, &classes_ab);
    const double dn = (double)n, ln = std::log(dn);
    // a single class has entropy 0 exactly (and then I = 0)
    const bool one_a = classes_a == 1, one_b = classes_b == 1;
    const double hx = one_a ? 0.0 : ln - sa / dn, hy = one_b ? 0.0 : ln - sb / dn;
    const double mi = (one_a || one_b) ? 0.0 : ln + (sab - sa - sb) / dn;
    *nmi_out = hx + hy <= 0.0 ? 1.0 : 2.0 * mi / (hx + hy);
    NMI_HIP(hipStreamSynchronize(st));
    return LPA_OK;
  } catch (Fail f) {
    return f.code;
  }
}
