// C ABI of the gate network's training side: forward pass, gradient, Adam
// training over a trace of (features, changed) samples and the choice of the
// decision threshold.  All arithmetic runs in gate_kernels.hip; this file
// moves arguments and owns temporary device buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "gvelpa.h"
#include "sweep_kernels.hpp"

using namespace gvelpa;

namespace {

struct Fail {
  int code;
};

#define GATE_HIP(expr)                                       \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) {                                  \
      note_hip_error(_e, #expr, __FILE__, __LINE__);         \
      throw Fail{LPA_ERR_DEVICE};                            \
    }                                                        \
  } while (0)

// Device buffers of one call, freed on every exit path.
struct Scope {
  int device = 0;
  hipStream_t st = nullptr;
  std::vector<void *> mem;
  ~Scope() {
    (void)hipStreamSynchronize(st);  // nothing is freed while a kernel may still use it
    for (void *p : mem) (void)hipFree(p);
  }
  template <class T>
  T *alloc(int64_t count) {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess) {
      (void)hipGetLastError();
      throw Fail{LPA_ERR_OUT_OF_MEMORY};
    }
    mem.push_back(p);
    return (T *)p;
  }
  // Device view of a caller array: the pointer itself with LPA_FLAG_DEVICE_PTRS, else a copy.
  template <class T>
  const T *in(const T *src, int64_t count, unsigned flags) {
    if (flags & LPA_FLAG_DEVICE_PTRS) return src;
    T *d = alloc<T>(count);
    if (count) GATE_HIP(hipMemcpyAsync(d, src, sizeof(T) * count, hipMemcpyHostToDevice, st));
    return d;
  }
};

template <class Fn>
int guarded(int device, void *stream, Fn &&fn) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return LPA_ERR_DEVICE;
  }
  if (device < 0 || device >= ndev) return LPA_ERR_INVALID_ARG;
  try {
    Scope s;
    GATE_HIP(hipSetDevice(device));
    s.device = device;
    s.st = (hipStream_t)stream;
    int rc = fn(s);
    GATE_HIP(hipStreamSynchronize(s.st));
    return rc;
  } catch (Fail f) {
    return f.code;
  }
}

bool finite_params(const float *p) {
  for (int k = 0; k < GATE_PARAMS; ++k)
    if (!std::isfinite(p[k])) return false;
  return true;
}

// Every index of a host array in [0, limit).
bool indices_ok(const int64_t *sel, int64_t len, int64_t limit) {
  for (int64_t k = 0; k < len; ++k)
    if (sel[k] < 0 || sel[k] >= limit) return false;
  return true;
}

void check_device_indices(Scope &s, const int64_t *sel, int64_t len, int64_t limit) {
  int32_t *bad = s.alloc<int32_t>(1);
  GATE_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s.st));
  launch_check_index(sel, len, limit, bad, s.st);
  int32_t h = 0;
  GATE_HIP(hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, s.st));
  GATE_HIP(hipStreamSynchronize(s.st));
  if (h) throw Fail{LPA_ERR_INVALID_ARG};
}

constexpr float ADAM_B1 = 0.9f, ADAM_B2 = 0.999f, ADAM_EPS = 1e-8f;

}  // namespace

// ---------------------------------------------------------------- no-allocation gradient
//
// Scratch of lpa_gate_backward_noalloc in a file-scope device array: the
// device copy of the parameters, the reduced gradient and the per-workgroup
// partials of up to LPA_GATE_NOALLOC_MAX_SAMPLES samples.  Each GPU holds its
// own copy at its own address until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns for that device.
constexpr int64_t NA_PARAMS_OFF = 0;
constexpr int64_t NA_ACC_OFF = 1408;   // GATE_PARAMS rounded up to 256-byte lines
constexpr int64_t NA_PART_OFF = 2816;
constexpr int64_t NA_FLOATS =
    NA_PART_OFF + (int64_t)((LPA_GATE_NOALLOC_MAX_SAMPLES + 127) / 128) * (GATE_PARAMS + 1);
static_assert(NA_ACC_OFF >= GATE_PARAMS && NA_PART_OFF - NA_ACC_OFF >= GATE_PARAMS + 1, "scratch layout");

static __device__ __align__(256) float scratch[NA_FLOATS];

namespace {

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mu;
float *na_ptr[NA_MAX_DEVICES] = {};

// Device address of this device's scratch (the device is current).
float *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(na_mu);
  if (!na_ptr[device]) {
    void *p = nullptr;
    GATE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    na_ptr[device] = (float *)p;
  }
  return na_ptr[device];
}

}  // namespace

extern "C" {

int lpa_gate_forward(const float *params, const float *features, int64_t count, float *probs, int device,
                     void *hip_stream, unsigned flags) {
  if (!params || count < 0 || (count > 0 && (!features || !probs))) return LPA_ERR_INVALID_ARG;
  if (!finite_params(params)) return LPA_ERR_INVALID_ARG;
  return guarded(device, hip_stream, [&](Scope &s) -> int {
    float *master = s.alloc<float>(GATE_PARAMS);
    GATE_HIP(hipMemcpyAsync(master, params, sizeof(float) * GATE_PARAMS, hipMemcpyHostToDevice, s.st));
    if (!count) return LPA_OK;
    const float *X = s.in(features, count * NFEAT, flags);
    float *p = (flags & LPA_FLAG_DEVICE_PTRS) ? probs : s.alloc<float>(count);
    launch_gate_forward(master, X, count, p, s.st);
    GATE_HIP(hipGetLastError());
    if (!(flags & LPA_FLAG_DEVICE_PTRS))
      GATE_HIP(hipMemcpyAsync(probs, p, sizeof(float) * count, hipMemcpyDeviceToHost, s.st));
    return LPA_OK;
  });
}

int lpa_gate_backward(const float *params, const float *features, const uint8_t *targets, int64_t count,
                      float pos_weight, float *grad, float *loss, int device, void *hip_stream, unsigned flags) {
  if (!params || !grad || count <= 0 || !features || !targets) return LPA_ERR_INVALID_ARG;
  if (!(pos_weight >= 0.0f) || !std::isfinite(pos_weight) || !finite_params(params)) return LPA_ERR_INVALID_ARG;
  return guarded(device, hip_stream, [&](Scope &s) -> int {
    float *master = s.alloc<float>(GATE_PARAMS);
    GATE_HIP(hipMemcpyAsync(master, params, sizeof(float) * GATE_PARAMS, hipMemcpyHostToDevice, s.st));
    const float *X = s.in(features, count * NFEAT, flags);
    const uint8_t *Y = s.in(targets, count, flags);
    // partial sums per workgroup, in slices that keep the partial buffer small
    const int64_t slice = (int64_t)1 << 22;
    float *partial = s.alloc<float>((int64_t)gate_grad_blocks(std::min(slice, count)) * (GATE_PARAMS + 1));
    float *acc = s.alloc<float>(GATE_PARAMS + 1);
    std::vector<double> total(GATE_PARAMS + 1, 0.0);
    std::vector<float> part(GATE_PARAMS + 1);
    for (int64_t base = 0; base < count; base += slice) {
      const int64_t nb = std::min(slice, count - base);
      launch_gate_grad(master, X, Y, nullptr, base, nb, pos_weight, (float)count, partial, acc, s.st);
      GATE_HIP(hipGetLastError());
      GATE_HIP(hipMemcpyAsync(part.data(), acc, sizeof(float) * (GATE_PARAMS + 1), hipMemcpyDeviceToHost, s.st));
      GATE_HIP(hipStreamSynchronize(s.st));
      for (int k = 0; k <= GATE_PARAMS; ++k) total[k] += part[k];
    }
    for (int k = 0; k < GATE_PARAMS; ++k) grad[k] = (float)total[k];
    if (loss) *loss = (float)total[GATE_PARAMS];
    return LPA_OK;
  });
}

int lpa_gate_backward_noalloc(const float *params, const float *features, const uint8_t *targets, int64_t count,
                              float pos_weight, float *grad, float *loss, int device, void *hip_stream) {
  if (!params || !grad || !features || !targets || count <= 0) return LPA_ERR_INVALID_ARG;
  if (count > LPA_GATE_NOALLOC_MAX_SAMPLES) return LPA_ERR_TOO_LARGE;
  if (!(pos_weight >= 0.0f) || !std::isfinite(pos_weight) || !finite_params(params)) return LPA_ERR_INVALID_ARG;
  if (device < 0 || device >= NA_MAX_DEVICES) return LPA_ERR_INVALID_ARG;
  return guarded(device, hip_stream, [&](Scope &s) -> int {
    float *base = noalloc_scratch(device);
    float *master = base + NA_PARAMS_OFF;
    float *acc = base + NA_ACC_OFF;
    float *partial = base + NA_PART_OFF;
    GATE_HIP(hipMemcpyAsync(master, params, sizeof(float) * GATE_PARAMS, hipMemcpyHostToDevice, s.st));
    // one pass (count fits the partials), so the sums are those of lpa_gate_backward
    launch_gate_grad(master, features, targets, nullptr, 0, count, pos_weight, (float)count, partial, acc, s.st);
    GATE_HIP(hipGetLastError());
    float part[GATE_PARAMS + 1];
    GATE_HIP(hipMemcpyAsync(part, acc, sizeof(float) * (GATE_PARAMS + 1), hipMemcpyDeviceToHost, s.st));
    GATE_HIP(hipStreamSynchronize(s.st));
    std::memcpy(grad, part, sizeof(float) * GATE_PARAMS);
    if (loss) *loss = part[GATE_PARAMS];
    return LPA_OK;
  });
}

int lpa_gate_train(float *params, const float *features, const uint8_t *targets, int64_t count,
                   const int64_t *order, int32_t epochs, int32_t batch, float lr, float pos_weight,
                   float *epoch_loss, int device, void *hip_stream, unsigned flags) {
  if (!params || count <= 0 || !features || !targets || epochs < 0 || batch <= 0 || batch > (1 << 24))
    return LPA_ERR_INVALID_ARG;
  if (!(lr > 0.0f) || !std::isfinite(lr) || !(pos_weight >= 0.0f) || !std::isfinite(pos_weight))
    return LPA_ERR_INVALID_ARG;
  if (!finite_params(params)) return LPA_ERR_INVALID_ARG;
  if (order && !(flags & LPA_FLAG_DEVICE_PTRS) && !indices_ok(order, count * (int64_t)epochs, count))
    return LPA_ERR_INVALID_ARG;
  return guarded(device, hip_stream, [&](Scope &s) -> int {
    float *theta = s.alloc<float>(GATE_PARAMS);
    float *mom = s.alloc<float>(2 * GATE_PARAMS);
    float *grad = s.alloc<float>(GATE_PARAMS + 1);
    float *losses = s.alloc<float>(std::max(epochs, 1));
    GATE_HIP(hipMemcpyAsync(theta, params, sizeof(float) * GATE_PARAMS, hipMemcpyHostToDevice, s.st));
    GATE_HIP(hipMemsetAsync(mom, 0, sizeof(float) * 2 * GATE_PARAMS, s.st));
    GATE_HIP(hipMemsetAsync(losses, 0, sizeof(float) * std::max(epochs, 1), s.st));
    const float *X = s.in(features, count * NFEAT, flags);
    const uint8_t *Y = s.in(targets, count, flags);
    const int64_t *sel = order ? s.in(order, count * (int64_t)epochs, flags) : nullptr;
    if (sel && (flags & LPA_FLAG_DEVICE_PTRS)) check_device_indices(s, sel, count * (int64_t)epochs, count);
    const int64_t nb_max = std::min<int64_t>(batch, count);
    float *partial = s.alloc<float>((int64_t)gate_grad_blocks(nb_max) * (GATE_PARAMS + 1));
    int t = 0;
    for (int e = 0; e < epochs; ++e) {
      for (int64_t b = 0; b < count; b += batch) {
        const int64_t nb = std::min<int64_t>(batch, count - b);
        const int64_t base = sel ? (int64_t)e * count + b : b;
        launch_gate_grad(theta, X, Y, sel, base, nb, pos_weight, (float)nb, partial, grad, s.st);
        launch_adam(theta, grad, mom, mom + GATE_PARAMS, ++t, lr, ADAM_B1, ADAM_B2, ADAM_EPS, losses + e,
                    (float)((double)nb / (double)count), s.st);
      }
      GATE_HIP(hipGetLastError());
    }
    GATE_HIP(hipMemcpyAsync(params, theta, sizeof(float) * GATE_PARAMS, hipMemcpyDeviceToHost, s.st));
    if (epoch_loss && epochs)
      GATE_HIP(hipMemcpyAsync(epoch_loss, losses, sizeof(float) * epochs, hipMemcpyDeviceToHost, s.st));
    return LPA_OK;
  });
}

int lpa_gate_threshold(const float *params, const float *features, const uint8_t *targets, int64_t count,
                       double recall, float *threshold, int device, void *hip_stream, unsigned flags) {
  if (!params || !threshold || count <= 0 || !features || !targets || !(recall >= 0.0) || !(recall <= 1.0))
    return LPA_ERR_INVALID_ARG;
  if (!finite_params(params)) return LPA_ERR_INVALID_ARG;
  return guarded(device, hip_stream, [&](Scope &s) -> int {
    float *master = s.alloc<float>(GATE_PARAMS);
    GATE_HIP(hipMemcpyAsync(master, params, sizeof(float) * GATE_PARAMS, hipMemcpyHostToDevice, s.st));
    const float *X = s.in(features, count * NFEAT, flags);
    const uint8_t *Y = s.in(targets, count, flags);
    float *p = s.alloc<float>(count);
    float *pos = s.alloc<float>(count);
    unsigned long long *npos = s.alloc<unsigned long long>(1);
    GATE_HIP(hipMemsetAsync(npos, 0, sizeof(unsigned long long), s.st));
    launch_gate_forward(master, X, count, p, s.st);
    launch_select_pos(p, Y, count, pos, npos, s.st);
    GATE_HIP(hipGetLastError());
    unsigned long long h_npos = 0;
    GATE_HIP(hipMemcpyAsync(&h_npos, npos, sizeof(h_npos), hipMemcpyDeviceToHost, s.st));
    GATE_HIP(hipStreamSynchronize(s.st));
    if (h_npos == 0) {
      *threshold = 1.0f;  // no sample ever changed: any threshold keeps recall
      return LPA_OK;
    }
    std::vector<float> h(h_npos);
    GATE_HIP(hipMemcpyAsync(h.data(), pos, sizeof(float) * h_npos, hipMemcpyDeviceToHost, s.st));
    GATE_HIP(hipStreamSynchronize(s.st));
    // largest t with #{positives with p >= t} >= recall * #positives: the k-th largest probability
    const int64_t need = std::max<int64_t>(1, (int64_t)std::ceil(recall * (double)h_npos));
    std::nth_element(h.begin(), h.begin() + (need - 1), h.end(), std::greater<float>());
    *threshold = h[need - 1];
    return LPA_OK;
  });
}

}  // extern "C"
