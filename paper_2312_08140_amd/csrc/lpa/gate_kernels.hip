// Training and evaluation of the learned active-set gate (8-32-32-1 network,
// ReLU, ReLU, sigmoid).  FP32 master parameters; every evaluation uses their
// bf16 rounding (round to nearest, ties to even) with FP32 accumulation.
// Loss: mean binary cross-entropy with positive-class weight pw,
//   l = -(pw y log p + (1 - y) log(1 - p)),  dl/dz = pw y (p - 1) + (1 - y) p.
// Optimiser: Adam with bias correction (Kingma and Ba, ICLR 2015).
#include <math.h>

#include "sweep_kernels.hpp"

namespace gvelpa {

constexpr int GB = 128;  // samples per workgroup (LDS: two 128 x 33 staging arrays)

__device__ __forceinline__ float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ void load_params(const float *master, float *P) {
  for (int k = threadIdx.x; k < GATE_PARAMS; k += blockDim.x) P[k] = bf16r(master[k]);
  __syncthreads();
}

struct Act {
  float a1[32];  // pre-activations of layer 1
  float a2[32];  // pre-activations of layer 2
  float z;
};

__device__ __forceinline__ void forward(const float *P, const float *x, Act &t) {
  const float *W1 = P, *b1 = P + 256, *W2 = P + 288, *b2 = P + 1312, *W3 = P + 1344;
#pragma unroll
  for (int o = 0; o < 32; ++o) {
    float acc = b1[o];
#pragma unroll
    for (int q = 0; q < NFEAT; ++q) acc = fmaf(W1[o * 8 + q], x[q], acc);
    t.a1[o] = acc;
  }
  float z = P[1376];
  for (int o = 0; o < 32; ++o) {
    float acc = b2[o];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc = fmaf(W2[o * 32 + q], fmaxf(t.a1[q], 0.0f), acc);
    t.a2[o] = acc;
    z = fmaf(W3[o], fmaxf(acc, 0.0f), z);
  }
  t.z = z;
}

__device__ __forceinline__ float sigmoidf_(float z) {
  return z >= 0.0f ? 1.0f / (1.0f + expf(-z)) : expf(z) / (1.0f + expf(z));
}

// softplus(z) = log(1 + e^z), stable
__device__ __forceinline__ float softplusf_(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }

__global__ __launch_bounds__(GB) void k_gate_forward(const float *master, const float *X, int64_t count, float *p) {
  __shared__ float P[GATE_PARAMS];
  load_params(master, P);
  for (int64_t s = (int64_t)blockIdx.x * GB + threadIdx.x; s < count; s += (int64_t)gridDim.x * GB) {
    float x[NFEAT];
#pragma unroll
    for (int q = 0; q < NFEAT; ++q) x[q] = X[s * NFEAT + q];
    Act t;
    forward(P, x, t);
    p[s] = sigmoidf_(t.z);
  }
}

// Per-workgroup partial gradient (and loss) over samples sel[base + r],
// r < nb (sel == NULL: samples base + r).  The loss is a mean over `denom`.
__global__ __launch_bounds__(GB) void k_gate_grad(const float *master, const float *X, const uint8_t *Y,
                                                  const int64_t *sel, int64_t base, int64_t nb, float pw,
                                                  float denom, float *partial) {
  __shared__ float P[GATE_PARAMS];
  __shared__ float s_a[GB][33];  // per-sample vectors, padded against bank conflicts
  __shared__ float s_b[GB][33];
  __shared__ float s_red[GB];
  load_params(master, P);
  const int64_t r = (int64_t)blockIdx.x * GB + threadIdx.x;
  const bool live = r < nb;
  float x[NFEAT] = {0, 0, 0, 0, 0, 0, 0, 0};
  float y = 0.0f;
  if (live) {
    const int64_t s = sel ? sel[base + r] : base + r;
#pragma unroll
    for (int q = 0; q < NFEAT; ++q) x[q] = X[s * NFEAT + q];
    y = Y[s] ? 1.0f : 0.0f;
  }
  Act t;
  forward(P, x, t);
  const float p = sigmoidf_(t.z);
  const float loss = live ? (pw * y * softplusf_(-t.z) + (1.0f - y) * softplusf_(t.z)) / denom : 0.0f;
  const float dz = live ? (pw * y * (p - 1.0f) + (1.0f - y) * p) / denom : 0.0f;
  const float *W2 = P + 288, *W3 = P + 1344;
  float *g = partial + (int64_t)blockIdx.x * (GATE_PARAMS + 1);
  // layer 3: dW3[o] = dz h2[o], db3 = dz; layer 2 deltas da2[o] = dz W3[o] [a2 > 0]
  float da2[32];
#pragma unroll
  for (int o = 0; o < 32; ++o) {
    da2[o] = t.a2[o] > 0.0f ? dz * W3[o] : 0.0f;
    s_a[threadIdx.x][o] = dz * fmaxf(t.a2[o], 0.0f);  // dW3 contribution
    s_b[threadIdx.x][o] = da2[o];                       // db2 contribution
  }
  s_a[threadIdx.x][32] = dz;
  s_red[threadIdx.x] = loss;
  __syncthreads();
  if (threadIdx.x < 32) {
    float a = 0.0f, b = 0.0f;
    for (int k = 0; k < GB; ++k) {
      a += s_a[k][threadIdx.x];
      b += s_b[k][threadIdx.x];
    }
    g[1344 + threadIdx.x] = a;  // W3
    g[1312 + threadIdx.x] = b;  // b2
  } else if (threadIdx.x == 32) {
    float a = 0.0f, l = 0.0f;
    for (int k = 0; k < GB; ++k) {
      a += s_a[k][32];
      l += s_red[k];
    }
    g[1376] = a;            // b3
    g[GATE_PARAMS] = l;     // loss
  }
  __syncthreads();
  // dW2[o][i] = da2[o] h1[i]: samples' da2 in s_a, h1 in s_b
#pragma unroll
  for (int o = 0; o < 32; ++o) {
    s_a[threadIdx.x][o] = da2[o];
    s_b[threadIdx.x][o] = fmaxf(t.a1[o], 0.0f);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < 1024; k += GB) {
    const int o = k >> 5, i = k & 31;
    float acc = 0.0f;
    for (int q = 0; q < GB; ++q) acc = fmaf(s_a[q][o], s_b[q][i], acc);
    g[288 + k] = acc;
  }
  // layer 1 deltas: dh1[i] = sum_o W2[o][i] da2[o]; da1[i] = dh1[i] [a1 > 0]
  float da1[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int o = 0; o < 32; ++o) acc = fmaf(W2[o * 32 + i], da2[o], acc);
    da1[i] = t.a1[i] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 32; ++i) s_a[threadIdx.x][i] = da1[i];
#pragma unroll
  for (int q = 0; q < NFEAT; ++q) s_b[threadIdx.x][q] = x[q];
  __syncthreads();
  // dW1[o][q] = da1[o] x[q]; db1[o] = da1[o]
  for (int k = threadIdx.x; k < 256 + 32; k += GB) {
    float acc = 0.0f;
    if (k < 256) {
      const int o = k >> 3, q = k & 7;
      for (int s = 0; s < GB; ++s) acc = fmaf(s_a[s][o], s_b[s][q], acc);
      g[k] = acc;
    } else {
      const int o = k - 256;
      for (int s = 0; s < GB; ++s) acc += s_a[s][o];
      g[256 + o] = acc;
    }
  }
}

// grad[k] = sum over workgroups of partial[.][k] (k <= GATE_PARAMS: the last is the loss)
__global__ void k_gate_reduce(const float *partial, int nblocks, float *grad) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k <= GATE_PARAMS; k += gridDim.x * blockDim.x) {
    double acc = 0.0;  // many partials: sum in double, round once
    for (int b = 0; b < nblocks; ++b) acc += (double)partial[(int64_t)b * (GATE_PARAMS + 1) + k];
    grad[k] = (float)acc;
  }
}

// One Adam update at step t (1-based); loss_acc (optional) += batch loss * loss_scale.
__global__ void k_adam(float *theta, const float *grad, float *m, float *v, int t, float lr, float b1, float b2,
                       float eps, float *loss_acc, float loss_scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && loss_acc) *loss_acc += grad[GATE_PARAMS] * loss_scale;
  if (k >= GATE_PARAMS) return;
  const float g = grad[k];
  const float mk = b1 * m[k] + (1.0f - b1) * g;
  const float vk = b2 * v[k] + (1.0f - b2) * g * g;
  m[k] = mk;
  v[k] = vk;
  const float mh = mk / (1.0f - powf(b1, (float)t));
  const float vh = vk / (1.0f - powf(b2, (float)t));
  theta[k] -= lr * mh / (sqrtf(vh) + eps);
}

// bad[0] = 1 if some sel[k], k < len, lies outside [0, limit)
__global__ void k_check_index(const int64_t *sel, int64_t len, int64_t limit, int32_t *bad) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += (int64_t)gridDim.x * blockDim.x)
    if (sel[k] < 0 || sel[k] >= limit) bad[0] = 1;
}

// probs of the samples with targets[s] != 0 (the positives), compacted to out; count in *npos
__global__ void k_select_pos(const float *p, const uint8_t *Y, int64_t count, float *out, unsigned long long *npos) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count; s += (int64_t)gridDim.x * blockDim.x)
    if (Y[s]) out[atomicAdd(npos, 1ull)] = p[s];
}

void launch_check_index(const int64_t *sel, int64_t len, int64_t limit, int32_t *bad, hipStream_t st) {
  hipLaunchKernelGGL(k_check_index, dim3(1024), dim3(256), 0, st, sel, len, limit, bad);
}

void launch_select_pos(const float *p, const uint8_t *Y, int64_t count, float *out, unsigned long long *npos,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_select_pos, dim3(1024), dim3(256), 0, st, p, Y, count, out, npos);
}

void launch_gate_forward(const float *master, const float *X, int64_t count, float *p, hipStream_t st) {
  int64_t blocks = (count + GB - 1) / GB;
  blocks = blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks);
  hipLaunchKernelGGL(k_gate_forward, dim3((unsigned)blocks), dim3(GB), 0, st, master, X, count, p);
}

int gate_grad_blocks(int64_t nb) { return (int)((nb + GB - 1) / GB); }

void launch_gate_grad(const float *master, const float *X, const uint8_t *Y, const int64_t *sel, int64_t base,
                      int64_t nb, float pw, float denom, float *partial, float *grad, hipStream_t st) {
  const int blocks = gate_grad_blocks(nb);
  hipLaunchKernelGGL(k_gate_grad, dim3(blocks), dim3(GB), 0, st, master, X, Y, sel, base, nb, pw, denom, partial);
  hipLaunchKernelGGL(k_gate_reduce, dim3(6), dim3(256), 0, st, partial, blocks, grad);
}

void launch_adam(float *theta, const float *grad, float *m, float *v, int t, float lr, float b1, float b2, float eps,
                 float *loss_acc, float loss_scale, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((GATE_PARAMS + 255) / 256), dim3(256), 0, st, theta, grad, m, v, t, lr, b1, b2,
                     eps, loss_acc, loss_scale);
}

}  // namespace gvelpa
