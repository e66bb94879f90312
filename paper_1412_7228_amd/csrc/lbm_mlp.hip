// Surrogate network for surface-tension inversion: (A, kappa, T/Tc) -> (sigma,
// rho_l, rho_v), all normalised by the caller.  3 -> 128 -> 128 -> 128 -> 3,
// tanh hidden layers, linear output.
//
// Weights are held as bfloat16 (rounded from an FP32 master copy after every
// Adam step) and expanded exactly to FP32; activations, biases and every
// accumulation are FP32.  A workgroup of 256 threads (4 waves) handles 32
// samples; the two 128x128 layers of the forward pass and the two 128x128
// products of each hidden layer's backward pass (weight gradient and input
// gradient) run on the matrix cores (v_mfma_f32_32x32x2f32), one 32x32 block
// per wave at a time; the 3-wide layers are plain FMAs.  Weight gradients are
// written per workgroup and summed over workgroups in a fixed order, so a
// training step is deterministic.
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {

constexpr int kH = 128, kIn = 3, kOut = 3, kRows = 32, kThreads = 256;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH;
constexpr int oW3 = oB2 + kH, oB3 = oW3 + kH * kH, oW4 = oB3 + kH, oB4 = oW4 + kOut * kH;
constexpr int kNP = oB4 + kOut;  // 33,923
static_assert(kNP == 33923, "parameter count");

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bfw(const unsigned short* __restrict__ w, int i) {
  return __uint_as_float((unsigned)w[i] << 16);
}

// bfloat16 of an FP32 value: round to nearest, ties to even.
__device__ __forceinline__ unsigned short to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Accumulator layout of a 32x32 MFMA block: register r of lane l holds
// (row, col) = (8 (r / 4) + 4 (l / 32) + r % 4, l % 32).
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// acc += A[32 x K] * B[K x 32]; the lane supplies A(i, k) and B(k, i) with
// i = lane % 32 and k = k0 + lane / 32 for k0 = 0, 2, 4, ...
template <class FA, class FB>
__device__ __forceinline__ f32x16 mfma_32x32(FA a, FB b, int K, f32x16 acc) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 31, kk = lane >> 5;
  for (int k = 0; k < K; k += 2) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a(i, k + kk), b(k + kk, i), acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.f;
  return z;
}

// ---------------------------------------------------------------------------
// Forward: y = W4 h3 + b4, h_l = tanh(W_l h_{l-1} + b_l); optionally keeps
// h1..h3 in acts[3][B][128] for the backward pass.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
    k_mlp_forward(const float* __restrict__ x, int B, const float* __restrict__ master,
                  const unsigned short* __restrict__ wb, float* __restrict__ acts,
                  float* __restrict__ y) {
  __shared__ float hA[kRows][kH + 1], hB[kRows][kH + 1];
  __shared__ float xs[kRows][kIn];
  const int r0 = blockIdx.x * kRows, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid < kRows * kIn) {
    const int r = tid / kIn, k = tid % kIn;
    xs[r][k] = (r0 + r < B) ? x[(long long)(r0 + r) * kIn + k] : 0.f;
  }
  __syncthreads();
  for (int e = tid; e < kRows * kH; e += kThreads) {
    const int r = e / kH, o = e % kH;
    float z = master[oB1 + o];
#pragma unroll
    for (int k = 0; k < kIn; ++k) z += bfw(wb, oW1 + o * kIn + k) * xs[r][k];
    hA[r][o] = tanhf(z);
  }
  __syncthreads();
  float (*in)[kH + 1] = hA;
  float (*out)[kH + 1] = hB;
  for (int layer = 0; layer < 2; ++layer) {
    if (acts)
      for (int e = tid; e < kRows * kH; e += kThreads) {
        const int r = e / kH, o = e % kH;
        if (r0 + r < B) acts[((long long)layer * B + r0 + r) * kH + o] = in[r][o];
      }
    const int oW = layer == 0 ? oW2 : oW3, oB = layer == 0 ? oB2 : oB3;
    // out[:, 32w .. 32w+32) = tanh(in W^T + b): A(i, k) = in[i][k], B(k, j) = W[32w + j][k]
    f32x16 acc = mfma_32x32([&](int i, int k) { return in[i][k]; },
                            [&](int k, int j) { return bfw(wb, oW + (32 * w + j) * kH + k); }, kH, zero16());
    const int col = 32 * w + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) out[acc_row(r, lane)][col] = tanhf(acc[r] + master[oB + col]);
    __syncthreads();
    float (*t)[kH + 1] = in;
    in = out;
    out = t;
  }
  if (acts)
    for (int e = tid; e < kRows * kH; e += kThreads) {
      const int r = e / kH, o = e % kH;
      if (r0 + r < B) acts[((long long)2 * B + r0 + r) * kH + o] = in[r][o];
    }
  if (tid < kRows * kOut) {
    const int r = tid / kOut, o = tid % kOut;
    float z = master[oB4 + o];
    for (int k = 0; k < kH; ++k) z += bfw(wb, oW4 + o * kH + k) * in[r][k];
    if (r0 + r < B) y[(long long)(r0 + r) * kOut + o] = z;
  }
}

// ---------------------------------------------------------------------------
// Backward of sum(dy * y): per-workgroup parameter gradients into
// gpart[blockIdx.x][kNP] and (optionally) the input gradient dx[B][3].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
    k_mlp_backward(const float* __restrict__ x, const float* __restrict__ acts,
                   const float* __restrict__ dy, int B, const unsigned short* __restrict__ wb,
                   float* __restrict__ gpart, float* __restrict__ dx) {
  __shared__ float hs[kRows][kH + 1];  // input activation of the current layer
  __shared__ float dz[kRows][kH + 1];  // gradient at the current layer's pre-activation
  __shared__ float dn[kRows][kH + 1];  // gradient at the layer below
  __shared__ float xs[kRows][kIn], dys[kRows][kOut];
  const int r0 = blockIdx.x * kRows, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  float* gp = gpart + (long long)blockIdx.x * kNP;
  auto load_act = [&](int layer) {  // h_{layer+1} into hs; rows past B are zero
    for (int e = tid; e < kRows * kH; e += kThreads) {
      const int r = e / kH, o = e % kH;
      hs[r][o] = (r0 + r < B) ? acts[((long long)layer * B + r0 + r) * kH + o] : 0.f;
    }
  };
  if (tid < kRows * kIn) {
    const int r = tid / kIn, k = tid % kIn;
    xs[r][k] = (r0 + r < B) ? x[(long long)(r0 + r) * kIn + k] : 0.f;
    dys[r][k] = (r0 + r < B) ? dy[(long long)(r0 + r) * kOut + k] : 0.f;
  }
  load_act(2);
  __syncthreads();
  // output layer: dW4[o][k] = sum_r dy[r][o] h3[r][k], db4, dz3 = (dy W4) (1 - h3^2)
  for (int e = tid; e < kOut * kH; e += kThreads) {
    const int o = e / kH, k = e % kH;
    float s = 0.f;
    for (int r = 0; r < kRows; ++r) s += dys[r][o] * hs[r][k];
    gp[oW4 + e] = s;
  }
  if (tid < kOut) {
    float s = 0.f;
    for (int r = 0; r < kRows; ++r) s += dys[r][tid];
    gp[oB4 + tid] = s;
  }
  for (int e = tid; e < kRows * kH; e += kThreads) {
    const int r = e / kH, k = e % kH;
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < kOut; ++o) s += dys[r][o] * bfw(wb, oW4 + o * kH + k);
    dz[r][k] = s * (1.f - hs[r][k] * hs[r][k]);
  }
  __syncthreads();
  // hidden layers 3 and 2 (128 x 128)
  for (int layer = 1; layer >= 0; --layer) {
    const int oW = layer == 1 ? oW3 : oW2, oB = layer == 1 ? oB3 : oB2;
    load_act(layer);  // h_{layer+1}: the input of weight layer (layer + 2)
    __syncthreads();
    // dW[o][k] = sum_r dz[r][o] hs[r][k]: wave w owns output rows 32w..32w+32
    for (int kb = 0; kb < 4; ++kb) {
      f32x16 acc = mfma_32x32([&](int i, int r) { return dz[r][32 * w + i]; },
                              [&](int r, int j) { return hs[r][32 * kb + j]; }, kRows, zero16());
#pragma unroll
      for (int r = 0; r < 16; ++r)
        gp[oW + (32 * w + acc_row(r, lane)) * kH + 32 * kb + (lane & 31)] = acc[r];
    }
    if (tid < kH) {
      float s = 0.f;
      for (int r = 0; r < kRows; ++r) s += dz[r][tid];
      gp[oB + tid] = s;
    }
    // dn[r][k] = (sum_o dz[r][o] W[o][k]) (1 - hs[r][k]^2): wave w owns columns 32w..32w+32
    f32x16 acc = mfma_32x32([&](int i, int o) { return dz[i][o]; },
                            [&](int o, int j) { return bfw(wb, oW + o * kH + 32 * w + j); }, kH, zero16());
    const int col = 32 * w + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = acc_row(r, lane);
      dn[row][col] = acc[r] * (1.f - hs[row][col] * hs[row][col]);
    }
    __syncthreads();
    for (int e = tid; e < kRows * kH; e += kThreads) {
      const int r = e / kH, k = e % kH;
      dz[r][k] = dn[r][k];
    }
    __syncthreads();
  }
  // first layer: dW1[o][k] = sum_r dz1[r][o] x[r][k], db1, dx = dz1 W1
  for (int e = tid; e < kH * kIn; e += kThreads) {
    const int o = e / kIn, k = e % kIn;
    float s = 0.f;
    for (int r = 0; r < kRows; ++r) s += dz[r][o] * xs[r][k];
    gp[oW1 + e] = s;
  }
  if (tid < kH) {
    float s = 0.f;
    for (int r = 0; r < kRows; ++r) s += dz[r][tid];
    gp[oB1 + tid] = s;
  }
  if (dx && tid < kRows * kIn) {
    const int r = tid / kIn, k = tid % kIn;
    float s = 0.f;
    for (int o = 0; o < kH; ++o) s += dz[r][o] * bfw(wb, oW1 + o * kIn + k);
    if (r0 + r < B) dx[(long long)(r0 + r) * kIn + k] = s;
  }
}

// grad[i] = sum over workgroups of gpart[w][i], in workgroup order.
__global__ void k_mlp_reduce(const float* __restrict__ gpart, int nwg, float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNP) return;
  float s = 0.f;
  for (int wg = 0; wg < nwg; ++wg) s += gpart[(long long)wg * kNP + i];
  grad[i] = s;
}

// Mean squared error over B x 3 outputs: dy = 2 (y - t) / (3B); loss[0] = mean.
__global__ void __launch_bounds__(kThreads)
    k_mlp_mse(const float* __restrict__ y, const float* __restrict__ t, int B, float* __restrict__ dy,
              float* __restrict__ loss) {
  __shared__ float sh[kThreads];
  const int n = B * kOut;
  const float inv = 1.f / (float)n;
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d * inv;
    s += d * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = sh[0] * inv;
}

// Adam on the FP32 master parameters, then the bfloat16 copy of every parameter.
__global__ void k_mlp_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, unsigned short* __restrict__ wb, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNP) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  wb[i] = to_bf16(pi);
}

__global__ void k_mlp_round(const float* __restrict__ p, unsigned short* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kNP) wb[i] = to_bf16(p[i]);
}

int mlp_param_count() { return kNP; }
int mlp_rows_per_block() { return kRows; }

hipError_t launch_mlp_forward(const float* x, int B, const float* master, const unsigned short* wb,
                              float* acts, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3((B + kRows - 1) / kRows), dim3(kThreads), 0, s, x, B, master,
                     wb, acts, y);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* x, const float* acts, const float* dy, int B,
                               const unsigned short* wb, float* gpart, float* grad, float* dx,
                               hipStream_t s) {
  const int nwg = (B + kRows - 1) / kRows;
  hipLaunchKernelGGL(k_mlp_backward, dim3(nwg), dim3(kThreads), 0, s, x, acts, dy, B, wb, gpart, dx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNP + 255) / 256), dim3(256), 0, s, gpart, nwg, grad);
  return hipGetLastError();
}

hipError_t launch_mlp_mse(const float* y, const float* t, int B, float* dy, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_mse, dim3(1), dim3(kThreads), 0, s, y, t, B, dy, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* p, float* m, float* v, const float* g, unsigned short* wb, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, p, m, v, g, wb, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_round(const float* p, unsigned short* wb, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_round, dim3((kNP + 255) / 256), dim3(256), 0, s, p, wb);
  return hipGetLastError();
}

}  // namespace lbm
