// Learned branching scorer: a 32 -> 128 -> 128 -> 1 ReLU perceptron.
// Inputs and weight matrices are bfloat16; biases, hidden activations and all
// accumulations are float32.  Forward, backward (MSE loss) and Adam are
// hand-written; weight gradients are reduced deterministically (per-block
// partials summed in block order).  Latency-bound at these sizes: one thread
// per hidden unit, 64 rows per workgroup.
#include "mlp.h"

namespace bbtn {

namespace {

constexpr int RB = 64;  // rows per workgroup

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void __launch_bounds__(MLP_H)
mlp_forward_kernel(int64_t R, const uint16_t* X, const uint16_t* W, const float* bias, float* y,
                   float* h1g, float* h2g) {
  __shared__ float xs[RB][MLP_IN];
  __shared__ float h1[RB][MLP_H + 1];
  __shared__ float h2[RB][MLP_H + 1];
  const int j = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int nr = (int)min<int64_t>(RB, R - r0);
  const uint16_t* W1 = W + MLP_W1;
  const uint16_t* W2 = W + MLP_W2;
  const uint16_t* w3 = W + MLP_W3;
  for (int e = j; e < nr * MLP_IN; e += MLP_H) xs[e / MLP_IN][e % MLP_IN] = bf2f(X[r0 * MLP_IN + e]);
  float w1[MLP_IN];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) w1[i] = bf2f(W1[j * MLP_IN + i]);
  const float b1 = bias[MLP_B1 + j], b2 = bias[MLP_B2 + j];
  __syncthreads();
  for (int r = 0; r < nr; ++r) {
    float z = b1;
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) z = fmaf(w1[i], xs[r][i], z);
    h1[r][j] = fmaxf(z, 0.f);
  }
  __syncthreads();
  for (int r = 0; r < nr; ++r) {
    float z = b2;
    for (int i = 0; i < MLP_H; ++i) z = fmaf(bf2f(W2[j * MLP_H + i]), h1[r][i], z);
    h2[r][j] = fmaxf(z, 0.f);
  }
  __syncthreads();
  if (j < nr) {
    float s = bias[MLP_B3];
    for (int i = 0; i < MLP_H; ++i) s = fmaf(bf2f(w3[i]), h2[j][i], s);
    y[r0 + j] = s;
  }
  if (h1g) {
    for (int r = 0; r < nr; ++r) {
      h1g[(r0 + r) * MLP_H + j] = h1[r][j];
      h2g[(r0 + r) * MLP_H + j] = h2[r][j];
    }
  }
}

// Per-block partial gradients of the mean squared error.
__global__ void __launch_bounds__(MLP_H)
mlp_backward_kernel(int64_t R, const uint16_t* X, const uint16_t* W, const float* y,
                    const float* t, const float* h1g, const float* h2g, float* part) {
  __shared__ float xs[RB][MLP_IN];
  __shared__ float h1[RB][MLP_H + 1];
  __shared__ float d2[RB][MLP_H + 1];
  __shared__ float dy[RB];
  const int j = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int nr = (int)min<int64_t>(RB, R - r0);
  const uint16_t* W2 = W + MLP_W2;
  const uint16_t* w3 = W + MLP_W3;
  float* P = part + (int64_t)blockIdx.x * MLP_NPART;
  for (int e = j; e < nr * MLP_IN; e += MLP_H) xs[e / MLP_IN][e % MLP_IN] = bf2f(X[r0 * MLP_IN + e]);
  if (j < nr) dy[j] = 2.f * (y[r0 + j] - t[r0 + j]) / (float)R;
  for (int r = 0; r < nr; ++r) h1[r][j] = h1g[(r0 + r) * MLP_H + j];
  __syncthreads();
  // output layer and second hidden layer
  const float w3j = bf2f(w3[j]);
  float gw3 = 0.f, gb2 = 0.f;
  for (int r = 0; r < nr; ++r) {
    const float h2v = h2g[(r0 + r) * MLP_H + j];
    gw3 = fmaf(dy[r], h2v, gw3);
    const float d = h2v > 0.f ? dy[r] * w3j : 0.f;
    d2[r][j] = d;
    gb2 += d;
  }
  P[MLP_W3 + j] = gw3;
  P[MLP_NW + MLP_B2 + j] = gb2;
  if (j == 0) {
    float s = 0.f, l = 0.f;
    for (int r = 0; r < nr; ++r) {
      s += dy[r];
      const float e = y[r0 + r] - t[r0 + r];
      l = fmaf(e, e, l);
    }
    P[MLP_NW + MLP_B3] = s;
    P[MLP_NW + MLP_NB] = l;  // sum of squared errors
  }
  __syncthreads();
  // dW2[j][i] = sum_r d2[r][j] h1[r][i]
  for (int i = 0; i < MLP_H; ++i) {
    float g = 0.f;
    for (int r = 0; r < nr; ++r) g = fmaf(d2[r][j], h1[r][i], g);
    P[MLP_W2 + j * MLP_H + i] = g;
  }
  // d1[r][j] = (sum_i d2[r][i] W2[i][j]) * (h1[r][j] > 0), then dW1, db1
  float w2col[MLP_H];
  for (int i = 0; i < MLP_H; ++i) w2col[i] = bf2f(W2[i * MLP_H + j]);
  float gw1[MLP_IN];
#pragma unroll
  for (int q = 0; q < MLP_IN; ++q) gw1[q] = 0.f;
  float gb1 = 0.f;
  for (int r = 0; r < nr; ++r) {
    float s = 0.f;
    for (int i = 0; i < MLP_H; ++i) s = fmaf(d2[r][i], w2col[i], s);
    const float d = h1[r][j] > 0.f ? s : 0.f;
    gb1 += d;
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) gw1[q] = fmaf(d, xs[r][q], gw1[q]);
  }
#pragma unroll
  for (int q = 0; q < MLP_IN; ++q) P[MLP_W1 + j * MLP_IN + q] = gw1[q];
  P[MLP_NW + MLP_B1 + j] = gb1;
}

// grad[p] = sum over blocks (in block order) of part[b][p]
__global__ void __launch_bounds__(256)
mlp_reduce_kernel(int64_t nblocks, const float* part, float* grad) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_NPART; p += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int64_t b = 0; b < nblocks; ++b) s += part[b * MLP_NPART + p];
    grad[p] = s;
  }
}

// Adam on the float32 master copy; refreshes the bfloat16 weight copy.
__global__ void __launch_bounds__(256)
mlp_adam_kernel(float* master, uint16_t* wbf, float* bias, float* m, float* v, const float* g,
                float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_NPARAM; p += gridDim.x * blockDim.x) {
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float upd = lr * (mp / c1) / (sqrtf(vp / c2) + eps);
    const float w = master[p] - upd;
    master[p] = w;
    if (p < MLP_NW) wbf[p] = f2bf(w);
    else bias[p - MLP_NW] = w;
  }
}

}  // namespace

void launch_mlp_forward(int64_t R, const uint16_t* X, const uint16_t* W, const float* bias,
                        float* y, float* h1, float* h2, hipStream_t st) {
  if (R <= 0) return;
  const int64_t nb = (R + RB - 1) / RB;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)nb), dim3(MLP_H), 0, st, R, X, W, bias,
                     y, h1, h2);
  BBTN_LAUNCHED("mlp forward");
}

void launch_mlp_backward(int64_t R, const uint16_t* X, const uint16_t* W, const float* y,
                         const float* t, const float* h1, const float* h2, float* part,
                         float* grad, hipStream_t st) {
  if (R <= 0) return;
  const int64_t nb = (R + RB - 1) / RB;
  hipLaunchKernelGGL(mlp_backward_kernel, dim3((unsigned)nb), dim3(MLP_H), 0, st, R, X, W, y, t,
                     h1, h2, part);
  BBTN_LAUNCHED("mlp backward");
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((MLP_NPART + 255) / 256), dim3(256), 0, st, nb, part,
                     grad);
  BBTN_LAUNCHED("mlp backward reduce");
}

int64_t mlp_partial_floats(int64_t R) { return ((R + RB - 1) / RB) * (int64_t)MLP_NPART; }

void launch_mlp_adam(float* master, uint16_t* wbf, float* bias, float* m, float* v,
                     const float* g, float lr, float b1, float b2, float eps, int step,
                     hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, master,
                     wbf, bias, m, v, g, lr, b1, b2, eps, c1, c2);
  BBTN_LAUNCHED("adam");
}

}  // namespace bbtn
