// Layout of the learned branching scorer (32 -> 128 -> 128 -> 1, ReLU).
#pragma once
#include "common.h"

namespace bbtn {

constexpr int MLP_IN = 32, MLP_H = 128;
// bfloat16 weight buffer: W1 [128][32], W2 [128][128], w3 [128]
constexpr int MLP_W1 = 0;
constexpr int MLP_W2 = MLP_W1 + MLP_H * MLP_IN;
constexpr int MLP_W3 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_NW = MLP_W3 + MLP_H;
// float32 bias buffer: b1 [128], b2 [128], b3
constexpr int MLP_B1 = 0;
constexpr int MLP_B2 = MLP_B1 + MLP_H;
constexpr int MLP_B3 = MLP_B2 + MLP_H;
constexpr int MLP_NB = MLP_B3 + 1;
// packed float32 parameters / gradients: [weights][biases]; partials add the
// sum of squared errors at the end
constexpr int MLP_NPARAM = MLP_NW + MLP_NB;
constexpr int MLP_NPART = MLP_NPARAM + 1;

void launch_mlp_forward(int64_t R, const uint16_t* X, const uint16_t* W, const float* bias,
                        float* y, float* h1, float* h2, hipStream_t st);
void launch_mlp_backward(int64_t R, const uint16_t* X, const uint16_t* W, const float* y,
                         const float* t, const float* h1, const float* h2, float* part,
                         float* grad, hipStream_t st);
int64_t mlp_partial_floats(int64_t R);
void launch_mlp_adam(float* master, uint16_t* wbf, float* bias, float* m, float* v,
                     const float* g, float lr, float b1, float b2, float eps, int step,
                     hipStream_t st);

}  // namespace bbtn
