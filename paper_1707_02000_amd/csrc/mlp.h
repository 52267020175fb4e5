// The cost model: a small fp32 MLP, MLP_IN features -> 3 hidden layers of
// MLP_H (ReLU) -> one predicted log2(microseconds) per launch choice.
//
// Parameter layout (floats, contiguous):
//   mu[IN], sigma[IN]          feature normalisation: x' = (x - mu) / sigma
//   W1[H][IN], b1[H]
//   W2[H][H],  b2[H]
//   W3[H][H],  b3[H]
//   W4[OUT][H], b4[OUT]
#pragma once
#include "common.h"

// The learned decision departs from the heuristic's launch only when the model
// predicts the other launch at least 10 % faster: log2(1.1) in the model's units
// (log2 microseconds).  Near the heuristic's threshold the two launches cost about
// the same and the model's error would otherwise flip them back and forth.
#ifndef MLP_MARGIN
#define MLP_MARGIN 0.13750352f
#endif

#define MLP_IN 6
#define MLP_H 64
#define MLP_OUT TRUSS_MODEL_CHOICES

#define MLP_OFF_MU 0
#define MLP_OFF_SIG (MLP_OFF_MU + MLP_IN)
#define MLP_OFF_W1 (MLP_OFF_SIG + MLP_IN)
#define MLP_OFF_B1 (MLP_OFF_W1 + MLP_H * MLP_IN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_H)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_H * MLP_H)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_H)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_H * MLP_H)
#define MLP_OFF_W4 (MLP_OFF_B3 + MLP_H)
#define MLP_OFF_B4 (MLP_OFF_W4 + MLP_OUT * MLP_H)
#define MLP_NPARAM (MLP_OFF_B4 + MLP_OUT)

// Forward pass of one feature vector by one block (blockDim.x >= MLP_H).
// x: raw features (LDS or registers of thread 0 copied to LDS), y: outputs
// (LDS, MLP_OUT), ha/hb: LDS scratch of MLP_H floats each.  All threads call it.
// Unit j walks its inputs from i = j (rotated): at every step the units of a wave
// read weights j * MLP_H + (i + j) % MLP_H, which fall in distinct LDS banks,
// where the plain order (every unit reading column i at once, a stride of
// MLP_H words) hits a single bank.
__device__ __forceinline__ void mlp_forward_block(const float* __restrict__ W, const float* x, float* y, float* ha,
                                                  float* hb) {
  const int j = threadIdx.x;
  if (j < MLP_H) {
    float s = W[MLP_OFF_B1 + j];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) {
      const float xn = (x[i] - W[MLP_OFF_MU + i]) / W[MLP_OFF_SIG + i];
      s = fmaf(W[MLP_OFF_W1 + j * MLP_IN + i], xn, s);
    }
    ha[j] = fmaxf(s, 0.f);
  }
  __syncthreads();
  if (j < MLP_H) {
    float s = W[MLP_OFF_B2 + j];
#pragma unroll 8
    for (int k = 0; k < MLP_H; ++k) {
      const int i = (k + j) & (MLP_H - 1);
      s = fmaf(W[MLP_OFF_W2 + j * MLP_H + i], ha[i], s);
    }
    hb[j] = fmaxf(s, 0.f);
  }
  __syncthreads();
  if (j < MLP_H) {
    float s = W[MLP_OFF_B3 + j];
#pragma unroll 8
    for (int k = 0; k < MLP_H; ++k) {
      const int i = (k + j) & (MLP_H - 1);
      s = fmaf(W[MLP_OFF_W3 + j * MLP_H + i], hb[i], s);
    }
    ha[j] = fmaxf(s, 0.f);
  }
  __syncthreads();
  if (j < MLP_OUT) {
    float s = W[MLP_OFF_B4 + j];
#pragma unroll 8
    for (int k = 0; k < MLP_H; ++k) {
      const int i = (k + j) & (MLP_H - 1);
      s = fmaf(W[MLP_OFF_W4 + j * MLP_H + i], ha[i], s);
    }
    y[j] = s;
  }
  __syncthreads();
}
