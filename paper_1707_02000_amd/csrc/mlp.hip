// Training and batched inference of the launch cost model (mlp.h).
//
// The model maps a frontier's features to the predicted log2(device
// microseconds) of every launch choice; it is fitted by masked mean squared
// error (only choices measured for a frontier count) with Adam, all on the GPU.
// The layers are 64 wide and the data a few thousand rows, so plain tiled FMA
// kernels suffice; nothing here is on the decomposition's critical path except
// mlp_forward_block, which the peeling loop calls when the learned policy is on.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "mlp.h"
#include "peel.h"

namespace {

#define GT 16  // GEMM tile

// C[M][N] = alpha * sum_k A(m,k) B(k,n) + beta * C, row-major;
// A(m,k) = tA ? A[k*lda + m] : A[m*lda + k], B(k,n) = tB ? B[n*ldb + k] : B[k*ldb + n].
__global__ __launch_bounds__(GT* GT) void k_gemm(int M, int N, int K, const float* __restrict__ A, int lda, int tA,
                                                 const float* __restrict__ B, int ldb, int tB, float* __restrict__ C,
                                                 int ldc, float alpha, float beta) {
  __shared__ float As[GT][GT + 1];
  __shared__ float Bs[GT][GT + 1];
  const int tx = threadIdx.x % GT, ty = threadIdx.x / GT;
  const int row = blockIdx.y * GT + ty, col = blockIdx.x * GT + tx;
  float acc = 0.f;
  for (int k0 = 0; k0 < K; k0 += GT) {
    const int ka = k0 + tx, kb = k0 + ty;
    float av = 0.f, bv = 0.f;
    if (row < M && ka < K) av = tA ? A[(size_t)ka * lda + row] : A[(size_t)row * lda + ka];
    if (col < N && kb < K) bv = tB ? B[(size_t)col * ldb + kb] : B[(size_t)kb * ldb + col];
    As[ty][tx] = av;
    Bs[ty][tx] = bv;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GT; ++k) acc = fmaf(As[ty][k], Bs[k][tx], acc);
    __syncthreads();
  }
  if (row < M && col < N) {
    float* c = &C[(size_t)row * ldc + col];
    *c = alpha * acc + (beta != 0.f ? beta * *c : 0.f);
  }
}

// Xn = (X - mu) / sigma
__global__ void k_normalize(const float* __restrict__ X, const float* __restrict__ W, float* __restrict__ Xn, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * MLP_IN; i += gridDim.x * blockDim.x) {
    const int f = i % MLP_IN;
    Xn[i] = (X[i] - W[MLP_OFF_MU + f]) / W[MLP_OFF_SIG + f];
  }
}

// H = act(Z + b) in place (Z already holds the product); act = ReLU or identity.
__global__ void k_bias_act(float* __restrict__ Z, const float* __restrict__ b, int n, int cols, int relu) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n * cols; i += gridDim.x * blockDim.x) {
    const float z = Z[i] + b[i % cols];
    Z[i] = relu ? fmaxf(z, 0.f) : z;
  }
}

// cnt = sum(M) (one block)
__global__ void k_mask_count(const float* __restrict__ Mk, int total, float* __restrict__ cnt) {
  __shared__ float part[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < total; i += blockDim.x) s += Mk[i] != 0.f ? 1.f : 0.f;
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *cnt = fmaxf(part[0], 1.f);
}

// dY = 2 M (Y - T) / cnt; loss += sum M (Y - T)^2 / cnt
__global__ void k_loss_grad(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ Mk,
                            int total, const float* __restrict__ cnt, float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float part[256];
  const float inv = 1.f / *cnt;
  float s = 0.f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const float d = Mk[i] != 0.f ? (Y[i] - T[i]) : 0.f;
    dY[i] = 2.f * d * inv;
    s += d * d * inv;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) atomicAdd(loss, part[0]);
}

// dZ = dH * (H > 0), in place on dH
__global__ void k_relu_back(float* __restrict__ dH, const float* __restrict__ H, int total) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x)
    if (!(H[i] > 0.f)) dH[i] = 0.f;
}

// db[j] = sum_i dZ[i][j] (one block per column)
__global__ void k_col_sum(const float* __restrict__ dZ, int n, int cols, float* __restrict__ db) {
  __shared__ float part[256];
  const int j = blockIdx.x;
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += dZ[(size_t)i * cols + j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = part[0];
}

// Adam on the trainable parameters [MLP_OFF_W1, MLP_NPARAM).
__global__ void k_adam(float* __restrict__ W, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int i = MLP_OFF_W1 + blockIdx.x * blockDim.x + threadIdx.x; i < MLP_NPARAM; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_fill_f32(float* __restrict__ a, int n, float x) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = x;
}

__device__ __forceinline__ float hash_uniform(unsigned long long seed, unsigned long long i) {
  unsigned long long z = seed + 0x9e3779b97f4a7c15ULL * (i + 1);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return (float)((z >> 40) * (1.0 / 16777216.0)) * 2.f - 1.f;  // [-1, 1)
}

// Initialisation: feature normalisation from X (mean, standard deviation;
// sigma >= 1e-3), layers uniform in +-1/sqrt(fan_in), hidden biases zero, output
// biases the mean measured target of each choice.  One block.
__global__ void k_mlp_init(const float* __restrict__ X, const float* __restrict__ T, const float* __restrict__ Mk, int n,
                           unsigned long long seed, float* __restrict__ W) {
  __shared__ double acc[2][MLP_IN];
  __shared__ double tacc[2][MLP_OUT];
  if (threadIdx.x < MLP_IN) acc[0][threadIdx.x] = acc[1][threadIdx.x] = 0.0;
  if (threadIdx.x < MLP_OUT) tacc[0][threadIdx.x] = tacc[1][threadIdx.x] = 0.0;
  __syncthreads();
  if (threadIdx.x < MLP_IN) {
    double s = 0.0, ss = 0.0;
    for (int i = 0; i < n; ++i) {
      const double x = X[(size_t)i * MLP_IN + threadIdx.x];
      s += x;
      ss += x * x;
    }
    const double mean = n ? s / n : 0.0;
    const double var = n ? ss / n - mean * mean : 1.0;
    W[MLP_OFF_MU + threadIdx.x] = (float)mean;
    W[MLP_OFF_SIG + threadIdx.x] = (float)fmax(sqrt(fmax(var, 0.0)), 1e-3);
  } else if (threadIdx.x >= 64 && threadIdx.x < 64 + MLP_OUT) {
    const int k = threadIdx.x - 64;
    double s = 0.0, c = 0.0;
    for (int i = 0; i < n; ++i)
      if (Mk[(size_t)i * MLP_OUT + k] != 0.f) {
        s += T[(size_t)i * MLP_OUT + k];
        c += 1.0;
      }
    W[MLP_OFF_B4 + k] = (float)(c > 0 ? s / c : 0.0);
  }
  for (int i = MLP_OFF_W1 + threadIdx.x; i < MLP_OFF_B4; i += blockDim.x) {
    float scale = 0.f;
    if (i < MLP_OFF_B1) scale = rsqrtf((float)MLP_IN);
    else if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) scale = rsqrtf((float)MLP_H);
    else if (i >= MLP_OFF_W3 && i < MLP_OFF_B3) scale = rsqrtf((float)MLP_H);
    else if (i >= MLP_OFF_W4 && i < MLP_OFF_B4) scale = rsqrtf((float)MLP_H);
    W[i] = scale * hash_uniform(seed, (unsigned long long)i);
  }
}

// Batched decisions with the peeling loop's own inference and decision routines:
// one block per row.
__global__ __launch_bounds__(MLP_H) void k_mlp_choose(const float* __restrict__ X, const i32* __restrict__ ncurr, int n,
                                                      const float* __restrict__ W, i32* __restrict__ choice,
                                                      float* __restrict__ Y) {
  __shared__ float sx[MLP_IN], sy[MLP_OUT], ha[MLP_H], hb[MLP_H];
  for (int r = blockIdx.x; r < n; r += gridDim.x) {
    if (threadIdx.x < MLP_IN) sx[threadIdx.x] = X[(size_t)r * MLP_IN + threadIdx.x];
    __syncthreads();
    mlp_forward_block(W, sx, sy, ha, hb);
    if (threadIdx.x == 0) {
      for (int k = 0; k < MLP_OUT; ++k)
        if (Y) Y[(size_t)r * MLP_OUT + k] = sy[k];
      choice[r] = mlp_decide(sy, ncurr[r]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ host helpers

struct Acts {
  float *Xn, *H1, *H2, *H3, *Y, *dY, *dA, *dB, *cnt, *grad, *m, *v;
};

size_t acts_layout(int n, void* base, Acts* a) {
  Carver cv(base);
  Acts t;
  t.Xn = cv.take<float>((size_t)n * MLP_IN);
  t.H1 = cv.take<float>((size_t)n * MLP_H);
  t.H2 = cv.take<float>((size_t)n * MLP_H);
  t.H3 = cv.take<float>((size_t)n * MLP_H);
  t.Y = cv.take<float>((size_t)n * MLP_OUT);
  t.dY = cv.take<float>((size_t)n * MLP_OUT);
  t.dA = cv.take<float>((size_t)n * MLP_H);
  t.dB = cv.take<float>((size_t)n * MLP_H);
  t.cnt = cv.take<float>(2);
  t.grad = cv.take<float>(MLP_NPARAM);
  t.m = cv.take<float>(MLP_NPARAM);
  t.v = cv.take<float>(MLP_NPARAM);
  if (a) *a = t;
  return cv.used;
}

inline dim3 gemm_grid(int M, int N) { return dim3((N + GT - 1) / GT, (M + GT - 1) / GT); }
inline int ew_grid(long long total) { return (int)std::min<long long>(1024, (total + 255) / 256 + 1); }

void gemm(hipStream_t s, int M, int N, int K, const float* A, int lda, int tA, const float* B, int ldb, int tB,
          float* C, int ldc, float alpha, float beta) {
  hipLaunchKernelGGL(k_gemm, gemm_grid(M, N), dim3(GT * GT), 0, s, M, N, K, A, lda, tA, B, ldb, tB, C, ldc, alpha, beta);
}

// Forward pass keeping the activations.
void forward(hipStream_t s, const float* X, int n, const float* W, const Acts& a) {
  hipLaunchKernelGGL(k_normalize, dim3(ew_grid((long long)n * MLP_IN)), dim3(256), 0, s, X, W, a.Xn, n);
  gemm(s, n, MLP_H, MLP_IN, a.Xn, MLP_IN, 0, W + MLP_OFF_W1, MLP_IN, 1, a.H1, MLP_H, 1.f, 0.f);
  hipLaunchKernelGGL(k_bias_act, dim3(ew_grid((long long)n * MLP_H)), dim3(256), 0, s, a.H1, W + MLP_OFF_B1, n, MLP_H, 1);
  gemm(s, n, MLP_H, MLP_H, a.H1, MLP_H, 0, W + MLP_OFF_W2, MLP_H, 1, a.H2, MLP_H, 1.f, 0.f);
  hipLaunchKernelGGL(k_bias_act, dim3(ew_grid((long long)n * MLP_H)), dim3(256), 0, s, a.H2, W + MLP_OFF_B2, n, MLP_H, 1);
  gemm(s, n, MLP_H, MLP_H, a.H2, MLP_H, 0, W + MLP_OFF_W3, MLP_H, 1, a.H3, MLP_H, 1.f, 0.f);
  hipLaunchKernelGGL(k_bias_act, dim3(ew_grid((long long)n * MLP_H)), dim3(256), 0, s, a.H3, W + MLP_OFF_B3, n, MLP_H, 1);
  gemm(s, n, MLP_OUT, MLP_H, a.H3, MLP_H, 0, W + MLP_OFF_W4, MLP_H, 1, a.Y, MLP_OUT, 1.f, 0.f);
  hipLaunchKernelGGL(k_bias_act, dim3(ew_grid((long long)n * MLP_OUT)), dim3(256), 0, s, a.Y, W + MLP_OFF_B4, n, MLP_OUT,
                     0);
}

// Loss and gradient (into a.grad; mu and sigma get zero).  loss (device) is
// overwritten when non-NULL.
void backward(hipStream_t s, const float* T, const float* Mk, int n, const float* W, const Acts& a, float* loss) {
  hipLaunchKernelGGL(k_fill_f32, dim3(ew_grid(MLP_NPARAM)), dim3(256), 0, s, a.grad, (int)MLP_NPARAM, 0.f);
  if (loss) hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(1), 0, s, loss, 1, 0.f);
  hipLaunchKernelGGL(k_mask_count, dim3(1), dim3(256), 0, s, Mk, n * MLP_OUT, a.cnt);
  hipLaunchKernelGGL(k_loss_grad, dim3(ew_grid((long long)n * MLP_OUT)), dim3(256), 0, s, a.Y, T, Mk, n * MLP_OUT,
                     (const float*)a.cnt, a.dY, loss);
  float* g = a.grad;
  // output layer: dW4 = dY^T H3, db4 = colsum dY, dH3 = dY W4
  gemm(s, MLP_OUT, MLP_H, n, a.dY, MLP_OUT, 1, a.H3, MLP_H, 0, g + MLP_OFF_W4, MLP_H, 1.f, 0.f);
  hipLaunchKernelGGL(k_col_sum, dim3(MLP_OUT), dim3(256), 0, s, a.dY, n, MLP_OUT, g + MLP_OFF_B4);
  gemm(s, n, MLP_H, MLP_OUT, a.dY, MLP_OUT, 0, W + MLP_OFF_W4, MLP_H, 0, a.dA, MLP_H, 1.f, 0.f);
  // layer 3
  hipLaunchKernelGGL(k_relu_back, dim3(ew_grid((long long)n * MLP_H)), dim3(256), 0, s, a.dA, a.H3, n * MLP_H);
  gemm(s, MLP_H, MLP_H, n, a.dA, MLP_H, 1, a.H2, MLP_H, 0, g + MLP_OFF_W3, MLP_H, 1.f, 0.f);
  hipLaunchKernelGGL(k_col_sum, dim3(MLP_H), dim3(256), 0, s, a.dA, n, MLP_H, g + MLP_OFF_B3);
  gemm(s, n, MLP_H, MLP_H, a.dA, MLP_H, 0, W + MLP_OFF_W3, MLP_H, 0, a.dB, MLP_H, 1.f, 0.f);
  // layer 2
  hipLaunchKernelGGL(k_relu_back, dim3(ew_grid((long long)n * MLP_H)), dim3(256), 0, s, a.dB, a.H2, n * MLP_H);
  gemm(s, MLP_H, MLP_H, n, a.dB, MLP_H, 1, a.H1, MLP_H, 0, g + MLP_OFF_W2, MLP_H, 1.f, 0.f);
  hipLaunchKernelGGL(k_col_sum, dim3(MLP_H), dim3(256), 0, s, a.dB, n, MLP_H, g + MLP_OFF_B2);
  gemm(s, n, MLP_H, MLP_H, a.dB, MLP_H, 0, W + MLP_OFF_W2, MLP_H, 0, a.dA, MLP_H, 1.f, 0.f);
  // layer 1
  hipLaunchKernelGGL(k_relu_back, dim3(ew_grid((long long)n * MLP_H)), dim3(256), 0, s, a.dA, a.H1, n * MLP_H);
  gemm(s, MLP_H, MLP_IN, n, a.dA, MLP_H, 1, a.Xn, MLP_IN, 0, g + MLP_OFF_W1, MLP_IN, 1.f, 0.f);
  hipLaunchKernelGGL(k_col_sum, dim3(MLP_H), dim3(256), 0, s, a.dA, n, MLP_H, g + MLP_OFF_B1);
}

}  // namespace

using namespace pkt;

extern "C" {

int32_t truss_mlp_num_params(void) { return MLP_NPARAM; }

size_t truss_mlp_workspace_bytes(int32_t n) { return n < 0 ? 0 : acts_layout(n, nullptr, nullptr); }

truss_status truss_mlp_init(const float* X, const float* T, const float* M, int32_t n, uint64_t seed,
                            float* weights, void* stream) {
  set_error("");
  if (n < 0 || (n > 0 && (!X || !T || !M)) || !weights) {
    set_error("bad arguments to truss_mlp_init");
    return TRUSS_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mlp_init, dim3(1), dim3(256), 0, s, X, T, M, n, (unsigned long long)seed, weights);
  PKT_LAUNCH_CHECK();
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

truss_status truss_mlp_forward(const float* X, int32_t n, const float* weights, float* Y, void* workspace,
                               size_t workspace_bytes, void* stream) {
  set_error("");
  if (n < 0 || (n > 0 && (!X || !Y)) || !weights) {
    set_error("bad arguments to truss_mlp_forward");
    return TRUSS_E_ARG;
  }
  if (n == 0) return TRUSS_OK;
  if (!workspace || workspace_bytes < acts_layout(n, nullptr, nullptr) || ((uintptr_t)workspace & 255u)) {
    set_error("workspace too small or misaligned");
    return TRUSS_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Acts a;
  acts_layout(n, workspace, &a);
  forward(s, X, n, weights, a);
  PKT_HIP(hipMemcpyAsync(Y, a.Y, sizeof(float) * (size_t)n * MLP_OUT, hipMemcpyDeviceToDevice, s));
  PKT_LAUNCH_CHECK();
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

truss_status truss_mlp_gradient(const float* X, const float* T, const float* M, int32_t n, const float* weights,
                                float* grad, float* loss, void* workspace, size_t workspace_bytes, void* stream) {
  set_error("");
  if (n <= 0 || !X || !T || !M || !weights || !grad) {
    set_error("bad arguments to truss_mlp_gradient");
    return TRUSS_E_ARG;
  }
  if (!workspace || workspace_bytes < acts_layout(n, nullptr, nullptr) || ((uintptr_t)workspace & 255u)) {
    set_error("workspace too small or misaligned");
    return TRUSS_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Acts a;
  acts_layout(n, workspace, &a);
  forward(s, X, n, weights, a);
  backward(s, T, M, n, weights, a, loss);
  PKT_HIP(hipMemcpyAsync(grad, a.grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, s));
  PKT_LAUNCH_CHECK();
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

truss_status truss_mlp_train(const float* X, const float* T, const float* M, int32_t n, float* weights, int32_t steps,
                             float lr, float* loss_history, void* workspace, size_t workspace_bytes, void* stream) {
  set_error("");
  if (n <= 0 || !X || !T || !M || !weights || steps < 0 || !(lr > 0.f)) {
    set_error("bad arguments to truss_mlp_train");
    return TRUSS_E_ARG;
  }
  if (!workspace || workspace_bytes < acts_layout(n, nullptr, nullptr) || ((uintptr_t)workspace & 255u)) {
    set_error("workspace too small or misaligned");
    return TRUSS_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  Acts a;
  acts_layout(n, workspace, &a);
  hipLaunchKernelGGL(k_fill_f32, dim3(ew_grid(MLP_NPARAM)), dim3(256), 0, s, a.m, (int)MLP_NPARAM, 0.f);
  hipLaunchKernelGGL(k_fill_f32, dim3(ew_grid(MLP_NPARAM)), dim3(256), 0, s, a.v, (int)MLP_NPARAM, 0.f);
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  double c1 = 1.0, c2 = 1.0;
  for (int t = 0; t < steps; ++t) {
    forward(s, X, n, weights, a);
    backward(s, T, M, n, weights, a, loss_history ? loss_history + t : nullptr);
    c1 *= b1;
    c2 *= b2;
    hipLaunchKernelGGL(k_adam, dim3(ew_grid(MLP_NPARAM)), dim3(256), 0, s, weights, (const float*)a.grad, a.m, a.v,
                       lr, b1, b2, eps, (float)(1.0 - c1), (float)(1.0 - c2));
  }
  PKT_LAUNCH_CHECK();
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

truss_status truss_mlp_choose(const float* X, const int32_t* ncurr, int32_t n, const float* weights, int32_t* choice,
                              float* Y, void* stream) {
  set_error("");
  if (n < 0 || (n > 0 && (!X || !ncurr || !choice)) || !weights) {
    set_error("bad arguments to truss_mlp_choose");
    return TRUSS_E_ARG;
  }
  if (n == 0) return TRUSS_OK;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_mlp_choose, dim3(std::min(n, 4096)), dim3(MLP_H), 0, s, X, ncurr, n, weights, choice, Y);
  PKT_LAUNCH_CHECK();
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

}  // extern "C"
