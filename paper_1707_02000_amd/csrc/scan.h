// Device-wide exclusive prefix sums over a count that may live on the device.
//
// Reduce-then-scan over a fixed grid of SCAN_BLOCKS workgroups: each block owns
// one contiguous chunk; pass 1 sums every chunk, pass 2 (one block) scans the
// chunk sums, pass 3 rescans each chunk from its offset.  The element values
// come from a functor F with
//   __device__ bool active() const;   // false: every pass returns at once
//   __device__ i64  count()  const;   // number of elements
//   __device__ i64  len(i64 i) const; // value of element i
// Output: out[i] = sum of len(0..i-1) for i in [0, count], so out[count] is the
// total.
#pragma once
#include "common.h"

#define SCAN_BLOCKS 1024

template <class F>
__global__ __launch_bounds__(PKT_BLOCK) void k_scan_reduce(F f, i64* __restrict__ partial) {
  if (!f.active()) return;
  const i64 count = f.count();
  const i64 chunk = (count + gridDim.x - 1) / gridDim.x;
  const i64 b0 = (i64)blockIdx.x * chunk;
  const i64 b1 = min(count, b0 + chunk);
  i64 s = 0;
  for (i64 i = b0 + threadIdx.x; i < b1; i += PKT_BLOCK) s += f.len(i);
  __shared__ i64 tmp[PKT_BLOCK / PKT_WAVE];
  s = wave_sum_i64(s);
  if (lane_id() == 0) tmp[threadIdx.x / PKT_WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    i64 t = 0;
    for (int w = 0; w < PKT_BLOCK / PKT_WAVE; ++w) t += tmp[w];
    partial[blockIdx.x] = t;
  }
}

// One block: exclusive scan of partial[0..nb) in place, partial[nb] = total.
template <class F>
__global__ __launch_bounds__(PKT_BLOCK) void k_scan_partials(F f, i64* __restrict__ partial, int nb) {
  if (!f.active()) return;
  __shared__ i64 tmp[PKT_BLOCK / PKT_WAVE];
  i64 running = 0;
  for (int base = 0; base < nb; base += PKT_BLOCK) {
    const int i = base + threadIdx.x;
    const i64 v = (i < nb) ? partial[i] : 0;
    i64 tot;
    const i64 ex = block_excl_scan_i64(v, tmp, &tot);
    if (i < nb) partial[i] = running + ex;
    running += tot;
  }
  if (threadIdx.x == 0) partial[nb] = running;
}

template <class F>
__global__ __launch_bounds__(PKT_BLOCK) void k_scan_down(F f, const i64* __restrict__ partial,
                                                        i64* __restrict__ out) {
  if (!f.active()) return;
  const i64 count = f.count();
  const i64 chunk = (count + gridDim.x - 1) / gridDim.x;
  const i64 b0 = (i64)blockIdx.x * chunk;
  const i64 b1 = min(count, b0 + chunk);
  __shared__ i64 tmp[PKT_BLOCK / PKT_WAVE];
  i64 running = partial[blockIdx.x];
  for (i64 t = b0; t < b1; t += PKT_BLOCK) {
    const i64 i = t + threadIdx.x;
    const i64 v = (i < b1) ? f.len(i) : 0;
    i64 tot;
    const i64 ex = block_excl_scan_i64(v, tmp, &tot);
    if (i < b1) out[i] = running + ex;
    running += tot;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[count] = partial[gridDim.x];
}

// Launches the three passes on `stream`.  partial needs SCAN_BLOCKS + 1 entries.
template <class F>
static inline hipError_t scan_launch(const F& f, i64* partial, i64* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_scan_reduce<F>, dim3(SCAN_BLOCKS), dim3(PKT_BLOCK), 0, stream, f, partial);
  hipLaunchKernelGGL(k_scan_partials<F>, dim3(1), dim3(PKT_BLOCK), 0, stream, f, partial, (int)SCAN_BLOCKS);
  hipLaunchKernelGGL(k_scan_down<F>, dim3(SCAN_BLOCKS), dim3(PKT_BLOCK), 0, stream, f, partial, out);
  return hipGetLastError();
}

// Functor over a plain array with a host-known count.
template <class T>
struct ArrayLen {
  const T* a;
  i64 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 i) const { return (i64)a[i]; }
};
