// Device-wide exclusive prefix sums over a count that may live on the device.
//
// Reduce-then-scan in two launches over a grid of up to SCAN_BLOCKS workgroups:
// the count is split into nb contiguous chunks of about SCAN_CHUNK elements
// (nb <= gridDim.x; blocks past nb return at once).  Pass 1 sums every chunk and
// its last-arriving block scans the chunk sums; pass 2 rescans each chunk from
// its offset.  The element values come from a functor F with
//   __device__ bool active() const;   // false: both passes return at once
//   __device__ i64  count()  const;   // number of elements
//   __device__ i64  len(i64 i) const; // value of element i
// Output: out[i] = sum of len(0..i-1) for i in [0, count], so out[count] is the
// total.  `arrive` is a zeroed counter the last block resets.  With CACHE, pass 1
// keeps every len(i) in out[i] and pass 2 reads it from there (the same thread
// reads and then overwrites each entry), for functors whose len is costly.
#pragma once
#include "common.h"

#define SCAN_BLOCKS 1024
#ifndef SCAN_CHUNK
#define SCAN_CHUNK 256  // elements per chunk below SCAN_BLOCKS chunks
#endif

__device__ __forceinline__ int scan_nblocks(i64 count) {
  i64 nb = (count + SCAN_CHUNK - 1) / SCAN_CHUNK;
  if (nb < 1) nb = 1;
  return (int)(nb < (i64)gridDim.x ? nb : (i64)gridDim.x);
}

template <class F, bool CACHE = false>
__global__ __launch_bounds__(PKT_BLOCK) void k_scan_reduce(F f, i64* __restrict__ partial, u32* __restrict__ arrive,
                                                          i64* __restrict__ out) {
  if (!f.active()) return;
  const i64 count = f.count();
  const int nb = scan_nblocks(count);
  if ((int)blockIdx.x >= nb) return;
  const i64 chunk = (count + nb - 1) / nb;
  const i64 b0 = (i64)blockIdx.x * chunk;
  const i64 b1 = min(count, b0 + chunk);
  i64 s = 0;
  for (i64 i = b0 + threadIdx.x; i < b1; i += PKT_BLOCK) {
    const i64 v = f.len(i);
    if (CACHE) out[i] = v;
    s += v;
  }
  __shared__ i64 tmp[PKT_BLOCK / PKT_WAVE];
  __shared__ int last;
  s = wave_sum_i64(s);
  if (lane_id() == 0) tmp[threadIdx.x / PKT_WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    i64 t = 0;
    for (int w = 0; w < PKT_BLOCK / PKT_WAVE; ++w) t += tmp[w];
    partial[blockIdx.x] = t;
    __threadfence();
    last = atomicAdd(arrive, 1u) == (u32)nb - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();  // every block's chunk sum is visible
  i64 running = 0;
  for (int base = 0; base < nb; base += PKT_BLOCK) {
    const int i = base + threadIdx.x;
    const i64 v = (i < nb) ? __hip_atomic_load(&partial[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    i64 tot;
    const i64 ex = block_excl_scan_i64(v, tmp, &tot);
    if (i < nb) partial[i] = running + ex;
    running += tot;
  }
  if (threadIdx.x == 0) {
    partial[nb] = running;
    *arrive = 0;
  }
}

template <class F, bool CACHE = false>
__global__ __launch_bounds__(PKT_BLOCK) void k_scan_down(F f, const i64* __restrict__ partial,
                                                        i64* __restrict__ out) {
  if (!f.active()) return;
  const i64 count = f.count();
  const int nb = scan_nblocks(count);
  if ((int)blockIdx.x >= nb) return;
  const i64 chunk = (count + nb - 1) / nb;
  const i64 b0 = (i64)blockIdx.x * chunk;
  const i64 b1 = min(count, b0 + chunk);
  __shared__ i64 tmp[PKT_BLOCK / PKT_WAVE];
  i64 running = partial[blockIdx.x];
  for (i64 t = b0; t < b1; t += PKT_BLOCK) {
    const i64 i = t + threadIdx.x;
    const i64 v = (i < b1) ? (CACHE ? out[i] : f.len(i)) : 0;
    i64 tot;
    const i64 ex = block_excl_scan_i64(v, tmp, &tot);
    if (i < b1) out[i] = running + ex;
    running += tot;
  }
  if ((int)blockIdx.x == nb - 1 && threadIdx.x == 0) out[count] = partial[nb];
}

template <class F, bool CACHE = false>
static inline hipError_t scan_launch(const F& f, i64* partial, i64* out, u32* arrive, hipStream_t stream) {
  hipLaunchKernelGGL((k_scan_reduce<F, CACHE>), dim3(SCAN_BLOCKS), dim3(PKT_BLOCK), 0, stream, f, partial, arrive,
                     out);
  hipLaunchKernelGGL((k_scan_down<F, CACHE>), dim3(SCAN_BLOCKS), dim3(PKT_BLOCK), 0, stream, f, partial, out);
  return hipGetLastError();
}

template <class T>
struct ArrayLen {
  const T* a;
  i64 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 i) const { return (i64)a[i]; }
};
