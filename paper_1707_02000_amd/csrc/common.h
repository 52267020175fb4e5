// Shared helpers of libpkt: types, error reporting, wave/block primitives for
// CDNA (wave64), workspace carving.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include "../../include/pkt.h"

typedef int64_t i64;
typedef int32_t i32;
typedef uint32_t u32;
typedef uint64_t u64;
typedef uint8_t u8;

#define PKT_WAVE 64
#define PKT_BLOCK 256  // 4 waves

// Edge states of the peeling (the paper's inCurr / inNext / processed): ST_ALIVE
// until the edge joins a frontier, then the tag of the round that processes it,
// three tags in rotation.  During round r an edge is current iff its tag is
// round_tag(r), joined the next frontier iff round_tag(r + 1), and processed iff
// ST_PROC or round_tag(r - 1): round r itself turns the round_tag(r - 1) edges
// (its previous frontier) into ST_PROC, so that tag is free again when round
// r + 1 hands it to its next frontier.  Ending a round is then a counter update,
// with no pass between rounds.
enum : u8 { ST_ALIVE = 0, ST_PROC = 1 };
__host__ __device__ __forceinline__ u8 round_tag(int r) { return (u8)(2 + (unsigned)r % 3u); }
__host__ __device__ __forceinline__ bool is_processed(u8 st, int r) {
  return st == ST_PROC || st == round_tag(r + 2);
}

// One 32-bit word per edge holds both its support and its state: the support in
// the upper 29 bits (two's complement, so the brief undershoot of a decrement
// that is then undone stays inside the field) and the state in the low 3.  A
// decrement subtracts SW_ONE and leaves the state bits alone; joining a frontier
// ORs a round tag into ST_ALIVE (zero) bits; retiring XORs the tag into ST_PROC.
// One load then answers both "is this edge processed" and "is its support above
// the level", where two arrays would cost two random lines.
#define SW_SHIFT 3
#define SW_ONE (1 << SW_SHIFT)
#define SW_MAX_SUPPORT ((1 << (31 - SW_SHIFT)) - 1)
__host__ __device__ __forceinline__ i32 sw_sup(i32 w) { return w >> SW_SHIFT; }
__host__ __device__ __forceinline__ u8 sw_st(i32 w) { return (u8)(w & (SW_ONE - 1)); }
__host__ __device__ __forceinline__ i32 sw_make(i32 sup, u8 st) { return (i32)((u32)sup << SW_SHIFT) | st; }

// Validation error bits.
enum : u32 { VERR_RANGE = 1u, VERR_NOT_SIMPLE = 2u, VERR_NOT_SYMMETRIC = 4u, VERR_DEGREE = 8u };

// ---------------------------------------------------------------- host errors
namespace pkt {
void set_error(const char* fmt, ...);
truss_status hip_fail(hipError_t e, const char* what, const char* file, int line);
}  // namespace pkt

#define PKT_HIP(call)                                                      \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) return pkt::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

#define PKT_LAUNCH_CHECK() PKT_HIP(hipGetLastError())

// ------------------------------------------------------------ device helpers

// First index in [lo, hi) with a[idx] >= x (hi if none).
template <class T, class I>
__device__ __forceinline__ I lower_bound_dev(const T* __restrict__ a, I lo, I hi, T x) {
  while (lo < hi) {
    I mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// First index in [lo, hi) with a[idx] > x (hi if none).
template <class T, class I>
__device__ __forceinline__ I upper_bound_dev(const T* __restrict__ a, I lo, I hi, T x) {
  while (lo < hi) {
    I mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (PKT_WAVE - 1)); }

// Wave-aggregated append: every lane with pred gets a distinct slot of
// out[*counter ...]; one atomic per wave.  Must be reached by all active lanes.
__device__ __forceinline__ i32 wave_append_slot(bool pred, i32* counter) {
  u64 mask = __ballot(pred);
  if (mask == 0) return -1;
  const int lane = lane_id();
  const int leader = __ffsll((unsigned long long)mask) - 1;
  i32 base = 0;
  if (lane == leader) base = atomicAdd(counter, (i32)__popcll(mask));
  base = __shfl(base, leader);
  return pred ? base + (i32)__popcll(mask & ((1ull << lane) - 1ull)) : -1;
}

__device__ __forceinline__ i64 wave_sum_i64(i64 v) {
  for (int o = PKT_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ i32 wave_min_i32(i32 v) {
  for (int o = PKT_WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ i32 wave_max_i32(i32 v) {
  for (int o = PKT_WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Inclusive scan within a wave.
__device__ __forceinline__ i64 wave_incl_scan_i64(i64 v) {
  const int lane = lane_id();
  for (int o = 1; o < PKT_WAVE; o <<= 1) {
    i64 y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  return v;
}

// Exclusive scan over a block of NT threads.  `tmp` is LDS of NT / PKT_WAVE
// entries.  Returns the exclusive prefix; *total gets the block sum.  All
// threads must call it.
template <int NT = PKT_BLOCK>
__device__ __forceinline__ i64 block_excl_scan_i64(i64 v, i64* tmp, i64* total) {
  const int lane = lane_id(), wid = threadIdx.x / PKT_WAVE;
  i64 inc = wave_incl_scan_i64(v);
  if (lane == PKT_WAVE - 1) tmp[wid] = inc;
  __syncthreads();
  i64 pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / PKT_WAVE; ++w) {
    i64 t = tmp[w];
    pre += (w < wid) ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__device__ __forceinline__ i32 atomic_load_relaxed(const i32* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ host helpers

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Sequential carving of one workspace buffer into 256-byte aligned pieces.
struct Carver {
  char* base;
  size_t used;
  explicit Carver(void* b) : base((char*)b), used(0) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? (T*)(base + used) : nullptr;
    used += align_up(count * sizeof(T) + 1, 256);
    return p;
  }
};
