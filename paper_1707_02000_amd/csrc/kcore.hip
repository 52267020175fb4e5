// Core numbers (k-core decomposition) by level-synchronous vertex peeling, the
// pattern the PKT section borrows for edges (the paper's related-work section on
// parallel k-core decomposition): the core number of v is the largest k such that
// v lies in the k-core, the maximal subgraph of minimum degree >= k.
//
// Level k: a scan of the alive vertices takes those of current degree k as the
// frontier (and finds the smallest degree above k, to skip empty levels).  Each
// round marks its frontier with core number k, then every frontier vertex takes
// one unit off each alive neighbour: the atomic's old value k + 1 puts the
// neighbour in the next frontier, an old value <= k is undone (the neighbour
// already sits at k), so a degree never drops below the level.  The level ends
// when a round finds no new vertex.  Frontier items are the adjacency slots of
// the frontier vertices, one lane each, located through a device-wide prefix of
// the row lengths (scan.h).  The host reads three counters per round.
#include <limits.h>

#include "common.h"
#include "scan.h"

namespace {

inline int kc_grid(i64 count) {
  const i64 g = (count + PKT_BLOCK - 1) / PKT_BLOCK;
  return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

struct KcCounters {
  i32 nfound, nkeep, minabove, nnext;
  u32 arrive, err;
};

// Degrees, unset core numbers, every vertex alive; offsets out of order or past
// the adjacency set the error flag (the rounds index adj through them).
__global__ __launch_bounds__(PKT_BLOCK) void k_kc_init(i32 n, i64 two_m, const i64* __restrict__ off,
                                                      i32* __restrict__ deg, i32* __restrict__ core,
                                                      i32* __restrict__ alive, KcCounters* cnt) {
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK) {
    const i64 b = off[v], e = off[v + 1];
    if (b < 0 || e < b || e > two_m || e - b > (i64)INT32_MAX) atomicOr(&cnt->err, 1u);
    deg[v] = (i32)(e - b);
    core[v] = -1;
    alive[v] = (i32)v;
  }
}

// Alive vertices of degree k -> frontier; of larger degree -> the next alive list.
__global__ __launch_bounds__(PKT_BLOCK) void k_kc_scan(i32 na, const i32* __restrict__ A, i32 k,
                                                      const i32* __restrict__ deg, i32* __restrict__ F,
                                                      i32* __restrict__ Aout, KcCounters* cnt) {
  i32 mn = INT_MAX;
  const i64 na_up = ((i64)na + PKT_WAVE - 1) / PKT_WAVE * PKT_WAVE;  // whole waves stay in the loop
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < na_up; i += (i64)gridDim.x * PKT_BLOCK) {
    const i32 v = i < na ? A[i] : -1;
    const i32 d = v >= 0 ? deg[v] : -1;
    const bool take = v >= 0 && d == k, keep = v >= 0 && d > k;
    if (keep) mn = min(mn, d);
    const i32 st = wave_append_slot(take, &cnt->nfound);
    if (take) F[st] = v;
    const i32 sk = wave_append_slot(keep, &cnt->nkeep);
    if (keep) Aout[sk] = v;
  }
  mn = wave_min_i32(mn);
  if (lane_id() == 0 && mn != INT_MAX) atomicMin(&cnt->minabove, mn);
}

__global__ __launch_bounds__(PKT_BLOCK) void k_kc_mark(i32 nf, const i32* __restrict__ F, i32 k,
                                                      i32* __restrict__ core) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < nf; i += (i64)gridDim.x * PKT_BLOCK) core[F[i]] = k;
}

// Row length of frontier vertex i, for the prefix over the round's items.
struct FrontierRows {
  const i32* F;
  const i64* off;
  i32 nf;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return nf; }
  __device__ i64 len(i64 i) const {
    const i32 u = F[i];
    return off[u + 1] - off[u];
  }
};

// One lane per adjacency slot of the frontier: the neighbour loses one unit if it
// is alive and above the level; reaching k + 1 -> k puts it in the next frontier.
__global__ __launch_bounds__(PKT_BLOCK) void k_kc_round(i32 n, i32 nf, const i32* __restrict__ F,
                                                       const i64* __restrict__ P, const i64* __restrict__ off,
                                                       const i32* __restrict__ adj, i32 k,
                                                       const i32* __restrict__ core, i32* __restrict__ deg,
                                                       i32* __restrict__ next, KcCounters* cnt) {
  const i64 total = P[nf];
  const i64 total_up = (total + PKT_WAVE - 1) / PKT_WAVE * PKT_WAVE;
  for (i64 g = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; g < total_up; g += (i64)gridDim.x * PKT_BLOCK) {
    bool join = false;
    i32 v = -1;
    if (g < total) {
      const i64 i = upper_bound_dev(P, (i64)0, (i64)nf + 1, g) - 1;
      const i32 u = F[i];
      v = adj[off[u] + (g - P[i])];
      if (v < 0 || v >= n) {  // checked before any use as an index
        atomicOr(&cnt->err, 1u);
        v = -1;
      } else if (core[v] < 0 && __hip_atomic_load(&deg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > k) {
        const i32 old = atomicSub(&deg[v], 1);
        if (old == k + 1)
          join = true;
        else if (old <= k)
          atomicAdd(&deg[v], 1);
      }
    }
    const i32 s = wave_append_slot(join, &cnt->nnext);
    if (join) next[s] = v;
  }
}

struct KcWork {
  i32* deg;
  i32* A[2];
  i32* F[2];
  i64* P;
  i64* partial;
  KcCounters* cnt;
};

size_t kc_layout(i32 n, void* ws, KcWork* w) {
  Carver cv(ws);
  KcWork t;
  t.deg = cv.take<i32>((size_t)n);
  for (int q = 0; q < 2; ++q) t.A[q] = cv.take<i32>((size_t)n);
  for (int q = 0; q < 2; ++q) t.F[q] = cv.take<i32>((size_t)n);
  t.P = cv.take<i64>((size_t)n + 1);
  t.partial = cv.take<i64>(SCAN_BLOCKS + 1);
  t.cnt = cv.take<KcCounters>(1);
  if (w) *w = t;
  return cv.used;
}

}  // namespace

extern "C" truss_status truss_kcore_workspace_bytes(int32_t n, size_t* bytes) {
  pkt::set_error("");
  if (n < 0 || bytes == nullptr) {
    pkt::set_error("bad arguments to truss_kcore_workspace_bytes");
    return TRUSS_E_ARG;
  }
  *bytes = kc_layout(n, nullptr, nullptr);
  return TRUSS_OK;
}

extern "C" truss_status truss_kcore(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* core,
                                    int32_t* max_core, void* workspace, size_t workspace_bytes, void* stream) {
  using namespace pkt;
  set_error("");
  if (n < 0 || (n > 0 && (offsets == nullptr || core == nullptr))) {
    set_error("bad n or NULL offsets / core");
    return TRUSS_E_ARG;
  }
  const size_t need = kc_layout(n, nullptr, nullptr);
  if (workspace == nullptr || workspace_bytes < need || ((uintptr_t)workspace & 255u)) {
    set_error("workspace: need %zu bytes at 256-byte alignment", need);
    return TRUSS_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  if (max_core) *max_core = 0;
  if (n == 0) return TRUSS_OK;
  i64 two_m = 0;
  PKT_HIP(hipMemcpyAsync(&two_m, offsets + n, sizeof(i64), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (two_m < 0 || (two_m > 0 && adj == nullptr)) {
    set_error("offsets[n] = %lld is negative, or NULL adj", (long long)two_m);
    return two_m < 0 ? TRUSS_E_RANGE : TRUSS_E_ARG;
  }
  KcWork w;
  kc_layout(n, workspace, &w);
  PKT_HIP(hipMemsetAsync(w.cnt, 0, sizeof(KcCounters), s));
  hipLaunchKernelGGL(k_kc_init, dim3(kc_grid(n)), dim3(PKT_BLOCK), 0, s, n, two_m, offsets, w.deg, core, w.A[0],
                     w.cnt);
  PKT_LAUNCH_CHECK();
  u32 err = 0;
  PKT_HIP(hipMemcpyAsync(&err, &w.cnt->err, sizeof(u32), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (err) {
    set_error("input CSR: offsets out of order or past offsets[n]");
    return TRUSS_E_RANGE;
  }
  i32 na = n, asel = 0, k = 0, kmax = 0;
  i64 guard = 0;
  KcCounters hc;
  while (na > 0) {
    if (++guard > (i64)n + 2) {  // every level either finds a vertex or jumps to a larger degree
      set_error("k-core level bound exceeded");
      return TRUSS_E_INTERNAL;
    }
    // level scan: the frontier and the vertices left
    KcCounters z = {0, 0, INT_MAX, 0, 0, 0};
    PKT_HIP(hipMemcpyAsync(w.cnt, &z, sizeof(z), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_kc_scan, dim3(kc_grid(na)), dim3(PKT_BLOCK), 0, s, na, (const i32*)w.A[asel], k,
                       (const i32*)w.deg, w.F[0], w.A[asel ^ 1], w.cnt);
    PKT_LAUNCH_CHECK();
    PKT_HIP(hipMemcpyAsync(&hc, w.cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    na = hc.nkeep;
    asel ^= 1;
    if (hc.nfound == 0) {
      if (na > 0) k = hc.minabove;  // no vertex at this level: skip to the smallest degree left
      continue;
    }
    // rounds of the level
    i32 nf = hc.nfound, fsel = 0;
    while (nf > 0) {
      if (++guard > 4 * (i64)n + 8) {
        set_error("k-core round bound exceeded");
        return TRUSS_E_INTERNAL;
      }
      hipLaunchKernelGGL(k_kc_mark, dim3(kc_grid(nf)), dim3(PKT_BLOCK), 0, s, nf, (const i32*)w.F[fsel], k, core);
      PKT_HIP(scan_launch(FrontierRows{w.F[fsel], offsets, nf}, w.partial, w.P, &w.cnt->arrive, s));
      i64 items = 0;
      PKT_HIP(hipMemcpyAsync(&items, w.P + nf, sizeof(i64), hipMemcpyDeviceToHost, s));
      i32 zero = 0;
      PKT_HIP(hipMemcpyAsync(&w.cnt->nnext, &zero, sizeof(i32), hipMemcpyHostToDevice, s));
      PKT_HIP(hipStreamSynchronize(s));
      if (items > 0)
        hipLaunchKernelGGL(k_kc_round, dim3(kc_grid(items)), dim3(PKT_BLOCK), 0, s, n, nf, (const i32*)w.F[fsel],
                           (const i64*)w.P, offsets, adj, k, (const i32*)core, w.deg, w.F[fsel ^ 1], w.cnt);
      PKT_LAUNCH_CHECK();
      i32 nn = 0;
      PKT_HIP(hipMemcpyAsync(&nn, &w.cnt->nnext, sizeof(i32), hipMemcpyDeviceToHost, s));
      PKT_HIP(hipMemcpyAsync(&err, &w.cnt->err, sizeof(u32), hipMemcpyDeviceToHost, s));
      PKT_HIP(hipStreamSynchronize(s));
      if (err) {
        set_error("input CSR: a neighbour id outside [0, n)");
        return TRUSS_E_RANGE;
      }
      kmax = k;
      nf = nn;
      fsel ^= 1;
    }
    k += 1;
  }
  if (max_core) *max_core = kmax;
  return TRUSS_OK;
}
