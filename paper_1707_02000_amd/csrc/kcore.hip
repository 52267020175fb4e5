// Core numbers (k-core decomposition) by level-synchronous vertex peeling, the
// pattern the PKT section borrows for edges (the Background section's passage on
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
// the row lengths (scan.h).  The host reads the counters once per round and once
// per level scan.
#include <limits.h>

#include "common.h"
#include "launch.h"
#include "scan.h"

namespace {

struct KcCounters {
  i32 nfound, nkeep, minabove;
  i32 nnext[2];  // next-frontier sizes of alternate rounds
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
// A block takes KC_TILE entries (KC_PER per thread, coalesced) and reserves its
// places in both lists with one atomic each: per-wave reservations on two
// counters that every wave of a million-vertex scan hits serialised the scan.
constexpr int KC_PER = 8;
constexpr int KC_TILE = KC_PER * PKT_BLOCK;

__global__ __launch_bounds__(PKT_BLOCK) void k_kc_scan(i32 na, const i32* __restrict__ A, i32 k,
                                                      const i32* __restrict__ deg, i32* __restrict__ F,
                                                      i32* __restrict__ Aout, KcCounters* cnt) {
  __shared__ i64 tmp[PKT_BLOCK / PKT_WAVE];
  __shared__ i32 base[2];
  i32 mn = INT_MAX;
  const i64 tiles = ((i64)na + KC_TILE - 1) / KC_TILE;
  for (i64 t = blockIdx.x; t < tiles; t += gridDim.x) {  // uniform over the block
    i32 v[KC_PER];
    u32 take = 0, keep = 0;
    i32 ct = 0, ck = 0;
#pragma unroll
    for (int j = 0; j < KC_PER; ++j) {
      const i64 i = t * KC_TILE + j * PKT_BLOCK + threadIdx.x;
      v[j] = i < na ? A[i] : -1;
      const i32 d = v[j] >= 0 ? deg[v[j]] : -1;
      if (d == k) {
        take |= 1u << j;
        ++ct;
      } else if (d > k) {
        keep |= 1u << j;
        ++ck;
        mn = min(mn, d);
      }
    }
    i64 tot;
    const i64 pre = block_excl_scan_i64(((i64)ct << 32) | (i64)ck, tmp, &tot);
    if (threadIdx.x == 0) {
      const i32 tt = (i32)(tot >> 32), tk = (i32)(tot & 0xffffffff);
      base[0] = tt ? atomicAdd(&cnt->nfound, tt) : 0;
      base[1] = tk ? atomicAdd(&cnt->nkeep, tk) : 0;
    }
    __syncthreads();
    i32 pt = base[0] + (i32)(pre >> 32), pk = base[1] + (i32)(pre & 0xffffffff);
#pragma unroll
    for (int j = 0; j < KC_PER; ++j) {
      if (take >> j & 1u) F[pt++] = v[j];
      if (keep >> j & 1u) Aout[pk++] = v[j];
    }
    __syncthreads();  // base[] is rewritten by the next tile
  }
  mn = wave_min_i32(mn);
  if (lane_id() == 0 && mn != INT_MAX) atomicMin(&cnt->minabove, mn);
}

// Level counters back to their start (the error flag stays).
__global__ void k_kc_reset(KcCounters* cnt) {
  cnt->nfound = 0;
  cnt->nkeep = 0;
  cnt->minabove = INT_MAX;
  cnt->nnext[0] = 0;
  cnt->nnext[1] = 0;
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

// One lane per adjacency slot of the frontier: the neighbour loses one unit if its
// degree is above the level; reaching k + 1 -> k puts it in the next frontier.
// Vertices of this or an earlier level sit at or below k and are never touched,
// so the degree test alone keeps them out.  The first nf lanes also mark the
// frontier with k.  The round appends to nnext[sel] and clears nnext[sel ^ 1] for
// the round after it (the host has read that one already).
__global__ __launch_bounds__(PKT_BLOCK) void k_kc_round(i32 n, i32 nf, const i32* __restrict__ F,
                                                       const i64* __restrict__ P, const i64* __restrict__ off,
                                                       const i32* __restrict__ adj, i32 k, i32* __restrict__ core,
                                                       i32* __restrict__ deg, i32* __restrict__ next, int sel,
                                                       KcCounters* cnt) {
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt->nnext[sel ^ 1] = 0;
  const i64 total = P[nf];
  const i64 lim = total > nf ? total : (i64)nf;
  const i64 lim_up = (lim + PKT_WAVE - 1) / PKT_WAVE * PKT_WAVE;  // whole waves stay in the loop
  for (i64 g = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; g < lim_up; g += (i64)gridDim.x * PKT_BLOCK) {
    if (g < nf) core[F[g]] = k;
    bool join = false;
    i32 v = -1;
    if (g < total) {
      const i64 i = upper_bound_dev(P, (i64)0, (i64)nf + 1, g) - 1;
      const i32 u = F[i];
      v = adj[off[u] + (g - P[i])];
      if (v < 0 || v >= n) {  // checked before any use as an index
        atomicOr(&cnt->err, 1u);
        v = -1;
      } else if (__hip_atomic_load(&deg[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > k) {
        const i32 old = atomicSub(&deg[v], 1);
        if (old == k + 1)
          join = true;
        else if (old <= k)
          atomicAdd(&deg[v], 1);
      }
    }
    const i32 s = wave_append_slot(join, &cnt->nnext[sel]);
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

// The counters come back through pinned host memory, one copy and one wait per
// round; the buffer stays with the calling thread for its later calls.
thread_local KcCounters* h_kc = nullptr;

truss_status kc_read(const KcWork& w, KcCounters* out, hipStream_t s) {
  if (!h_kc) PKT_HIP(hipHostMalloc((void**)&h_kc, sizeof(KcCounters), hipHostMallocDefault));
  PKT_HIP(hipMemcpyAsync(h_kc, w.cnt, sizeof(KcCounters), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  *out = *h_kc;
  return TRUSS_OK;
}

// Lanes for a round's items without reading their count back: a frontier vertex
// at level k has at least k slots, and the average row length is the other
// estimate; the grid-stride loop covers any count.
inline int kc_round_grid(i32 nf, i32 k, i64 two_m, i32 n) {
  const i64 avg = (two_m + n - 1) / n;
  i64 est = (i64)nf * (k > avg ? (i64)k : avg);
  if (est > two_m) est = two_m;
  return grid_items(est);
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
  hipLaunchKernelGGL(k_kc_init, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, two_m, offsets, w.deg, core, w.A[0],
                     w.cnt);
  PKT_LAUNCH_CHECK();
  KcCounters hc;
  if (truss_status st = kc_read(w, &hc, s)) return st;
  if (hc.err) {
    set_error("input CSR: offsets out of order or past offsets[n]");
    return TRUSS_E_RANGE;
  }
  i32 na = n, asel = 0, k = 0, kmax = 0;
  i64 guard = 0;
  while (na > 0) {
    if (++guard > (i64)n + 2) {  // every level either finds a vertex or jumps to a larger degree
      set_error("k-core level bound exceeded");
      return TRUSS_E_INTERNAL;
    }
    // level scan: the frontier and the vertices left
    hipLaunchKernelGGL(k_kc_reset, dim3(1), dim3(1), 0, s, w.cnt);
    const i64 tiles = ((i64)na + KC_TILE - 1) / KC_TILE;
    hipLaunchKernelGGL(k_kc_scan, dim3((int)(tiles < 4096 ? tiles : 4096)), dim3(PKT_BLOCK), 0, s, na,
                       (const i32*)w.A[asel], k, (const i32*)w.deg, w.F[0], w.A[asel ^ 1], w.cnt);
    PKT_LAUNCH_CHECK();
    if (truss_status st = kc_read(w, &hc, s)) return st;
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
      PKT_HIP(scan_launch(FrontierRows{w.F[fsel], offsets, nf}, w.partial, w.P, &w.cnt->arrive, s));
      hipLaunchKernelGGL(k_kc_round, dim3(kc_round_grid(nf, k, two_m, n)), dim3(PKT_BLOCK), 0, s, n, nf,
                         (const i32*)w.F[fsel], (const i64*)w.P, offsets, adj, k, core, w.deg, w.F[fsel ^ 1],
                         fsel, w.cnt);
      PKT_LAUNCH_CHECK();
      if (truss_status st = kc_read(w, &hc, s)) return st;
      if (hc.err) {
        set_error("input CSR: a neighbour id outside [0, n)");
        return TRUSS_E_RANGE;
      }
      kmax = k;
      nf = hc.nnext[fsel];
      fsel ^= 1;
    }
    k += 1;
  }
  if (max_core) *max_core = kmax;
  return TRUSS_OK;
}
