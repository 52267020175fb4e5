// Trussness by the local h-index iteration: the barrier-free alternative to
// level-synchronous peeling that the Background section cites (Sariyuce et
// al.'s nucleus decomposition by repeated local updates, after Montresor et al.'s
// rule for core numbers).  Sweep 0 sets every edge's estimate to its support;
// every later sweep gives each edge, all at once, the h-index of
// min(est(f1), est(f2)) over its triangles {e, f1, f2} under the previous
// sweep's estimates (the largest h such that h of those values are >= h).
// Estimates never grow and stop at trussness - 2.
//
// One wave per edge.  The triangles of (u, v) are the common neighbours w: the
// lanes take entries of the shorter row 64 at a time and binary-search the longer
// one, and the other two edges' ids come from a per-slot edge-id array.  The new
// value of an edge whose estimate was `old` lies in [0, old]; a pass over its
// triangles counts, for 64 thresholds spread over the current interval (one per
// lane), the values at or above each, and keeps the sub-interval where "count >=
// threshold" turns false, so an interval of length L takes ceil(log64 L) passes
// (one pass when the estimate holds).  Only edges with a triangle neighbour that
// changed in the previous sweep are recomputed (the others would get the same
// value again); an edge that changes marks its neighbours in one more pass.
#include <limits.h>

#include "common.h"
#include "launch.h"
#include "scan.h"

namespace {

constexpr int HX_WAVES = PKT_BLOCK / PKT_WAVE;

struct HxFlags {
  u32 err;
  i32 changed;
};

__global__ __launch_bounds__(PKT_BLOCK) void k_hx_check(i32 n, i64 two_m, const i64* __restrict__ off, HxFlags* fl) {
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK) {
    const i64 b = off[v], e = off[v + 1];
    if ((v == 0 && b != 0) || b < 0 || e < b || e > two_m) atomicOr(&fl->err, 1u);
  }
}

// First slot of row u above u: the row's canonical edges run from there.
__global__ __launch_bounds__(PKT_BLOCK) void k_hx_first_upper(i32 n, const i64* __restrict__ off,
                                                             const i32* __restrict__ adj, i64* __restrict__ fa) {
  for (i64 u = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; u < n; u += (i64)gridDim.x * PKT_BLOCK)
    fa[u] = upper_bound_dev(adj, off[u], off[u + 1], (i32)u);
}

struct UpperLen {
  const i64* off;
  const i64* fa;
  i32 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 u) const { return off[u + 1] - fa[u]; }
};

// Edge id of every slot (canonical: row-major rank of (u, v), u < v) and the
// endpoints of every edge.  A block takes PKT_BLOCK consecutive slots at a time
// and finds the rows of its first and last slot once.  Error bits: 4 a neighbour
// outside [0, n), 8 a slot with no mirror (or an edge id out of range, which only
// an asymmetric CSR gives), 16 a row not strictly increasing, 32 a self loop.
__global__ __launch_bounds__(PKT_BLOCK) void k_hx_eid(i32 n, i64 two_m, i64 m, const i64* __restrict__ off,
                                                     const i32* __restrict__ adj, const i64* __restrict__ fa,
                                                     const i64* __restrict__ U, i32* __restrict__ eid,
                                                     i32* __restrict__ eu, i32* __restrict__ ev, HxFlags* fl) {
  __shared__ i64 rows[2];
  const i64 chunks = (two_m + PKT_BLOCK - 1) / PKT_BLOCK;
  for (i64 c = blockIdx.x; c < chunks; c += gridDim.x) {  // uniform over the block
    const i64 j0 = c * PKT_BLOCK;
    const i64 j1 = min(j0 + PKT_BLOCK, two_m) - 1;
    if (threadIdx.x < 2)
      rows[threadIdx.x] = upper_bound_dev(off, (i64)0, (i64)n + 1, threadIdx.x == 0 ? j0 : j1) - 1;
    __syncthreads();
    const i64 j = j0 + threadIdx.x;
    if (j <= j1) {
      const i32 u = (i32)(upper_bound_dev(off, rows[0], rows[1] + 1, j) - 1);
      const i32 v = adj[j];
      i64 e = 0;
      if (v < 0 || v >= n) {  // checked before any use as an index
        atomicOr(&fl->err, 4u);
      } else {
        if (j + 1 < off[u + 1] && adj[j + 1] <= v) atomicOr(&fl->err, 16u);
        if (v == u) {
          atomicOr(&fl->err, 32u);
        } else if (v > u) {
          e = U[u] + (j - fa[u]);
          if (e >= 0 && e < m) {  // unsorted rows could put it anywhere
            eu[e] = u;
            ev[e] = v;
          } else {
            atomicOr(&fl->err, 8u);
            e = 0;
          }
        } else {
          const i64 end = off[v + 1];
          const i64 pos = lower_bound_dev(adj, off[v], end, u);
          if (pos == end || adj[pos] != u) {
            atomicOr(&fl->err, 8u);
          } else {
            e = U[v] + (pos - fa[v]);
            if (e < 0 || e >= m) {
              atomicOr(&fl->err, 8u);
              e = 0;
            }
          }
        }
      }
      eid[j] = (i32)e;
    }
    __syncthreads();  // rows[] is rewritten for the next chunk
  }
}

// Runs f(found, jS, jL) for the common neighbours of u and v, 64 entries of the
// shorter row per call (jS its slot, jL the matching slot of the longer row).
// Every lane of the wave calls f the same number of times.
template <class F>
__device__ __forceinline__ void walk_common(const i64* __restrict__ off, const i32* __restrict__ adj, i32 u, i32 v,
                                            F&& f) {
  i64 sS = off[u], eS = off[u + 1], sL = off[v], eL = off[v + 1];
  if (eS - sS > eL - sL) {
    i64 t = sS;
    sS = sL;
    sL = t;
    t = eS;
    eS = eL;
    eL = t;
  }
  for (i64 base = sS; base < eS; base += PKT_WAVE) {
    const i64 j = base + lane_id();
    bool found = false;
    i64 jl = 0;
    if (j < eS) {
      const i32 x = adj[j];
      jl = lower_bound_dev(adj, sL, eL, x);
      found = jl < eL && adj[jl] == x;
    }
    f(found, j, jl);
  }
}

// Sweep 0: the support of every edge.
__global__ __launch_bounds__(PKT_BLOCK) void k_hx_support(i64 m, const i64* __restrict__ off,
                                                         const i32* __restrict__ adj, const i32* __restrict__ eu,
                                                         const i32* __restrict__ ev, i32* __restrict__ est) {
  const i64 wstride = (i64)gridDim.x * HX_WAVES;
  for (i64 e = (i64)blockIdx.x * HX_WAVES + threadIdx.x / PKT_WAVE; e < m; e += wstride) {
    i32 c = 0;
    walk_common(off, adj, eu[e], ev[e], [&](bool found, i64, i64) { c += __popcll(__ballot(found)); });
    if (lane_id() == 0) est[e] = c;
  }
}

// One sweep.  Edges not flagged in act keep their estimate; a flagged edge takes
// the h-index of its triangle values under cur, and if that differs it flags its
// triangle neighbours in act_next and counts itself in fl->changed.
__global__ __launch_bounds__(PKT_BLOCK) void k_hx_sweep(i64 m, const i64* __restrict__ off,
                                                       const i32* __restrict__ adj, const i32* __restrict__ eid,
                                                       const i32* __restrict__ eu, const i32* __restrict__ ev,
                                                       const i32* __restrict__ cur, i32* __restrict__ nxt,
                                                       const u8* __restrict__ act, u8* __restrict__ act_next,
                                                       HxFlags* fl) {
  __shared__ i32 changed;
  if (threadIdx.x == 0) changed = 0;
  __syncthreads();
  const int lane = lane_id();
  const i64 wstride = (i64)gridDim.x * HX_WAVES;
  for (i64 e = (i64)blockIdx.x * HX_WAVES + threadIdx.x / PKT_WAVE; e < m; e += wstride) {
    const i32 old = cur[e];
    if (!act[e] || old == 0) {  // an estimate of 0 cannot fall
      if (lane == 0) nxt[e] = old;
      continue;
    }
    const i32 u = eu[e], v = ev[e];
    i32 lo = 0, hi = old;  // the new value lies in [lo, hi]; P(lo) holds
    while (lo < hi) {
      const i64 span = (i64)(hi - lo);
      const i32 T = lo + (i32)(((i64)(lane + 1) * span + PKT_WAVE - 1) / PKT_WAVE);  // nondecreasing, T63 = hi
      i32 cnt = 0;
      walk_common(off, adj, u, v, [&](bool found, i64 jS, i64 jL) {
        const i32 val = found ? min(cur[eid[jS]], cur[eid[jL]]) : -1;
        u64 fm = __ballot(found);
        while (fm) {
          const int i = __ffsll((unsigned long long)fm) - 1;
          fm &= fm - 1ull;
          cnt += __shfl(val, i) >= T;
        }
      });
      // count >= threshold holds on a prefix of the lanes (counts fall, thresholds rise)
      const int q = __popcll(__ballot(cnt >= T));
      const i32 tq1 = __shfl(T, q > 0 ? q - 1 : 0), tq = __shfl(T, q < PKT_WAVE ? q : PKT_WAVE - 1);
      if (q == 0) {
        hi = tq1 - 1;  // T0 - 1
      } else {
        lo = tq1;
        if (q < PKT_WAVE) hi = tq - 1;
      }
    }
    if (lane == 0) nxt[e] = lo;
    if (lo != old) {
      walk_common(off, adj, u, v, [&](bool found, i64 jS, i64 jL) {
        if (found) {
          act_next[eid[jS]] = 1;
          act_next[eid[jL]] = 1;
        }
      });
      if (lane == 0) atomicAdd(&changed, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && changed) atomicAdd(&fl->changed, changed);
}

__global__ __launch_bounds__(PKT_BLOCK) void k_hx_fill_u8(u8* __restrict__ a, i64 count, u8 value) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < count; i += (i64)gridDim.x * PKT_BLOCK) a[i] = value;
}

__global__ __launch_bounds__(PKT_BLOCK) void k_hx_out(i64 m, const i32* __restrict__ est, i32* __restrict__ tau) {
  for (i64 e = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; e < m; e += (i64)gridDim.x * PKT_BLOCK) tau[e] = est[e] + 2;
}

struct HxWork {
  i64* fa;
  i64* U;
  i64* partial;
  u32* arrive;
  HxFlags* fl;
  i32* eid;
  i32* eu;
  i32* ev;
  i32* est[2];
  u8* act[2];
};

size_t hx_layout(i32 n, i64 two_m, void* ws, HxWork* w) {
  Carver cv(ws);
  HxWork t;
  const i64 m = two_m / 2;
  t.fa = cv.take<i64>((size_t)n);
  t.U = cv.take<i64>((size_t)n + 1);
  t.partial = cv.take<i64>(SCAN_BLOCKS + 1);
  t.arrive = cv.take<u32>(1);
  t.fl = cv.take<HxFlags>(1);
  t.eid = cv.take<i32>((size_t)two_m);
  t.eu = cv.take<i32>((size_t)m);
  t.ev = cv.take<i32>((size_t)m);
  for (int q = 0; q < 2; ++q) t.est[q] = cv.take<i32>((size_t)m);
  for (int q = 0; q < 2; ++q) t.act[q] = cv.take<u8>((size_t)m);
  if (w) *w = t;
  return cv.used;
}

truss_status hx_read(const HxWork& w, HxFlags* h, hipStream_t s) {
  PKT_HIP(hipMemcpyAsync(h, w.fl, sizeof(HxFlags), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

}  // namespace

extern "C" truss_status truss_hindex_workspace_bytes(int32_t n, int64_t two_m, size_t* bytes) {
  pkt::set_error("");
  if (n < 0 || two_m < 0 || bytes == nullptr) {
    pkt::set_error("bad arguments to truss_hindex_workspace_bytes");
    return TRUSS_E_ARG;
  }
  *bytes = hx_layout(n, two_m, nullptr, nullptr);
  return TRUSS_OK;
}

extern "C" truss_status truss_hindex(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* trussness,
                                     int32_t max_sweeps, int32_t* sweeps, int32_t* converged, void* workspace,
                                     size_t workspace_bytes, void* stream) {
  using namespace pkt;
  set_error("");
  if (sweeps) *sweeps = 0;
  if (converged) *converged = 0;
  if (n < 0 || (n > 0 && offsets == nullptr)) {
    set_error("bad n or NULL offsets");
    return TRUSS_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  i64 two_m = 0;
  if (n > 0) {
    PKT_HIP(hipMemcpyAsync(&two_m, offsets + n, sizeof(i64), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
  }
  if (two_m < 0 || two_m > (i64)INT32_MAX) {  // edge ids are int32
    set_error("offsets[n] = %lld is out of range", (long long)two_m);
    return TRUSS_E_RANGE;
  }
  if (two_m > 0 && (adj == nullptr || trussness == nullptr)) {
    set_error("NULL adj or trussness");
    return TRUSS_E_ARG;
  }
  const size_t need = hx_layout(n, two_m, nullptr, nullptr);
  if (workspace == nullptr || workspace_bytes < need || ((uintptr_t)workspace & 255u)) {
    set_error("workspace: need %zu bytes at 256-byte alignment", need);
    return TRUSS_E_WORKSPACE;
  }
  if (two_m == 0) {
    if (converged) *converged = 1;
    return TRUSS_OK;
  }
  if (two_m & 1) {
    set_error("offsets[n] = %lld is odd: the CSR is not symmetric", (long long)two_m);
    return TRUSS_E_NOT_SYMMETRIC;
  }
  const i64 m = two_m / 2;
  HxWork w;
  hx_layout(n, two_m, workspace, &w);
  PKT_HIP(hipMemsetAsync(w.fl, 0, sizeof(HxFlags), s));
  PKT_HIP(hipMemsetAsync(w.arrive, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_hx_check, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, two_m, offsets, w.fl);
  PKT_LAUNCH_CHECK();
  HxFlags h;
  if (truss_status st = hx_read(w, &h, s)) return st;
  if (h.err) {
    set_error("input CSR: offsets not starting at 0, out of order or past offsets[n]");
    return TRUSS_E_RANGE;
  }
  hipLaunchKernelGGL(k_hx_first_upper, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, offsets, adj, w.fa);
  PKT_HIP(scan_launch(UpperLen{offsets, w.fa, n}, w.partial, w.U, w.arrive, s));
  hipLaunchKernelGGL(k_hx_eid, dim3(grid_items(two_m)), dim3(PKT_BLOCK), 0, s, n, two_m, m, offsets, adj,
                     (const i64*)w.fa, (const i64*)w.U, w.eid, w.eu, w.ev, w.fl);
  PKT_LAUNCH_CHECK();
  if (truss_status st = hx_read(w, &h, s)) return st;
  i64 mu = 0;  // canonical edges found: m exactly when every slot has its mirror
  PKT_HIP(hipMemcpyAsync(&mu, w.U + n, sizeof(i64), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (h.err & 4u) {
    set_error("input CSR: a neighbour id outside [0, n)");
    return TRUSS_E_RANGE;
  }
  if (h.err & (16u | 32u)) {
    set_error(h.err & 16u ? "input CSR: a row not strictly increasing" : "input CSR: a self loop");
    return TRUSS_E_NOT_SIMPLE;
  }
  if (h.err || mu != m) {
    set_error("input CSR: (u, v) present without (v, u)");
    return TRUSS_E_NOT_SYMMETRIC;
  }
  hipLaunchKernelGGL(k_hx_support, dim3(grid_waves(m)), dim3(PKT_BLOCK), 0, s, m, offsets, adj,
                     (const i32*)w.eu, (const i32*)w.ev, w.est[0]);
  hipLaunchKernelGGL(k_hx_fill_u8, dim3(grid_items(m)), dim3(PKT_BLOCK), 0, s, w.act[0], m, (u8)1);
  PKT_LAUNCH_CHECK();
  int q = 0;
  i32 done = 0;
  bool conv = false;
  for (;;) {
    if (max_sweeps >= 0 && done >= max_sweeps) break;
    if (done > 1000000) {
      set_error("h-index iteration: sweep bound exceeded");
      return TRUSS_E_INTERNAL;
    }
    hipLaunchKernelGGL(k_hx_fill_u8, dim3(grid_items(m)), dim3(PKT_BLOCK), 0, s, w.act[q ^ 1], m, (u8)0);
    PKT_HIP(hipMemsetAsync(&w.fl->changed, 0, sizeof(i32), s));
    hipLaunchKernelGGL(k_hx_sweep, dim3(grid_waves(m)), dim3(PKT_BLOCK), 0, s, m, offsets, adj, (const i32*)w.eid,
                       (const i32*)w.eu, (const i32*)w.ev, (const i32*)w.est[q], w.est[q ^ 1], (const u8*)w.act[q],
                       w.act[q ^ 1], w.fl);
    PKT_LAUNCH_CHECK();
    if (truss_status st = hx_read(w, &h, s)) return st;
    if (h.changed == 0) {  // the new estimates equal the old ones
      conv = true;
      break;
    }
    q ^= 1;
    ++done;
  }
  hipLaunchKernelGGL(k_hx_out, dim3(grid_items(m)), dim3(PKT_BLOCK), 0, s, m, (const i32*)w.est[q], trussness);
  PKT_LAUNCH_CHECK();
  PKT_HIP(hipStreamSynchronize(s));  // the output is complete when the call returns
  if (sweeps) *sweeps = done;
  if (converged) *converged = conv ? 1 : 0;
  return TRUSS_OK;
}
