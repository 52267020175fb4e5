// Maximal k-trusses from the trussness (Introduction and Background sections of Kabir and
// Madduri, arXiv:1707.02000: a k-truss is a maximal connected subgraph in which
// every edge lies in at least k - 2 triangles of the subgraph).  The edges of
// trussness >= k form the largest subgraph with that property and contain every
// k-truss, so the k-trusses are the connected components of those edges.
//
// Components by a lock-free union-find over the vertices: every edge of
// trussness >= k joins its endpoints' sets by hooking the larger root under the
// smaller one with a compare-and-swap (parents only ever decrease, so there are
// no cycles and every find ends), finds halve their paths as they go; then one
// pass points every vertex at its root, a second takes the smallest edge id of
// every set, and a third labels the edges with it.
#include <limits.h>

#include "common.h"
#include "launch.h"

namespace {

__device__ __forceinline__ i32 ld_par(const i32* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x's set.  Halving writes x's grandparent into x: an ancestor, so the
// invariant parent <= vertex still holds whatever other threads do meanwhile.
__device__ __forceinline__ i32 uf_find(i32* par, i32 x) {
  for (;;) {
    const i32 p = ld_par(&par[x]);
    if (p == x) return x;
    const i32 gp = ld_par(&par[p]);
    if (gp != p) __hip_atomic_store(&par[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = p;
  }
}

// Joins the sets of a and b.  A failed hook means the root got a parent in the
// meantime; the loop goes on from that parent, a strictly smaller vertex.
__device__ __forceinline__ void uf_union(i32* par, i32 a, i32 b) {
  for (;;) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    if (a < b) {
      const i32 t = a;
      a = b;
      b = t;
    }
    const i32 old = atomicCAS(&par[a], a, b);
    if (old == a) return;
    a = old;
  }
}

__global__ __launch_bounds__(PKT_BLOCK) void k_kt_init(i32 n, i32* __restrict__ par, i32* __restrict__ first) {
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK) {
    par[v] = (i32)v;
    first[v] = INT_MAX;
  }
}

__global__ __launch_bounds__(PKT_BLOCK) void k_kt_union(i32 n, i64 m, const i32* __restrict__ eu,
                                                       const i32* __restrict__ ev, const i32* __restrict__ tau,
                                                       i32 k, i32* par, u32* __restrict__ err) {
  for (i64 e = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; e < m; e += (i64)gridDim.x * PKT_BLOCK) {
    if (tau[e] < k) continue;
    const i32 u = eu[e], v = ev[e];
    if (u < 0 || u >= n || v < 0 || v >= n) {  // checked before any use as an index
      atomicOr(err, 1u);
      continue;
    }
    uf_union(par, u, v);
  }
}

__global__ __launch_bounds__(PKT_BLOCK) void k_kt_compress(i32 n, i32* par) {
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK)
    par[v] = uf_find(par, (i32)v);
}

// Smallest edge id of every set: every kept edge offers its id to its set's root
// (par is fully compressed here, so par[u] is the root).  The edge list may come
// in any order.  In the canonical row-major order the lanes of a wave mostly share
// one root (consecutive edges of one row, or one large k-truss), so the lanes
// that share the first active lane's root take their minimum first and one atomic
// reaches memory for them; every other lane takes its own atomic.  A set's value
// only decreases, so an offer no smaller than a plain read of it (possibly older,
// hence no smaller than the current value) is dropped without an atomic: with
// one giant k-truss the low ids arrive first and most waves end there.
__global__ __launch_bounds__(PKT_BLOCK) void k_kt_first(i64 m, const i32* __restrict__ eu,
                                                       const i32* __restrict__ tau, i32 k,
                                                       const i32* __restrict__ par, i32* first,
                                                       const u32* __restrict__ err) {
  if (*err) return;
  const i64 stride = (i64)gridDim.x * PKT_BLOCK;
  const i64 m_up = (m + PKT_WAVE - 1) / PKT_WAVE * PKT_WAVE;  // whole waves stay in the loop
  for (i64 e = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; e < m_up; e += stride) {
    i32 r = -1;
    if (e < m && tau[e] >= k) r = par[eu[e]];
    const u64 act = __ballot(r >= 0);
    if (act == 0) continue;
    const int lead = __ffsll((unsigned long long)act) - 1;
    const i32 rl = __shfl(r, lead);
    const i32 mn = wave_min_i32(r == rl ? (i32)e : INT_MAX);
    if (lane_id() == lead && mn < first[rl]) atomicMin(&first[rl], mn);
    if (r >= 0 && r != rl && (i32)e < first[r]) atomicMin(&first[r], (i32)e);
  }
}

__global__ __launch_bounds__(PKT_BLOCK) void k_kt_label(i64 m, const i32* __restrict__ eu,
                                                       const i32* __restrict__ tau, i32 k,
                                                       const i32* __restrict__ par,
                                                       const i32* __restrict__ first, i32* __restrict__ label,
                                                       i32* __restrict__ count, const u32* __restrict__ err) {
  if (*err) return;
  i32 c = 0;
  for (i64 e = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; e < m; e += (i64)gridDim.x * PKT_BLOCK) {
    const i32 l = tau[e] >= k ? first[par[eu[e]]] : -1;
    label[e] = l;
    c += l == (i32)e;  // the smallest edge of its k-truss
  }
  c = (i32)wave_sum_i64(c);
  if (lane_id() == 0 && c) atomicAdd(count, c);
}

struct KtWork {
  i32* par;    // [n] union-find parents
  i32* first;  // [n] smallest edge id per root
  u32* err;    // range error flag
  i32* count;  // number of k-trusses
};

size_t kt_layout(i32 n, void* ws, KtWork* w) {
  Carver cv(ws);
  KtWork t;
  t.par = cv.take<i32>((size_t)n);
  t.first = cv.take<i32>((size_t)n);
  t.err = cv.take<u32>(1);
  t.count = cv.take<i32>(1);
  if (w) *w = t;
  return cv.used;
}

}  // namespace

extern "C" truss_status truss_ktruss_workspace_bytes(int32_t n, size_t* bytes) {
  pkt::set_error("");
  if (n < 0 || bytes == nullptr) {
    pkt::set_error("bad arguments to truss_ktruss_workspace_bytes");
    return TRUSS_E_ARG;
  }
  *bytes = kt_layout(n, nullptr, nullptr);
  return TRUSS_OK;
}

extern "C" truss_status truss_ktruss(int32_t n, int64_t m, const int32_t* el_u, const int32_t* el_v,
                                     const int32_t* trussness, int32_t k, int32_t* label, int32_t* num_trusses,
                                     void* workspace, size_t workspace_bytes, void* stream) {
  using namespace pkt;
  set_error("");
  if (n < 0 || m < 0 || k < 2 || m > (i64)INT32_MAX) {
    set_error("bad n, m or k (n >= 0, 0 <= m < 2^31, k >= 2)");
    return TRUSS_E_ARG;
  }
  if (m > 0 && (el_u == nullptr || el_v == nullptr || trussness == nullptr || label == nullptr)) {
    set_error("NULL edge list, trussness or label");
    return TRUSS_E_ARG;
  }
  const size_t need = kt_layout(n, nullptr, nullptr);
  if (workspace == nullptr || workspace_bytes < need || ((uintptr_t)workspace & 255u)) {
    set_error("workspace: need %zu bytes at 256-byte alignment", need);
    return TRUSS_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  KtWork w;
  kt_layout(n, workspace, &w);
  PKT_HIP(hipMemsetAsync(w.err, 0, sizeof(u32), s));
  PKT_HIP(hipMemsetAsync(w.count, 0, sizeof(i32), s));
  if (n > 0)
    hipLaunchKernelGGL(k_kt_init, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, w.par, w.first);
  if (m > 0) {
    hipLaunchKernelGGL(k_kt_union, dim3(grid_items(m)), dim3(PKT_BLOCK), 0, s, n, (i64)m, el_u, el_v, trussness, k,
                       w.par, w.err);
    if (n > 0) hipLaunchKernelGGL(k_kt_compress, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, w.par);
    hipLaunchKernelGGL(k_kt_first, dim3(grid_items(m)), dim3(PKT_BLOCK), 0, s, (i64)m, el_u, trussness, k,
                       (const i32*)w.par, w.first, (const u32*)w.err);
    hipLaunchKernelGGL(k_kt_label, dim3(grid_items(m)), dim3(PKT_BLOCK), 0, s, (i64)m, el_u, trussness, k,
                       (const i32*)w.par, (const i32*)w.first, label, w.count, (const u32*)w.err);
  }
  PKT_LAUNCH_CHECK();
  u32 err = 0;
  i32 count = 0;
  PKT_HIP(hipMemcpyAsync(&err, w.err, sizeof(u32), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipMemcpyAsync(&count, w.count, sizeof(i32), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (err) {
    set_error("edge list: an endpoint outside [0, n)");
    return TRUSS_E_RANGE;
  }
  if (num_trusses) *num_trusses = count;
  return TRUSS_OK;
}
