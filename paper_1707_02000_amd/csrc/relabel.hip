// Decomposition of a graph relabelled by increasing (degree, id), with the
// trussness mapped back to the input's edges (truss_options::relabel).
//
// Trussness does not depend on the vertex labels (Background section: it is a
// property of each edge's triangles), and the paper itself relabels its inputs by
// increasing core number before decomposing them (Performance Results section, the
// support study and Table 2).  Here the key is the degree, which costs only the sort:
// after relabelling, the high-degree vertices -- whose rows every round searches --
// sit together at the top of the id range, their rows and support words in a few
// places of memory.  Steps, all on the stream:
//   1. validate the input CSR (when asked), copy int32 offsets to int64;
//   2. new ids: a stable radix sort of (degree, id); the relabelled CSR, rows sorted;
//   3. decompose the relabelled graph (edge ids, support, level loop);
//   4. for every edge (a, b) of the relabelled graph, the input edge (order[a],
//      order[b]) and its canonical id (the upper entries of the rows before its
//      smaller endpoint, then its rank in that row): trussness (and the round, when
//      a peeling order is asked for) scattered there.
// Workspace: region A (the decomposition's own layout, which the order and relabel
// steps use as scratch before the decomposition starts), then the relabelled CSR,
// the permutation and the map's arrays.
#include <string.h>

#include "scan.h"
#include "truss.h"

namespace pkt {
truss_status run_single(const Work& w, const truss_options& opt, truss_stats* stats, i32* trussness,
                        hipStream_t s, bool support_only);
truss_status prepare_off64(Work& w, const i32* off32, hipStream_t s);
truss_status validate_input(const Work& w, hipStream_t s);
size_t kco_scratch_bytes(i32 n, i64 two_m);
truss_status kco_order_run(i32 n, const i32* keys, int key_bits, i32* new_id, i32* order, void* scratch,
                           hipStream_t s);
truss_status kco_relabel_run(i32 n, i64 two_m, const i64* off, const i32* adj, const i32* new_id, const i32* order,
                             i64* off2, i32* adj2, void* scratch, hipStream_t s);
int kco_bits(i64 x);
}  // namespace pkt

using namespace pkt;

namespace {

inline int grid_r(i64 count, int cap = 8192) {
  i64 g = (count + PKT_BLOCK - 1) / PKT_BLOCK;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__global__ __launch_bounds__(PKT_BLOCK) void k_degree(i32 n, const i64* __restrict__ off, i32* __restrict__ deg) {
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK)
    deg[v] = (i32)(off[v + 1] - off[v]);
}

// First slot of input row x above x: the row's canonical edges run from there.
__global__ __launch_bounds__(PKT_BLOCK) void k_upper_start(i32 n, const i64* __restrict__ off,
                                                          const i32* __restrict__ adj, i64* __restrict__ us) {
  for (i64 x = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; x < n; x += (i64)gridDim.x * PKT_BLOCK)
    us[x] = lower_bound_dev(adj, off[x], off[x + 1], (i32)x + 1);
}

struct UpperLen {
  const i64* off;
  const i64* us;
  i32 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 x) const { return off[x + 1] - us[x]; }
};

// Relabelled edge e2 = (a, b) is the input edge (order[a], order[b]); its canonical
// id is eb[x] + (rank of y among x's entries above x), x < y its endpoints.
__global__ __launch_bounds__(PKT_BLOCK) void k_map_back(i64 m, const int2* __restrict__ el2,
                                                       const i32* __restrict__ order, const i64* __restrict__ off,
                                                       const i32* __restrict__ adj, const i64* __restrict__ us,
                                                       const i64* __restrict__ eb, const i32* __restrict__ tau2,
                                                       i32* __restrict__ tau, const i32* __restrict__ rounds2,
                                                       i32* __restrict__ rounds) {
  for (i64 e2 = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; e2 < m; e2 += (i64)gridDim.x * PKT_BLOCK) {
    const int2 ab = el2[e2];
    const i32 u = order[ab.x], v = order[ab.y];
    const i32 x = min(u, v), y = max(u, v);
    const i64 b = us[x], end = off[x + 1];
    const i64 pos = lower_bound_dev(adj, b, end, y);
    const i64 e = eb[x] + (pos - b);
    if (e < 0 || e >= m) continue;  // only for a CSR outside the contract (validation off)
    tau[e] = tau2[e2];
    if (rounds) rounds[e] = rounds2[e2];
  }
}

struct RelabelWork {
  void* regionA;  // the decomposition's layout; scratch of the order and relabel steps before it
  i64* off64;     // [n+1] input offsets as int64 (int32 entry point)
  i64* off2;      // [n+1] relabelled offsets
  i32* adj2;      // [2m] relabelled adjacency
  i32* tau2;      // [m] trussness of the relabelled graph
  i32* rounds2;   // [m] its rounds (peeling order), when asked for
  i32* key;       // [n] degrees (the sort key)
  i32* new_id;    // [n]
  i32* order;     // [n]
  i64* us;        // [n] first slot above the vertex, input rows
  i64* eb;        // [n+1] first canonical edge id of every input row
  i64* partial;   // [SCAN_BLOCKS + 1]
  u32* arrive;
};

size_t relabel_layout(i32 n, i64 two_m, void* ws, RelabelWork* r) {
  const size_t a = work_layout(n, two_m, false, nullptr, nullptr), b = kco_scratch_bytes(n, two_m);
  Carver cv(ws);
  RelabelWork t;
  t.regionA = cv.take<char>(a > b ? a : b);
  t.off64 = cv.take<i64>((size_t)n + 1);
  t.off2 = cv.take<i64>((size_t)n + 1);
  t.adj2 = cv.take<i32>((size_t)two_m);
  t.tau2 = cv.take<i32>((size_t)(two_m / 2));
  t.rounds2 = cv.take<i32>((size_t)(two_m / 2));
  t.key = cv.take<i32>((size_t)n);
  t.new_id = cv.take<i32>((size_t)n);
  t.order = cv.take<i32>((size_t)n);
  t.us = cv.take<i64>((size_t)n);
  t.eb = cv.take<i64>((size_t)n + 1);
  t.partial = cv.take<i64>(SCAN_BLOCKS + 1);
  t.arrive = cv.take<u32>(1);
  if (r) *r = t;
  return cv.used;
}

}  // namespace

namespace pkt {

size_t relabel_workspace_bytes(i32 n, i64 two_m) { return relabel_layout(n, two_m, nullptr, nullptr); }

// The whole relabelled decomposition (see the top of this file).  off32 / off64: the
// input offsets (one of them).  Phase times: the validation in ms_validate, the
// relabelling in ms_build, the map back in ms_total only.
truss_status run_relabelled(i32 n, i64 two_m, const i64* off64_in, const i32* off32_in, const i32* adj, i32* out,
                            void* ws, const truss_options& opt, truss_stats* stats, hipStream_t s) {
  RelabelWork r;
  relabel_layout(n, two_m, ws, &r);
  const i64 m = two_m / 2;
  const bool timed = stats != nullptr;
  hipEvent_t ev[5];
  if (timed)
    for (int k = 0; k < 5; ++k) PKT_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableSystemFence));
  struct EventGuard {
    hipEvent_t* e;
    bool on;
    ~EventGuard() {
      if (on)
        for (int k = 0; k < 5; ++k) (void)hipEventDestroy(e[k]);
    }
  } guard{ev, timed};
  if (timed) PKT_HIP(hipEventRecord(ev[0], s));
  // 1. the input, as int64 offsets, validated when asked
  Work wv;
  work_layout(n, two_m, false, r.regionA, &wv);
  wv.adj = adj;
  if (off32_in) {
    wv.off64 = r.off64;
    truss_status st = prepare_off64(wv, off32_in, s);
    if (st) return st;
  } else {
    wv.off = off64_in;
  }
  const i64* off = wv.off;
  if (opt.validate) {
    truss_status st = validate_input(wv, s);
    if (st) return st;
  }
  if (timed) PKT_HIP(hipEventRecord(ev[1], s));
  // 2. new ids by increasing (degree, id), the relabelled CSR
  hipLaunchKernelGGL(k_degree, dim3(grid_r(n)), dim3(PKT_BLOCK), 0, s, n, off, r.key);
  PKT_LAUNCH_CHECK();
  truss_status st = kco_order_run(n, r.key, kco_bits((i64)n - 1), r.new_id, r.order, r.regionA, s);
  if (st) return st;
  st = kco_relabel_run(n, two_m, off, adj, r.new_id, r.order, r.off2, r.adj2, r.regionA, s);
  if (st) return st;
  if (timed) PKT_HIP(hipEventRecord(ev[2], s));
  // 3. the decomposition of the relabelled graph
  Work w2;
  work_layout(n, two_m, false, r.regionA, &w2);
  w2.off = r.off2;
  w2.adj = r.adj2;
  truss_options o2 = opt;
  o2.validate = 0;
  o2.relabel = 0;
  o2.peel_round = opt.peel_round ? r.rounds2 : nullptr;
  st = run_single(w2, o2, stats, r.tau2, s, false);
  if (st) return st;
  if (timed) PKT_HIP(hipEventRecord(ev[3], s));
  // 4. back to the input's edges
  PKT_HIP(hipMemsetAsync(r.arrive, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_upper_start, dim3(grid_r(n)), dim3(PKT_BLOCK), 0, s, n, off, adj, r.us);
  PKT_HIP(scan_launch(UpperLen{off, r.us, n}, r.partial, r.eb, r.arrive, s));
  hipLaunchKernelGGL(k_map_back, dim3(grid_r(m)), dim3(PKT_BLOCK), 0, s, m, (const int2*)w2.el,
                     (const i32*)r.order, off, adj, (const i64*)r.us, (const i64*)r.eb, (const i32*)r.tau2, out,
                     (const i32*)r.rounds2, opt.peel_round);
  PKT_LAUNCH_CHECK();
  if (timed) PKT_HIP(hipEventRecord(ev[4], s));
  PKT_HIP(hipStreamSynchronize(s));
  if (timed) {
    float t_val = 0.f, t_rel = 0.f, t_map = 0.f;
    PKT_HIP(hipEventElapsedTime(&t_val, ev[0], ev[1]));
    PKT_HIP(hipEventElapsedTime(&t_rel, ev[1], ev[2]));
    PKT_HIP(hipEventElapsedTime(&t_map, ev[3], ev[4]));
    stats->ms_validate += t_val;
    stats->ms_build += t_rel;
    stats->ms_total += t_val + t_rel + t_map;
  }
  return TRUSS_OK;
}

}  // namespace pkt
