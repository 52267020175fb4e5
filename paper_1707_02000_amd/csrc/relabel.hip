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
//   2. degrees and their maximum: under the automatic policy (which sends graphs below
//      TRUSS_RELABEL_MIN_EDGES edges elsewhere), a graph whose maximum degree is below
//      TRUSS_RELABEL_MIN_SKEW times the mean is decomposed as given from here;
//   3. new ids: a stable radix sort of (degree, id); the relabelled CSR, rows sorted;
//   4. decompose the relabelled graph (edge ids, support, level loop);
//   5. for every input edge (x, y), x < y, in input edge order: its image {new_id[x],
//      new_id[y]} located in the relabelled row of the lower-degree endpoint, whose
//      slot gives the relabelled edge id; its trussness (and round, when a peeling
//      order is asked for) gathered from there.
// Workspace: region A (the decomposition's own layout, which the order and relabel
// steps use as scratch before the decomposition starts), then the relabelled CSR,
// the permutation and the map's arrays.
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

// Degrees (the sort key) and their maximum (atomicMax of every wave's maximum).
__global__ __launch_bounds__(PKT_BLOCK) void k_degree(i32 n, const i64* __restrict__ off, i32* __restrict__ deg,
                                                     u32* __restrict__ dmax) {
  u32 mx = 0;
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK) {
    const i32 d = (i32)(off[v + 1] - off[v]);
    deg[v] = d;
    mx = max(mx, (u32)d);
  }
  for (int o = PKT_WAVE / 2; o >= 1; o >>= 1) mx = max(mx, (u32)__shfl_xor((int)mx, o));
  if (lane_id() == 0 && mx > 0) atomicMax(dmax, mx);
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

// Input slot j of row x with y = adj[j] above x holds the input edge e = eb[x] + (j - us[x]).
// Its image is the relabelled edge {new_id[x], new_id[y]}, found in the relabelled row of the
// smaller new id -- the endpoint of lower degree, so a short row -- whose slot carries the
// relabelled edge id.  A block takes PKT_BLOCK consecutive slots at a time and finds the
// rows of its first and last slot once; the output is written in input edge order.
__global__ __launch_bounds__(PKT_BLOCK) void k_map_back(i32 n, i64 two_m, const i64* __restrict__ off,
                                                       const i32* __restrict__ adj, const i64* __restrict__ us,
                                                       const i64* __restrict__ eb, const i32* __restrict__ new_id,
                                                       const i64* __restrict__ off2, const i32* __restrict__ adj2,
                                                       const i32* __restrict__ eid2, const i32* __restrict__ tau2,
                                                       i32* __restrict__ tau, const i32* __restrict__ rounds2,
                                                       i32* __restrict__ rounds) {
  __shared__ i64 rows[2];
  const i64 m = two_m / 2;
  for (i64 base = (i64)blockIdx.x * PKT_BLOCK; base < two_m; base += (i64)gridDim.x * PKT_BLOCK) {
    const i64 last = min(base + PKT_BLOCK, two_m) - 1;
    if (threadIdx.x == 0) rows[0] = upper_bound_dev(off, (i64)0, (i64)n + 1, base) - 1;
    if (threadIdx.x == PKT_WAVE) rows[1] = upper_bound_dev(off, (i64)0, (i64)n + 1, last) - 1;
    __syncthreads();
    const i64 j = base + threadIdx.x;
    if (j < two_m) {
      const i32 x = (i32)(upper_bound_dev(off, rows[0], rows[1] + 1, j) - 1);
      const i32 y = adj[j];
      if (y > x) {
        const i32 a = new_id[x], b = new_id[y];
        const i32 lo = min(a, b), hi = max(a, b);
        const i64 rb = off2[lo], re = off2[lo + 1];
        const i64 q = lower_bound_dev(adj2, rb, re, hi);
        const i64 e = eb[x] + (j - us[x]);
        if (q < re && adj2[q] == hi && e >= 0 && e < m) {  // always, for a CSR within the contract
          const i32 e2 = eid2[q];
          tau[e] = tau2[e2];
          if (rounds) rounds[e] = rounds2[e2];
        }
      }
    }
    __syncthreads();
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
  u32* dmax;      // maximum degree
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
  t.dmax = cv.take<u32>(1);
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
  // 2. degrees; with relabel = 1, the graph as given unless its degrees are skewed (the
  // caller has checked its size)
  PKT_HIP(hipMemsetAsync(r.dmax, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_degree, dim3(grid_r(n)), dim3(PKT_BLOCK), 0, s, n, off, r.key, r.dmax);
  PKT_LAUNCH_CHECK();
  if (opt.relabel == 1) {
    u32 dmax = 0;
    PKT_HIP(hipMemcpyAsync(&dmax, r.dmax, sizeof(u32), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    if ((i64)dmax * (i64)n < (i64)TRUSS_RELABEL_MIN_SKEW * two_m) {  // dmax below skew x (2m / n)
      truss_options o1 = opt;
      o1.validate = 0;  // done above
      truss_status st = run_single(wv, o1, stats, out, s, false);
      if (st) return st;
      if (timed) {
        float t_val = 0.f;
        PKT_HIP(hipEventElapsedTime(&t_val, ev[0], ev[1]));
        stats->ms_validate += t_val;
        stats->ms_total += t_val;
      }
      return TRUSS_OK;
    }
  }
  // 3. new ids by increasing (degree, id), the relabelled CSR
  truss_status st = kco_order_run(n, r.key, kco_bits((i64)n - 1), r.new_id, r.order, r.regionA, s);
  if (st) return st;
  st = kco_relabel_run(n, two_m, off, adj, r.new_id, r.order, r.off2, r.adj2, r.regionA, s);
  if (st) return st;
  if (timed) PKT_HIP(hipEventRecord(ev[2], s));
  // 4. the decomposition of the relabelled graph
  Work w2;
  work_layout(n, two_m, false, r.regionA, &w2);
  w2.off = r.off2;
  w2.adj = r.adj2;
  w2.id_order = true;  // new ids increase with (degree, id): the support walk needs no edge ids
  truss_options o2 = opt;
  o2.validate = 0;
  o2.relabel = 0;
  o2.peel_round = opt.peel_round ? r.rounds2 : nullptr;
  st = run_single(w2, o2, stats, r.tau2, s, false);
  if (st) return st;
  if (timed) PKT_HIP(hipEventRecord(ev[3], s));
  // 5. back to the input's edges
  PKT_HIP(hipMemsetAsync(r.arrive, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_upper_start, dim3(grid_r(n)), dim3(PKT_BLOCK), 0, s, n, off, adj, r.us);
  PKT_HIP(scan_launch(UpperLen{off, r.us, n}, r.partial, r.eb, r.arrive, s));
  hipLaunchKernelGGL(k_map_back, dim3(grid_r(two_m)), dim3(PKT_BLOCK), 0, s, n, two_m, off, adj, (const i64*)r.us,
                     (const i64*)r.eb, (const i32*)r.new_id, (const i64*)r.off2, (const i32*)r.adj2,
                     (const i32*)w2.eid, (const i32*)r.tau2, out, (const i32*)r.rounds2, opt.peel_round);
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
