// Batched decomposition of many independent graphs, three ways (truss_options::
// batch_mode):
//   0 (default) the disjoint union: trussness is a property of each connected component, and
//     the edge order of the output (row-major, per graph, graphs back to back) is
//     exactly the edge order of the disjoint union of the graphs with vertex ids
//     shifted by the graph's vertex base, so the batch is decomposed as one union
//     graph: one level loop, one sequence of launches for every graph at once;
//   1 one graph after another through the single-graph path (a comparison point);
//   2 one persistent launch, every workgroup decomposing whole graphs taken from a
//     queue ordered by decreasing size (persist.hip).
#include <string.h>

#include <vector>

#include "truss.h"

namespace pkt {
truss_status run_single(const Work& w, const truss_options& opt, truss_stats* stats, i32* trussness,
                        hipStream_t s, bool support_only);
truss_status prepare_off64(Work& w, const i32* off32, hipStream_t s);
size_t persist_workspace_bytes(i32 G, i64 total_vtx, i64 total_adj);
truss_status run_persistent(i32 G, const i64* d_vo, const i64* d_ao, const i32* offs, const i32* adj, i32* out,
                            const std::vector<i64>& vo, const std::vector<i64>& ao, void* ws, const truss_options& opt,
                            truss_stats* stats, hipStream_t s);
}  // namespace pkt

using namespace pkt;

namespace {

// Structure of the batch, one thread per graph: both offset arrays start at 0,
// every graph has at least its one offsets entry (n_g >= 0), an even slot count,
// n_g <= 2^20 and m_g <= 2^24.  A graph with no offsets entry would shift every
// later graph onto the previous one's vertices.
__global__ __launch_bounds__(PKT_BLOCK) void k_batch_check(i32 G, const i64* __restrict__ vo,
                                                          const i64* __restrict__ ao, u32* __restrict__ err) {
  for (i64 g = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; g < G; g += (i64)gridDim.x * PKT_BLOCK) {
    const i64 nv = vo[g + 1] - vo[g] - 1, two_m = ao[g + 1] - ao[g];
    bool bad = nv < 0 || two_m < 0 || (two_m & 1) || nv > ((i64)1 << 20) || two_m > ((i64)2 << 24);
    if (g == 0) bad = bad || vo[0] != 0 || ao[0] != 0;
    if (bad) atomicOr(err, 1u);
  }
}

// Union offsets: the offsets of graph g (local, n_g + 1 entries at vtx_off[g])
// become global offsets adj_off[g] + local at union vertex vtx_off[g] - g + i.
__global__ __launch_bounds__(PKT_BLOCK) void k_union_offsets(i32 G, const i64* __restrict__ vo, const i64* __restrict__ ao,
                                                            const i32* __restrict__ loc, i64 total_vtx, i64 n_union,
                                                            i64* __restrict__ uoff, u32* __restrict__ err) {
  for (i64 idx = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; idx < total_vtx; idx += (i64)gridDim.x * PKT_BLOCK) {
    const i32 g = (i32)(upper_bound_dev(vo, (i64)0, (i64)G + 1, idx) - 1);
    const i64 i = idx - vo[g];
    const i64 ng = vo[g + 1] - vo[g] - 1;
    const i64 two_mg = ao[g + 1] - ao[g];
    const i32 x = loc[idx];
    if ((i == 0 && x != 0) || x < 0 || x > two_mg || (i == ng && x != two_mg)) atomicOr(err, VERR_RANGE);
    const i64 t = vo[g] - g + i;
    if (i < ng && t >= 0 && t < n_union) uoff[t] = ao[g] + x;
  }
}

// Union adjacency: local id + the graph's vertex base; local ids must be < n_g.
__global__ __launch_bounds__(PKT_BLOCK) void k_union_adj(i32 G, const i64* __restrict__ vo, const i64* __restrict__ ao,
                                                        const i32* __restrict__ adj, i64 total_adj,
                                                        i32* __restrict__ uadj, u32* __restrict__ err) {
  __shared__ i32 sg[2];
  for (i64 s0 = (i64)blockIdx.x * PKT_BLOCK; s0 < total_adj; s0 += (i64)gridDim.x * PKT_BLOCK) {
    const i64 s1 = min(s0 + PKT_BLOCK, total_adj) - 1;
    if (threadIdx.x == 0) sg[0] = (i32)(upper_bound_dev(ao, (i64)0, (i64)G + 1, s0) - 1);
    if (threadIdx.x == PKT_WAVE) sg[1] = (i32)(upper_bound_dev(ao, (i64)0, (i64)G + 1, s1) - 1);
    __syncthreads();
    const i64 j = s0 + threadIdx.x;
    if (j <= s1) {
      const i32 g = (i32)(upper_bound_dev(ao, (i64)sg[0], (i64)sg[1] + 1, j) - 1);
      const i64 ng = vo[g + 1] - vo[g] - 1;
      const i32 x = adj[j];
      if (x < 0 || x >= ng) atomicOr(err, VERR_RANGE);
      uadj[j] = (i32)(x + vo[g] - g);
    }
    __syncthreads();
  }
}

__global__ void k_set_i64(i64* p, i64 v) { *p = v; }

inline int grid_for_b(i64 count, int cap = 8192) {
  i64 g = (count + PKT_BLOCK - 1) / PKT_BLOCK;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

size_t union_bytes(i64 n_union, i64 total_adj) {
  return align_up(((size_t)n_union + 1) * sizeof(i64) + 1, 256) + align_up((size_t)total_adj * sizeof(i32) + 1, 256) +
         256;
}

}  // namespace

extern "C" {

truss_status truss_batched_workspace_bytes(int32_t num_graphs, int64_t total_vtx_entries, int64_t total_adj,
                                           const truss_options* opt, size_t* bytes) {
  (void)opt;
  if (num_graphs < 0 || total_vtx_entries < num_graphs || total_adj < 0 || (total_adj & 1) || bytes == nullptr) {
    set_error("bad arguments to truss_batched_workspace_bytes");
    return TRUSS_E_ARG;
  }
  const i64 n_union = total_vtx_entries - num_graphs;
  if (n_union > (i64)INT32_MAX || total_adj / 2 > (i64)INT32_MAX) {
    set_error("batch too large: %lld vertices, %lld edges", (long long)n_union, (long long)total_adj / 2);
    return TRUSS_E_RANGE;
  }
  const size_t single = work_layout((i32)n_union, total_adj, false, nullptr, nullptr);
  // the sequential mode reuses one single-graph workspace (int32 offsets converted)
  const size_t seq = work_layout((i32)n_union, total_adj, true, nullptr, nullptr);
  const size_t uni = single + union_bytes(n_union, total_adj);
  const size_t per = persist_workspace_bytes(num_graphs, total_vtx_entries, total_adj);
  *bytes = uni > seq ? uni : seq;
  if (per > *bytes) *bytes = per;
  return TRUSS_OK;
}

truss_status truss_decompose_batched(int32_t num_graphs, const int64_t* graph_vtx_off,
                                     const int64_t* graph_adj_off, const int32_t* offsets_packed,
                                     const int32_t* adj_packed, int32_t* trussness_packed,
                                     int64_t total_vtx_entries, int64_t total_adj, void* workspace,
                                     size_t workspace_bytes, const truss_options* opt_in, truss_stats* stats,
                                     void* stream) {
  set_error("");
  if (num_graphs < 0 || (num_graphs > 0 && (!graph_vtx_off || !graph_adj_off || !offsets_packed))) {
    set_error("bad batch arguments");
    return TRUSS_E_ARG;
  }
  if (total_adj > 0 && (!adj_packed || !trussness_packed)) {
    set_error("NULL adjacency or output");
    return TRUSS_E_ARG;
  }
  truss_options opt;
  truss_default_options(&opt);
  if (opt_in) opt = *opt_in;
  size_t need = 0;
  truss_status st = truss_batched_workspace_bytes(num_graphs, total_vtx_entries, total_adj, &opt, &need);
  if (st) return st;
  if (workspace == nullptr || workspace_bytes < need || ((uintptr_t)workspace & 255u)) {
    set_error("workspace: need %zu bytes at 256-byte alignment", need);
    return TRUSS_E_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (num_graphs == 0) return TRUSS_OK;
  i64 ends[2] = {0, 0};
  PKT_HIP(hipMemcpyAsync(&ends[0], graph_vtx_off + num_graphs, sizeof(i64), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipMemcpyAsync(&ends[1], graph_adj_off + num_graphs, sizeof(i64), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (ends[0] != total_vtx_entries || ends[1] != total_adj) {
    set_error("graph offset arrays end at %lld / %lld, totals given %lld / %lld", (long long)ends[0],
              (long long)ends[1], (long long)total_vtx_entries, (long long)total_adj);
    return TRUSS_E_ARG;
  }
  {
    // the per-graph structure, checked whatever opt.validate says: the union's vertex
    // bases and the per-graph limits depend on it
    Work w0;
    work_layout(0, 0, false, workspace, &w0);
    PKT_HIP(hipMemsetAsync(w0.verr, 0, sizeof(u32), s));
    hipLaunchKernelGGL(k_batch_check, dim3(grid_for_b(num_graphs)), dim3(PKT_BLOCK), 0, s, num_graphs, graph_vtx_off,
                       graph_adj_off, w0.verr);
    PKT_LAUNCH_CHECK();
    u32 bits = 0;
    PKT_HIP(hipMemcpyAsync(&bits, w0.verr, sizeof(u32), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    if (bits) {
      set_error("batch: graph offsets not starting at 0, a graph without its offsets entry, an odd slot count, "
                "or a graph above n = 2^20 / m = 2^24");
      return TRUSS_E_RANGE;
    }
  }

  if (opt.batch_mode < 0 || opt.batch_mode > 2) {
    set_error("batch_mode must be 0 (union), 1 (sequential) or 2 (persistent)");
    return TRUSS_E_ARG;
  }
  if (opt.batch_mode == 2) {
    std::vector<i64> vo(num_graphs + 1), ao(num_graphs + 1);
    PKT_HIP(hipMemcpyAsync(vo.data(), graph_vtx_off, sizeof(i64) * (num_graphs + 1), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipMemcpyAsync(ao.data(), graph_adj_off, sizeof(i64) * (num_graphs + 1), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    return run_persistent(num_graphs, graph_vtx_off, graph_adj_off, offsets_packed, adj_packed, trussness_packed, vo,
                          ao, workspace, opt, stats, s);
  }
  if (opt.batch_mode == 1) {
    // one graph after another through the single-graph path
    std::vector<i64> vo(num_graphs + 1), ao(num_graphs + 1);
    PKT_HIP(hipMemcpyAsync(vo.data(), graph_vtx_off, sizeof(i64) * (num_graphs + 1), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipMemcpyAsync(ao.data(), graph_adj_off, sizeof(i64) * (num_graphs + 1), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    for (int g = 0; g < num_graphs; ++g) {
      const i64 nv = vo[g + 1] - vo[g] - 1;
      const i64 two_m = ao[g + 1] - ao[g];
      if (nv < 0 || two_m < 0 || (two_m & 1) || (ao[g] & 1)) {
        set_error("graph %d: bad offsets", g);
        return TRUSS_E_RANGE;
      }
      Work w;
      work_layout((i32)nv, two_m, true, workspace, &w);
      w.adj = adj_packed + ao[g];
      st = prepare_off64(w, offsets_packed + vo[g], s);
      if (st) return st;
      truss_stats gs;
      st = run_single(w, opt, stats ? &gs : nullptr, trussness_packed + ao[g] / 2, s, false);
      if (st) {
        set_error("graph %d: %s", g, truss_last_error());
        return st;
      }
      if (stats) {
        stats->m += gs.m;
        stats->levels += gs.levels;
        stats->sublevels += gs.sublevels;
        stats->triangles += gs.triangles;
        stats->t_max = gs.t_max > stats->t_max ? gs.t_max : stats->t_max;
        stats->ms_total += gs.ms_total;
        stats->ms_support += gs.ms_support;
        stats->ms_peel += gs.ms_peel;
      }
    }
    return TRUSS_OK;
  }

  // disjoint union
  const i64 n_union = total_vtx_entries - num_graphs;
  Work w;
  const size_t single = work_layout((i32)n_union, total_adj, false, workspace, &w);
  Carver cv((char*)workspace + single);
  i64* uoff = cv.take<i64>((size_t)n_union + 1);
  i32* uadj = cv.take<i32>((size_t)total_adj);
  PKT_HIP(hipMemsetAsync(w.verr, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_union_offsets, dim3(grid_for_b(total_vtx_entries)), dim3(PKT_BLOCK), 0, s, num_graphs,
                     graph_vtx_off, graph_adj_off, offsets_packed, total_vtx_entries, n_union, uoff, w.verr);
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, uoff + n_union, total_adj);
  hipLaunchKernelGGL(k_union_adj, dim3(grid_for_b(total_adj)), dim3(PKT_BLOCK), 0, s, num_graphs, graph_vtx_off,
                     graph_adj_off, adj_packed, total_adj, uadj, w.verr);
  PKT_LAUNCH_CHECK();
  if (opt.validate) {
    u32 bits = 0;
    PKT_HIP(hipMemcpyAsync(&bits, w.verr, sizeof(u32), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    if (bits) {
      set_error("batch: local offsets or vertex ids out of range");
      return TRUSS_E_RANGE;
    }
  }
  w.off = uoff;
  w.adj = uadj;
  return run_single(w, opt, stats, trussness_packed, s, false);
}

}  // extern "C"
