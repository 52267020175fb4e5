// Batched decomposition of many small graphs.
#include <string.h>

#include <vector>

#include "truss.h"

namespace pkt {
truss_status run_single(const Work& w, const truss_options& opt, truss_stats* stats, i32* trussness,
                        hipStream_t s, bool support_only);
truss_status prepare_off64(Work& w, const i32* off32, hipStream_t s);
}  // namespace pkt

using namespace pkt;

extern "C" {

truss_status truss_batched_workspace_bytes(int32_t num_graphs, int64_t total_vtx_entries, int64_t total_adj,
                                           const truss_options* opt, size_t* bytes) {
  (void)opt;
  if (num_graphs < 0 || total_vtx_entries < 0 || total_adj < 0 || bytes == nullptr) {
    set_error("bad arguments to truss_batched_workspace_bytes");
    return TRUSS_E_ARG;
  }
  const i64 nv = total_vtx_entries < (i64)INT32_MAX ? total_vtx_entries : (i64)INT32_MAX;
  *bytes = work_layout((i32)nv, total_adj, true, nullptr, nullptr);
  return TRUSS_OK;
}

// One graph after another through the single-graph path.
truss_status truss_decompose_batched(int32_t num_graphs, const int64_t* graph_vtx_off,
                                     const int64_t* graph_adj_off, const int32_t* offsets_packed,
                                     const int32_t* adj_packed, int32_t* trussness_packed,
                                     int64_t total_vtx_entries, int64_t total_adj, void* workspace,
                                     size_t workspace_bytes, const truss_options* opt_in, truss_stats* stats,
                                     void* stream) {
  set_error("");
  if (num_graphs < 0 || (num_graphs > 0 && (!graph_vtx_off || !graph_adj_off))) {
    set_error("bad batch arguments");
    return TRUSS_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<i64> vo(num_graphs + 1), ao(num_graphs + 1);
  PKT_HIP(hipMemcpyAsync(vo.data(), graph_vtx_off, sizeof(i64) * (num_graphs + 1), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipMemcpyAsync(ao.data(), graph_adj_off, sizeof(i64) * (num_graphs + 1), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (vo[num_graphs] != total_vtx_entries || ao[num_graphs] != total_adj) {
    set_error("graph offset arrays disagree with the totals");
    return TRUSS_E_ARG;
  }
  truss_options opt;
  truss_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (stats) memset(stats, 0, sizeof(*stats));
  for (int g = 0; g < num_graphs; ++g) {
    const i64 nv = vo[g + 1] - vo[g] - 1;
    const i64 two_m = ao[g + 1] - ao[g];
    if (nv < 0 || two_m < 0 || (two_m & 1) || (ao[g] & 1)) {
      set_error("graph %d: bad offsets", g);
      return TRUSS_E_RANGE;
    }
    const size_t need = work_layout((i32)nv, two_m, true, nullptr, nullptr);
    if (workspace == nullptr || workspace_bytes < need) {
      set_error("workspace too small for graph %d", g);
      return TRUSS_E_WORKSPACE;
    }
    Work w;
    work_layout((i32)nv, two_m, true, workspace, &w);
    w.adj = adj_packed + ao[g];
    truss_status st = prepare_off64(w, offsets_packed + vo[g], s);
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
    }
  }
  return TRUSS_OK;
}

}  // extern "C"
