// C ABI of libpkt: argument checks, workspace sizing, error reporting.
#include <stdarg.h>
#include <string.h>

#include <mutex>

#include "truss.h"

namespace pkt {

static thread_local char g_err[512] = {0};

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

truss_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return TRUSS_E_DEVICE;
}

truss_status run_single(const Work& w, const truss_options& opt, truss_stats* stats, i32* trussness,
                        hipStream_t s, bool support_only);
truss_status prepare_off64(Work& w, const i32* off32, hipStream_t s);
truss_status run_edge_list(const Work& w, i32* el_u, i32* el_v, hipStream_t s);
size_t relabel_workspace_bytes(i32 n, i64 two_m);
truss_status run_relabelled(i32 n, i64 two_m, const i64* off64_in, const i32* off32_in, const i32* adj, i32* out,
                            void* ws, const truss_options& opt, truss_stats* stats, hipStream_t s);

static truss_status check_options(const truss_options* o) {
  if (o->variant < TRUSS_VARIANT_AUTO || o->variant > TRUSS_VARIANT_LEARNED) {
    set_error("unknown variant %d", o->variant);
    return TRUSS_E_ARG;
  }
  if (o->owner_rule != 0 && o->owner_rule != 1) {
    set_error("owner_rule must be 0 or 1");
    return TRUSS_E_ARG;
  }
  if (o->device_loop < 0 || o->device_loop > 3) {
    set_error("device_loop must be 0 (host), 1 (device), 2 (device, hipGraph) or 3 (pipelined host)");
    return TRUSS_E_ARG;
  }
  if (o->relabel < 0 || o->relabel > 2) {
    set_error("relabel must be 0 (off), 1 (auto) or 2 (always)");
    return TRUSS_E_ARG;
  }
  if (o->steps_per_sync < 0) {
    set_error("steps_per_sync must be >= 0");
    return TRUSS_E_ARG;
  }
  if (o->variant == TRUSS_VARIANT_FIXED && (o->force_choice < 0 || o->force_choice >= TRUSS_NUM_CHOICES)) {
    set_error("force_choice must be a truss_choice");
    return TRUSS_E_ARG;
  }
  if (o->variant == TRUSS_VARIANT_LEARNED && o->mlp_weights == nullptr) {
    set_error("TRUSS_VARIANT_LEARNED needs mlp_weights");
    return TRUSS_E_ARG;
  }
  return TRUSS_OK;
}

// Reads offsets[n] (the slot count) from the device and checks sizes.
template <class OffT>
static truss_status read_two_m(i32 n, const OffT* offsets, hipStream_t s, i64* two_m) {
  OffT t = 0;
  PKT_HIP(hipMemcpyAsync(&t, offsets + n, sizeof(OffT), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (t < 0 || (t & 1)) {
    set_error("offsets[n] = %lld is negative or odd", (long long)t);
    return TRUSS_E_RANGE;
  }
  if ((i64)t / 2 > (i64)INT32_MAX) {
    set_error("m = %lld exceeds 2^31 - 1", (long long)t / 2);
    return TRUSS_E_RANGE;
  }
  *two_m = (i64)t;
  return TRUSS_OK;
}

template <class OffT>
static truss_status decompose_common(i32 n, const OffT* offsets, const i32* adj, i32* out, void* ws,
                                     size_t ws_bytes, const truss_options* opt_in, truss_stats* stats,
                                     void* stream, bool support_only) {
  set_error("");
  truss_options opt;
  truss_default_options(&opt);
  if (opt_in) opt = *opt_in;
  truss_status st = check_options(&opt);
  if (st) return st;
  if (n < 0 || (n > 0 && offsets == nullptr) || offsets == nullptr) {
    set_error("bad n or NULL offsets");
    return TRUSS_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  i64 two_m = 0;
  st = read_two_m(n, offsets, s, &two_m);
  if (st) return st;
  if (two_m > 0 && (adj == nullptr || out == nullptr)) {
    set_error("NULL adj or output");
    return TRUSS_E_ARG;
  }
  const bool off32 = sizeof(OffT) == 4;
  // the workspace truss_workspace_bytes gives for these options; relabel = 1 (auto) leaves
  // graphs below TRUSS_RELABEL_MIN_EDGES edges as they are
  const bool relabel_ws = opt.relabel != 0 && !support_only && two_m > 0;
  const bool relabel =
      relabel_ws && (opt.relabel == 2 || two_m / 2 >= (i64)TRUSS_RELABEL_MIN_EDGES);
  const size_t need =
      relabel_ws ? relabel_workspace_bytes(n, two_m) : work_layout(n, two_m, off32, nullptr, nullptr);
  if (ws == nullptr || ws_bytes < need || ((uintptr_t)ws & 255u)) {
    set_error("workspace: need %zu bytes at 256-byte alignment, got %zu at %p", need, ws_bytes, ws);
    return TRUSS_E_WORKSPACE;
  }
  if (relabel)
    return run_relabelled(n, two_m, off32 ? nullptr : (const i64*)offsets, off32 ? (const i32*)offsets : nullptr,
                          adj, out, ws, opt, stats, s);
  Work w;
  work_layout(n, two_m, off32, ws, &w);
  w.adj = adj;
  if (off32) {
    st = prepare_off64(w, (const i32*)offsets, s);
    if (st) return st;
  } else {
    w.off = (const i64*)offsets;
  }
  return run_single(w, opt, stats, out, s, support_only);
}

// ---- decomposition with no allocation at all
// The workspace of truss_decompose32_static lives in this file-scope device array,
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name (a host-side stand-in) to a kernel or a copy: it uses the device
// address hipGetSymbolAddress gives for the current device, looked up once per
// device.
#define PKT_SCRATCH_BYTES ((size_t)64 << 20)
static __device__ __align__(256) char scratch[PKT_SCRATCH_BYTES];

#define PKT_SCRATCH_DEVICES 64
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[PKT_SCRATCH_DEVICES] = {nullptr};

static truss_status scratch_of_current_device(void** out) {
  int dev = 0;
  PKT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= PKT_SCRATCH_DEVICES) {
    set_error("device %d is beyond the %d devices the static scratch serves", dev, PKT_SCRATCH_DEVICES);
    return TRUSS_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    if (p == nullptr || ((uintptr_t)p & 255u)) {
      set_error("static scratch at %p: not 256-byte aligned", p);
      return TRUSS_E_INTERNAL;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TRUSS_OK;
}

static truss_status decompose32_static(i32 n, const i32* offsets, const i32* adj, i32* out,
                                       const truss_options* opt_in, truss_stats* stats, void* stream) {
  set_error("");
  truss_options opt;
  truss_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.trace || opt.profile) {
    set_error("truss_decompose32_static takes no trace and no profile (both need host allocations)");
    return TRUSS_E_ARG;
  }
  if (opt.device_loop == 2 || opt.device_loop == 3) opt.device_loop = 1;  // no graph, no mapped host slots
  truss_status st = check_options(&opt);
  if (st) return st;
  if (n < 0 || offsets == nullptr) {
    set_error("bad n or NULL offsets");
    return TRUSS_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  i64 two_m = 0;
  st = read_two_m(n, offsets, s, &two_m);
  if (st) return st;
  if (two_m > 0 && (adj == nullptr || out == nullptr)) {
    set_error("NULL adj or output");
    return TRUSS_E_ARG;
  }
  const size_t need = work_layout(n, two_m, true, nullptr, nullptr);
  if (need > PKT_SCRATCH_BYTES) {
    set_error("graph needs %zu bytes of workspace; the static scratch holds %zu (use truss_decompose32)", need,
              PKT_SCRATCH_BYTES);
    return TRUSS_E_WORKSPACE;
  }
  void* ws = nullptr;
  st = scratch_of_current_device(&ws);
  if (st) return st;
  Work w;
  work_layout(n, two_m, true, ws, &w);
  w.adj = adj;
  w.no_alloc = true;
  st = prepare_off64(w, offsets, s);
  if (st) return st;
  return run_single(w, opt, stats, out, s, false);
}

}  // namespace pkt

using namespace pkt;

extern "C" {

truss_status truss_decompose32_static(int32_t n, const int32_t* offsets, const int32_t* adj, int32_t* trussness,
                                      const truss_options* opt, truss_stats* stats, void* stream) {
  return decompose32_static(n, offsets, adj, trussness, opt, stats, stream);
}

void truss_default_options(truss_options* opt) {
  if (!opt) return;
  memset(opt, 0, sizeof(*opt));
  opt->variant = TRUSS_VARIANT_AUTO;
  opt->device_loop = 3;
  opt->validate = 1;
  opt->owner_rule = 0;
  opt->compact = 1;
  opt->steps_per_sync = 0;
  opt->mlp_weights = nullptr;
  opt->trace = nullptr;
  opt->profile = 0;
  opt->batch_mode = 0;
  opt->force_choice = 0;
  opt->single_round = 0;
  opt->relabel = 1;
}

truss_status truss_workspace_bytes(int32_t n, int64_t two_m, const truss_options* opt, size_t* bytes) {
  if (n < 0 || two_m < 0 || (two_m & 1) || bytes == nullptr) {
    set_error("bad arguments to truss_workspace_bytes");
    return TRUSS_E_ARG;
  }
  if (two_m / 2 > (int64_t)INT32_MAX) {
    set_error("m exceeds 2^31 - 1");
    return TRUSS_E_RANGE;
  }
  size_t need = work_layout(n, two_m, true, nullptr, nullptr);
  if (opt == nullptr || opt->relabel) {
    const size_t r = relabel_workspace_bytes(n, two_m);
    if (r > need) need = r;
  }
  *bytes = need;
  return TRUSS_OK;
}

truss_status truss_decompose(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* trussness,
                             void* workspace, size_t workspace_bytes, const truss_options* opt,
                             truss_stats* stats, void* stream) {
  return decompose_common<i64>(n, offsets, adj, trussness, workspace, workspace_bytes, opt, stats, stream, false);
}

truss_status truss_decompose32(int32_t n, const int32_t* offsets, const int32_t* adj, int32_t* trussness,
                               void* workspace, size_t workspace_bytes, const truss_options* opt,
                               truss_stats* stats, void* stream) {
  return decompose_common<i32>(n, offsets, adj, trussness, workspace, workspace_bytes, opt, stats, stream, false);
}

truss_status truss_support(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* support,
                           void* workspace, size_t workspace_bytes, const truss_options* opt, void* stream) {
  return decompose_common<i64>(n, offsets, adj, support, workspace, workspace_bytes, opt, nullptr, stream, true);
}

truss_status truss_edge_list(int32_t n, const int64_t* offsets, const int32_t* adj, int32_t* el_u,
                             int32_t* el_v, void* workspace, size_t workspace_bytes, void* stream) {
  set_error("");
  if (n < 0 || offsets == nullptr) {
    set_error("bad n or NULL offsets");
    return TRUSS_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  i64 two_m = 0;
  truss_status st = read_two_m(n, offsets, s, &two_m);
  if (st) return st;
  if (two_m > 0 && (adj == nullptr || el_u == nullptr || el_v == nullptr)) {
    set_error("NULL adj or output");
    return TRUSS_E_ARG;
  }
  const size_t need = work_layout(n, two_m, false, nullptr, nullptr);
  if (workspace == nullptr || workspace_bytes < need || ((uintptr_t)workspace & 255u)) {
    set_error("workspace: need %zu bytes at 256-byte alignment", need);
    return TRUSS_E_WORKSPACE;
  }
  Work w;
  work_layout(n, two_m, false, workspace, &w);
  w.adj = adj;
  w.off = offsets;
  return run_edge_list(w, el_u, el_v, s);
}

const char* truss_strerror(truss_status status) {
  switch (status) {
    case TRUSS_OK: return "success";
    case TRUSS_E_ARG: return "invalid argument";
    case TRUSS_E_NOT_SIMPLE: return "input graph is not simple (unsorted row, duplicate or self-loop)";
    case TRUSS_E_NOT_SYMMETRIC: return "input graph is not symmetric";
    case TRUSS_E_RANGE: return "vertex id, offsets or size out of range";
    case TRUSS_E_WORKSPACE: return "workspace too small or misaligned";
    case TRUSS_E_DEVICE: return "HIP runtime error";
    case TRUSS_E_INTERNAL: return "internal error (iteration bound exceeded)";
  }
  return "unknown status";
}

const char* truss_last_error(void) { return g_err; }

}  // extern "C"
