// Device state of one single-graph decomposition: control block, working CSR
// set and workspace layout.
#pragma once
#include "common.h"

// Control block in device memory.  Kernels of the level loop read it at entry
// and gate themselves on it, so the same launch sequence serves the host-driven
// loop and the device-driven (graph-replayed) loop.
struct Ctl {
  i32 ncurr;       // edges in the current frontier F[sel]
  i32 nfound;      // edges appended to F[sel] by the level scan (atomic; becomes ncurr)
  i32 nnext;       // edges appended to the next frontier F[(sel + 1) % 3] (atomic)
  i32 nprev;       // edges of the previous round's frontier F[(sel + 2) % 3]
  i32 nalive;      // entries of the alive list A[asel]
  i32 nalive_out;  // entries written to A[asel ^ 1] by the level scan (atomic)
  i32 level;       // support level l
  i32 sel;         // frontier buffer of the current round (0..2, rotating)
  i32 asel;        // alive-list buffer in use
  i32 min_above;   // min support among edges kept alive by the last scan (atomic min)
  i32 done;        // 1 once every edge is processed
  u32 arrive;      // last-block-arrival counter (reset by the last block)
  i32 levels;      // level scans done
  i32 sublevels;   // frontier rounds done
  i32 processed;   // edges marked processed
  i32 csel;        // working CSR: 0 = input rows, 1 or 2 = compacted copies
  i32 csr_edges;   // edges present when the working CSR was built
  i32 compactions; // working-CSR rebuilds
  i32 variant;     // intersection search of the current round (TRUSS_VARIANT_BSEARCH / MERGE)
  i32 tmax_s;      // max final support (output pass)
  i64 items;       // unused
  i64 tri3;        // sum of initial supports (= 3 x triangles)
  i32 work_queue;  // next vertex for the support kernel's work queue
  i32 wide_launches;  // launches of the wide sub-level kernel that found work
  i64 wide_items;     // their intersection items
  i64 wide_frontier;  // their frontier edges
  // decision for the current frontier
  i32 choice;         // truss_choice picked for the round
  i32 policy;         // truss_variant policy of the run
  i32 force_choice;   // for TRUSS_VARIANT_FIXED
  float feat[8];      // features of the current frontier (TRUSS_NUM_FEATURES used)
  i32 scan_pending;   // level scan counted, not yet written (between its passes)
  u32 scan_arrive;    // last-block-arrival counter of the device-wide scans (scan.h)
  i32 chosen[TRUSS_NUM_CHOICES];  // rounds launched with each truss_choice
  i32 round_done;     // a round kernel ran; k_decide ends the round
  struct LoopSnap* snap;  // host-mapped loop-state slots (pipelined host loop) or null
  // multi-round launch (k_psl_multi): next-frontier counters of rounds r % 3 (zeroed by
  // the decision before the launch), grid-barrier arrivals and generation, and a flag
  // set when a barrier's bounded wait ran out
  i32 mcnt[3];
  u32 bar_count, bar_gen;
  i32 bar_timeout;
};

// Adjacency with edge ids: rows off[u]..off[u+1] of adj (sorted) and eid.
struct Csr {
  const i64* off;
  const i32* adj;
  const i32* eid;
};

// The working CSR is one of three: the input rows (with their edge ids) and two
// compaction targets used alternately.  Kernels pick by Ctl::csel so a captured
// launch sequence stays valid after a rebuild.
struct CsrSet {
  Csr c[3];
  __device__ __forceinline__ Csr pick(int k) const { return k == 0 ? c[0] : (k == 1 ? c[1] : c[2]); }
};

// Pointers into the workspace of one decomposition.
struct Work {
  i32 n;
  i64 two_m, m;
  const i64* off;   // input offsets (int64; a converted copy for the int32 entry point)
  const i32* adj;   // input adjacency
  i64* off64;       // int64 copy of int32 offsets (truss_decompose32 only)
  i32* deg;         // [n] degrees
  i32* locnt;       // [n] neighbours below the vertex
  i32* upcnt;       // [n] neighbours above the vertex
  i64* ebase;       // [n+1] first edge id of each row (exclusive scan of upper counts)
  i32* eid;         // [2m] edge id per adjacency slot
  int2* el;         // [m] endpoints (u < v)
  i32* sw;          // [m] support word: support and edge state (sw_make)
  i32* F[3];        // [m] frontiers: current, next, previous (rotating)
  i32* A[2];        // [m] alive lists
  i64* coff[2];     // [n+1] compacted offsets
  i32* cadj[2];     // [2m]
  i32* ceid[2];     // [2m]
  u8* flag;         // [2m] scratch flags
  i64* X;           // [2m+1] scan output (orientation / compaction / frontier work)
  i64* partial;     // [SCAN_BLOCKS+1]
  i32* bmin;        // [SCAN_BLOCKS] per-block minima of the level scan
  i64* ooff;        // [n+1] oriented CSR (aliases coff[1])
  i32* oadj;        // [m] (aliases cadj[1])
  i32* oeid;        // [m] (aliases ceid[1])
  Ctl* ctl;
  u32* verr;        // validation error bits
  bool no_alloc;    // host side allocates nothing: pageable readbacks, no events or graphs
  bool id_order;    // vertex ids follow the (degree, id) rank (a graph relabelled by it), so the
                    // oriented CSR is the upper half of every row and its slot k holds edge k
};

size_t work_layout(i32 n, i64 two_m, bool off32, void* base, Work* w);
