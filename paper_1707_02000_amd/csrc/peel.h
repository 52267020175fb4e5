// Peeling (level loop) shared definitions.
#pragma once
#include "mlp.h"
#include "truss.h"

#define SCAN_ITEMS 16        // alive-list entries per thread per tile of a level scan
#define SMALL_FRONTIER 2048  // frontiers up to this size may run as one fused launch
#ifndef SMALL_THREADS
#define SMALL_THREADS 512    // threads per block of the fused launch
#endif
#define FUSED_NARROW_BLOCKS 32
#define WIDE_NARROW_BLOCKS 256
// Launch constants a build may override (tuning runs):
#ifndef FUSED_THRESHOLD
#define FUSED_THRESHOLD 2048  // the heuristic fuses up to this size (end-to-end runs of the tuner's
                              // candidates: the single-block continuation favours the largest)
#endif
#ifndef FUSED_BLOCKS
#define FUSED_BLOCKS 512      // blocks of TRUSS_CHOICE_FUSED (measured: 512 beats 256 and 1024)
#endif
#ifndef WIDE_BLOCKS
#define WIDE_BLOCKS 2048      // blocks of TRUSS_CHOICE_WIDE
#endif
#ifndef WIDE_THREADS
#define WIDE_THREADS PKT_BLOCK  // threads per block of TRUSS_CHOICE_WIDE (one tile of items)
#endif
// Single-block continuation (host-driven loop only; see peel_args):
#ifndef ALONE_FRONTIER
#define ALONE_FRONTIER 512    // the deciding block goes on alone on frontiers up to this size,
#endif
#ifndef ALONE_ITEMS
#define ALONE_ITEMS 2048      // with at most this many intersection items,
#endif
// The working CSR is rebuilt without its processed edges once the edges left
// are under COMPACT_NUM / COMPACT_DEN of the edges it holds (7/8 measured best
// on R-MAT scale 22 among 1/2 .. 31/32: stale entries cost every later round's
// items more than the rebuilds; 3/4 ties it at scale 20).
#ifndef COMPACT_NUM
#define COMPACT_NUM 7
#define COMPACT_DEN 8
#endif
__host__ __device__ __forceinline__ bool needs_compact(i64 alive, i64 csr_edges) {
  return alive * COMPACT_DEN < csr_edges * COMPACT_NUM;
}
#ifndef ALONE_ALIVE
#define ALONE_ALIVE 32768     // and scans alone when the alive list is at most this long
#endif
#define GALLOP_K 8           // shorter-row entries per item when galloping
#define DECIDE_THREADS 512   // threads of the one-block kernel that picks a round's launch
#ifndef LEARNED_MIN_FRONTIER
#define LEARNED_MIN_FRONTIER 32768  // the learned policy consults the model above this frontier size;
                                    // smaller frontiers (most rounds) take the heuristic's launch: the
                                    // features and the forward pass cost more there than a choice gains
                                    // (end to end on R-MAT s20-s24 and Chung-Lu 2^23, 2048 to 131072
                                    // tried)
#endif
#define CHOICE_NONE (-1)     // Ctl::choice while no launch is picked for the current frontier

// Loop state published by k_decide for the pipelined host loop, in host-mapped
// slots (LOOP_SNAP_SLOTS, by sequence number).  Two 64-bit words per slot, each
// carrying the low 24 bits of the sequence number, so the host checks each word
// on its own and the device needs no fence between them:
//   w0 = tag | ncurr << 24 | (choice + 1) << 55 | done << 59 | compact << 60
//   w1 = tag | nalive << 24
// (compact: under half of the working adjacency's edges are left).
#define LOOP_SNAP_SLOTS 8
#define SNAP_TAG_MASK 0xFFFFFFull
struct LoopSnap {
  u64 w0, w1;
  u64 pad[6];  // one 64-byte line per slot
};
struct LoopState {
  i32 ncurr, choice, done, nalive, compact;
};

__host__ __device__ __forceinline__ u64 snap_w0(i64 seq, i32 ncurr, i32 choice, i32 done, i32 compact) {
  return ((u64)seq & SNAP_TAG_MASK) | ((u64)(u32)ncurr << 24) | ((u64)(u32)(choice + 1) << 55) |
         ((u64)(done != 0) << 59) | ((u64)(compact != 0) << 60);
}
__host__ __device__ __forceinline__ u64 snap_w1(i64 seq, i32 nalive) {
  return ((u64)seq & SNAP_TAG_MASK) | ((u64)(u32)nalive << 24);
}

// Everything a peeling kernel touches.
struct PeelArgs {
  Ctl* ctl;
  i32* F[3];  // frontier buffers; round buffers by Ctl::sel (cur_of, next_of, prev_of)
  i32* A0;
  i32* A1;
  const int2* el;
  CsrSet csr;
  i32* sw;  // support words (sw_make)
  i32* order;  // truss_options::peel_round, or NULL
  i64 m;  // edges
  i32 alone_frontier, alone_items, alone_alive;  // single-block continuation limits (0: none)
  int owner_higher;
  int single_round;
  const float* mlp;  // cost-model weights (TRUSS_VARIANT_LEARNED) or NULL
  int want_features; // frontier features: 0 never, 1 learned policy (large frontiers), 2 every decision (tracing)
  int multi;         // fused rounds run as one cooperative multi-round launch (k_psl_multi)
  int lite;          // rounds end in k_decide_lite (no continuation, features or cost model)
};

__device__ __forceinline__ i32* cur_of(const PeelArgs& a, int sel) { return a.F[sel]; }
__device__ __forceinline__ i32* next_of(const PeelArgs& a, int sel) { return a.F[sel == 2 ? 0 : sel + 1]; }
__device__ __forceinline__ i32* prev_of(const PeelArgs& a, int sel) { return a.F[sel == 0 ? 2 : sel - 1]; }

// The learned decision from the model's outputs y (log2 microseconds per
// launch choice) for a frontier of ncurr edges: the valid choice predicted
// fastest, if it beats the heuristic's launch by MLP_MARGIN; otherwise, and
// whenever an output is not finite, the heuristic's launch.
__device__ __forceinline__ int mlp_decide(const float* y, i32 ncurr) {
  const int h = ncurr <= FUSED_THRESHOLD ? TRUSS_CHOICE_FUSED : TRUSS_CHOICE_WIDE;
  int best = -1;
  float bv = INFINITY;
  for (int k = 0; k < MLP_OUT; ++k) {
    if ((k == TRUSS_CHOICE_FUSED || k == TRUSS_CHOICE_FUSED_NARROW) && ncurr > SMALL_FRONTIER) continue;
    if (!isfinite(y[k])) return h;
    if (y[k] < bv) {
      bv = y[k];
      best = k;
    }
  }
  return (best >= 0 && bv + MLP_MARGIN < y[h]) ? best : h;
}

namespace pkt {
CsrSet csr_set(const Work& w);
truss_status validate_input(const Work& w, hipStream_t s);
truss_status build_edges(const Work& w, hipStream_t s);
truss_status compute_support(const Work& w, hipStream_t s);
truss_status init_peel(const Work& w, hipStream_t s);
truss_status compact(const Work& w, hipStream_t s);
truss_status write_output(const Work& w, i32* out, hipStream_t s);
truss_status write_support(const Work& w, i32* out, hipStream_t s);
}  // namespace pkt
