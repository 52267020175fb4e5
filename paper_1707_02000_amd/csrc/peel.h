// Peeling (level loop) shared definitions.
#pragma once
#include "truss.h"

#define SCAN_ITEMS 16        // alive-list entries per thread per tile of a level scan
#define SMALL_FRONTIER 2048  // frontiers up to this size may run as one fused launch
#define FUSED_THRESHOLD 2048 // the heuristic fuses up to this size (end-to-end runs of the tuner's
                             // candidates: the fused launch's continuation favours the largest)
#define SMALL_THREADS 512    // threads per block of the fused launch
#define FUSED_BLOCKS 256     // blocks of TRUSS_CHOICE_FUSED
#define FUSED_NARROW_BLOCKS 32
#define WIDE_BLOCKS 2048     // blocks of TRUSS_CHOICE_WIDE
#define WIDE_NARROW_BLOCKS 256
#define ALONE_FRONTIER 512   // the fused launch's last block goes on alone on frontiers up to this size,
#define ALONE_ITEMS 2048     // with at most this many intersection items,
#define ALONE_ALIVE 32768    // and scans alone when the alive list is at most this long
#define GALLOP_K 8           // shorter-row entries per item when galloping
#define DECIDE_THREADS 512   // threads of the one-block kernel that picks a round's launch
#define CHOICE_NONE (-1)     // Ctl::choice while no launch is picked for the current frontier

// Loop state published by k_decide for the pipelined host loop (host-mapped,
// LOOP_SNAP_SLOTS slots by sequence number).
#define LOOP_SNAP_SLOTS 8
struct LoopSnap {
  i32 ncurr, choice, done, nalive, level, sublevels, processed, csr_edges;
  i64 seq;
  i64 pad[3];  // one 64-byte line per slot
};

// Everything a peeling kernel touches.
struct PeelArgs {
  Ctl* ctl;
  i32* F[3];  // frontier buffers; round buffers by Ctl::sel (cur_of, next_of, prev_of)
  i32* A0;
  i32* A1;
  const int2* el;
  CsrSet csr;
  i32* S;
  u8* state;
  i32* order;  // truss_options::peel_round, or NULL
  int owner_higher;
  int single_round;
  const float* mlp;  // cost-model weights (TRUSS_VARIANT_LEARNED) or NULL
  int want_features; // compute frontier features at each decision (learned policy or tracing)
};

__device__ __forceinline__ i32* cur_of(const PeelArgs& a, int sel) { return a.F[sel]; }
__device__ __forceinline__ i32* next_of(const PeelArgs& a, int sel) { return a.F[sel == 2 ? 0 : sel + 1]; }
__device__ __forceinline__ i32* prev_of(const PeelArgs& a, int sel) { return a.F[sel == 0 ? 2 : sel - 1]; }

namespace pkt {
CsrSet csr_set(const Work& w);
truss_status validate_input(const Work& w, hipStream_t s);
truss_status build_edges(const Work& w, hipStream_t s);
truss_status compute_support(const Work& w, hipStream_t s);
truss_status init_peel(const Work& w, hipStream_t s);
truss_status compact(const Work& w, hipStream_t s);
truss_status write_output(const Work& w, i32* out, hipStream_t s);
}  // namespace pkt
