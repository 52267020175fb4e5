// Level-synchronous peeling on gfx950 (Kabir and Madduri, arXiv:1707.02000,
// PKT section: Algorithm 4 -- level scan and sub-level loop; Algorithm 5 --
// sub-level processing; the text on concurrent triangle processing and on
// reducing concurrent array additions).
//
// Kernels (each reads the control block at entry and returns at once when the
// loop state or the round's launch choice says it has nothing to do):
//   k_scan_count, k_scan_write  level scan over the alive list in two passes
//                 (per-block counts and their prefix, then stable writes at the
//                 prefix offsets), so the alive list and the frontier stay in
//                 edge-id order
//   k_psl_small   a whole round of a frontier of <= SMALL_FRONTIER edges in one
//                 launch: every block builds the frontier's work prefix in LDS and
//                 takes a share of the intersection items
//   k_psl_bsearch wide round over a device-wide scan of the per-edge work (scan.h)
//   k_decide      one block after each of the above: ends the round (a counter
//                 update), with the host-driven loop goes on alone through further
//                 tiny rounds and short level scans, then picks the launch of the
//                 round on the frontier left (heuristic, forced, or the MLP cost
//                 model, which reads features sampled from the frontier) and
//                 publishes the loop state
// Edge states are round tags (three in rotation, the previous frontier turned
// processed by the next round's own blocks), so ending a round needs no pass over
// the edges.  The round kernels stay lean (their register counts set the
// occupancy of the item loops); the rest sits in k_decide.  The host reads the
// control block after every launch sequence, enqueues steps holding every
// launch, gated, and checks in batches (optionally as a replayed hipGraph), or
// (default) keeps launch sequences guessed from the last published state in
// flight.
#include <limits.h>
#include <math.h>
#include <string.h>

#include <chrono>
#include <vector>

#include "mlp.h"
#include "peel.h"
#include "psl.h"
#include "scan.h"

namespace {

// Shorter-row entries handled by one item: 1 (binary search per entry) or
// GALLOP_K (one binary search, then galloping forward in the longer row).
__device__ __forceinline__ i64 chunk_of(int variant) { return variant == TRUSS_VARIANT_MERGE ? GALLOP_K : 1; }

// Work of a frontier edge at level l (items): the shorter working row in chunks;
// nothing at level 0 (a frontier edge at level l lies in at most l triangles
// whose edges are all unprocessed).
__device__ __forceinline__ i64 work_of(const PeelArgs& a, const Csr& c, i32 e1, i32 l, int variant) {
  if (l == 0) return 0;
  const Rows r = rows_of(c, a.el[e1]);
  const i64 k = chunk_of(variant);
  return (r.slen + k - 1) / k;
}

// First index q in [p, le) with B[q] >= w: exponential steps from p, then a
// binary search inside the last step.
__device__ __forceinline__ i64 gallop(const i32* __restrict__ B, i64 p, i64 le, i32 w) {
  i64 lo = p, step = 1, hi;
  for (;;) {
    hi = lo + step - 1;
    if (hi >= le) {
      hi = le;
      break;
    }
    if (B[hi] >= w) {
      hi += 1;
      break;
    }
    lo = hi + 1;
    step <<= 1;
  }
  return lower_bound_dev(B, lo, hi, w);
}

// ---------------------------------------------------------------- features

__device__ __forceinline__ int log2_bin(i64 d) { return 63 - __clzll((unsigned long long)(d + 1)); }

#define FEAT_SAMPLE 512  // frontier edges sampled (evenly spaced) for the features

__device__ __forceinline__ bool is_fused(int c) { return c == TRUSS_CHOICE_FUSED || c == TRUSS_CHOICE_FUSED_NARROW; }
__device__ __forceinline__ bool is_wide(int c) {
  return c == TRUSS_CHOICE_WIDE || c == TRUSS_CHOICE_WIDE_NARROW || c == TRUSS_CHOICE_WIDE_GALLOP;
}
__device__ __forceinline__ bool is_wave(int c) { return c == TRUSS_CHOICE_WAVE; }
__device__ __forceinline__ bool is_hash(int c) { return c == TRUSS_CHOICE_HASH; }

// The built-in heuristic: fused launch up to FUSED_THRESHOLD frontier edges (the
// threshold the tuner's trace search picked), else the wide sequence.
__device__ __forceinline__ int heuristic_choice(int policy, i32 ncurr) {
  if (ncurr <= FUSED_THRESHOLD) return TRUSS_CHOICE_FUSED;
  return policy == TRUSS_VARIANT_MERGE ? TRUSS_CHOICE_WIDE_GALLOP : TRUSS_CHOICE_WIDE;
}

// Picks the launch of the round on the current frontier (ctl->ncurr > 0).
// Features (learned policy above LEARNED_MIN_FRONTIER edges, or tracing) come
// from up to FEAT_SAMPLE evenly spaced frontier edges.  Called by every thread of one block (blockDim.x >=
// MLP_H) after the control block's counts are final.
__device__ void decide(const PeelArgs& a, float* sx, float* sy, float* ha, float* hb, int* schoice) {
  Ctl* ctl = a.ctl;
  __shared__ i64 s_sum_deg, s_sum_min, s_cnt;
  __shared__ i32 s_max, s_hist[32];
  const bool feats = a.want_features == 2 || (a.want_features == 1 && ctl->ncurr > LEARNED_MIN_FRONTIER);
  // With the model in use, its weights are loaded into registers first and
  // staged in LDS after the features, so their load overlaps the feature reads.
  constexpr int WPER = (MLP_NPARAM + DECIDE_THREADS - 1) / DECIDE_THREADS;
  __shared__ float wl[MLP_NPARAM];
  const bool use_mlp = ctl->policy == TRUSS_VARIANT_LEARNED && a.mlp && feats && blockDim.x == DECIDE_THREADS;
  float wr[WPER];
  if (use_mlp) {
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int idx = threadIdx.x + k * DECIDE_THREADS;
      wr[k] = idx < MLP_NPARAM ? a.mlp[idx] : 0.f;
    }
  }
  if (feats) {
    if (threadIdx.x < 32) s_hist[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      s_sum_deg = s_sum_min = s_cnt = 0;
      s_max = 0;
    }
    __syncthreads();
    const i32 nc = ctl->ncurr;
    const i32* curr = cur_of(a, ctl->sel);
    const Csr c = a.csr.pick(ctl->csel);
    const i32 ns = min(nc, FEAT_SAMPLE);
    i64 sd = 0, sm = 0, cnt = 0;
    i32 mx = 0;
    for (i32 k = threadIdx.x; k < ns; k += blockDim.x) {
      const i32 e = curr[(i64)k * nc / ns];
      const int2 uv = a.el[e];
      const i64 du = c.off[uv.x + 1] - c.off[uv.x], dv = c.off[uv.y + 1] - c.off[uv.y];
      sd += du + dv;
      sm += min(du, dv);
      cnt += 2;
      mx = max(mx, (i32)max(du, dv));
      atomicAdd(&s_hist[min(31, log2_bin(du))], 1);
      atomicAdd(&s_hist[min(31, log2_bin(dv))], 1);
    }
    sd = wave_sum_i64(sd);
    sm = wave_sum_i64(sm);
    cnt = wave_sum_i64(cnt);
    mx = wave_max_i32(mx);
    if (lane_id() == 0) {
      atomicAdd((unsigned long long*)&s_sum_deg, (unsigned long long)sd);
      atomicAdd((unsigned long long*)&s_sum_min, (unsigned long long)sm);
      atomicAdd((unsigned long long*)&s_cnt, (unsigned long long)cnt);
      atomicMax(&s_max, mx);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double cn = (double)max((i64)1, s_cnt);
      i64 run = 0;
      int p99 = 0;
      for (int b = 0; b < 32; ++b) {
        run += s_hist[b];
        if ((double)run >= 0.99 * (double)s_cnt) {
          p99 = b + 1;
          break;
        }
      }
      sx[0] = log2f(1.f + (float)nc);
      sx[1] = log2f(1.f + (float)((double)s_sum_deg / cn));
      sx[2] = log2f(1.f + (float)s_max);
      sx[3] = (float)p99;  // log2(1 + p99 degree), in whole bins
      sx[4] = log2f(1.f + (float)ctl->level);
      sx[5] = log2f(1.f + (float)((double)s_sum_min / (cn * 0.5)));
    }
  } else if (threadIdx.x == 0) {
    for (int i = 0; i < 8; ++i) sx[i] = 0.f;
    sx[0] = log2f(1.f + (float)ctl->ncurr);
  }
  __syncthreads();
  const int policy = ctl->policy;
  if (use_mlp) {
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int idx = threadIdx.x + k * DECIDE_THREADS;
      if (idx < MLP_NPARAM) wl[idx] = wr[k];
    }
    __syncthreads();
    mlp_forward_block(wl, sx, sy, ha, hb);
  } else if (policy == TRUSS_VARIANT_LEARNED && a.mlp && feats) {
    mlp_forward_block(a.mlp, sx, sy, ha, hb);
  }
  if (threadIdx.x == 0) {
    const i32 nc = ctl->ncurr;
    int c = heuristic_choice(policy, nc);
    if (policy == TRUSS_VARIANT_FIXED) {
      const int f = ctl->force_choice;
      if (f >= 0 && f < TRUSS_NUM_CHOICES && (!is_fused(f) || nc <= SMALL_FRONTIER)) c = f;
    } else if (policy == TRUSS_VARIANT_LEARNED && a.mlp && feats) {
      c = mlp_decide(sy, nc);
    }
    ctl->choice = c;
    ctl->chosen[c] += 1;
    for (int k = 0; k < 3; ++k) ctl->mcnt[k] = 0;  // counters of a multi-round launch
    ctl->variant = (policy == TRUSS_VARIANT_MERGE || c == TRUSS_CHOICE_WIDE_GALLOP) ? TRUSS_VARIANT_MERGE
                                                                                     : TRUSS_VARIANT_BSEARCH;
    for (int i = 0; i < 8; ++i) ctl->feat[i] = i < TRUSS_NUM_FEATURES ? sx[i] : 0.f;
    *schoice = c;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- items

// Item t of frontier edge e1: chunk t of the shorter row, located in the
// longer row; for every triangle found with no processed edge, the decrement
// rule on both other edges (rd: the round index).  Edges that reached l come
// back in x0, x1 for the caller's append; more than two from one item are
// appended at once.
__device__ __forceinline__ void psl_item_rows(const PeelArgs& a, const Csr& c, i32 e1, const Rows& r, i64 t, i32 l,
                                              i32 rd, int variant, i32& x0, i32& x1, i32* spill_next,
                                              i32* spill_ctr) {
  const i64 k = chunk_of(variant);
  const i64 j0 = r.sb + t * k, j1 = min(r.sb + r.slen, j0 + k);
  i64 p = r.lb;
  for (i64 j = j0; j < j1; ++j) {
    const i32 es = c.eid[j];
    const i32 ws = a.sw[es];
    if (is_processed(sw_st(ws), rd)) continue;
    const i32 w = c.adj[j];
    p = (j == j0) ? lower_bound_dev(c.adj, p, r.le, w) : gallop(c.adj, p, r.le, w);
    if (p == r.le) break;
    if (c.adj[p] != w) continue;
    const i32 eo = c.eid[p];
    ++p;
    const i32 wo = a.sw[eo];
    if (is_processed(sw_st(wo), rd)) continue;
    i32 y[2];
    psl_tri(es, ws, eo, wo, e1, l, rd, a.sw, a.order, a.owner_higher, y[0], y[1]);
    for (int q = 0; q < 2; ++q) {
      if (y[q] < 0) continue;
      if (x0 < 0)
        x0 = y[q];
      else if (x1 < 0)
        x1 = y[q];
      else
        spill_next[atomicAdd(spill_ctr, 1)] = y[q];
    }
  }
}

__device__ __forceinline__ void psl_item(const PeelArgs& a, const Csr& c, i32 e1, i64 t, i32 l, i32 rd, int variant,
                                         i32& x0, i32& x1, i32* spill_next, i32* spill_ctr) {
  psl_item_rows(a, c, e1, rows_of(c, a.el[e1]), t, l, rd, variant, x0, x1, spill_next, spill_ctr);
}

__device__ __forceinline__ void append_next(i32 x0, i32 x1, i32* next, i32* counter) {
  const i32 s0 = wave_append_slot(x0 >= 0, counter);
  if (x0 >= 0) next[s0] = x0;
  const i32 s1 = wave_append_slot(x1 >= 0, counter);
  if (x1 >= 0) next[s1] = x1;
}

// ---------------------------------------------------------------- control

// Control-block update after a round: frontier processed, next frontier
// current, buffers swapped, an empty next frontier ends the level.
__device__ __forceinline__ void ctl_after_sublevel(Ctl* ctl, i32 nc, i32 nn, i32 sel) {
  ctl->processed += nc;
  ctl->ncurr = nn;
  ctl->nnext = 0;
  ctl->nprev = nc;
  ctl->sel = sel == 2 ? 0 : sel + 1;
  ctl->sublevels += 1;
  if (nn == 0) ctl->level += 1;
}

// Control-block update after a level scan: the found edges form the frontier;
// if none were found, jump to the lowest support left, or finish.
__device__ __forceinline__ void ctl_after_scan(Ctl* ctl, i32 nfound, i32 nkeep, i32 minabove, i32 asel) {
  ctl->ncurr = nfound;
  ctl->nfound = 0;
  ctl->nalive = nkeep;
  ctl->nalive_out = 0;
  ctl->asel = asel ^ 1;
  ctl->levels += 1;
  if (nfound == 0) {
    if (nkeep == 0)
      ctl->done = 1;
    else
      ctl->level = minabove;
  }
  ctl->min_above = INT_MAX;
}

// Stable compaction inside one tile of NT * SCAN_ITEMS entries, where entry
// t + k * NT belongs to thread t, slot k: its position among the taken (kept)
// entries of the tile, in entry order.  Per-wave ballots per slot, then an
// exclusive scan of the (slot, wave) counts in slot-major order.  Keeping entry
// order keeps the alive list and the frontier sorted by edge id, so the next
// scan's gathers stay coalesced.  *ntake, *nkeep get the tile's totals.
template <int NT>
__device__ __forceinline__ void stable_tile(u32 tk, u32 kp, i32* pt, i32* pk, i32* ntake, i32* nkeep, i64* cnt,
                                            i64* tmp) {
  constexpr int NW = NT / PKT_WAVE;
  const int lane = lane_id(), w = threadIdx.x / PKT_WAVE;
  const u64 lt = (1ull << lane) - 1ull;
  u64 bt[SCAN_ITEMS], bk[SCAN_ITEMS];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    bt[k] = __ballot((tk >> k) & 1u);
    bk[k] = __ballot((kp >> k) & 1u);
    if (lane == 0) cnt[k * NW + w] = ((i64)__popcll(bt[k]) << 32) | (i64)__popcll(bk[k]);
  }
  __syncthreads();
  const int E = SCAN_ITEMS * NW;
  const i64 v = (threadIdx.x < E) ? cnt[threadIdx.x] : 0;
  i64 tot;
  const i64 ex = block_excl_scan_i64<NT>(v, tmp, &tot);
  if (threadIdx.x < E) cnt[threadIdx.x] = ex;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const i64 o = cnt[k * NW + w];
    pt[k] = (i32)(o >> 32) + (i32)__popcll(bt[k] & lt);
    pk[k] = (i32)(o & 0xffffffffll) + (i32)__popcll(bk[k] & lt);
  }
  *ntake = (i32)(tot >> 32);
  *nkeep = (i32)(tot & 0xffffffffll);
  __syncthreads();  // cnt is reused by the next tile
}

// Level scan over tiles of the alive list (tiles tile0, tile0 + tstride, ...):
// edges still alive with support l join the frontier of round r (its tag);
// other alive edges are copied to the other alive list; edges no longer alive
// drop out.  Stable (entry order kept); one atomic per counter per tile of NT *
// SCAN_ITEMS entries (used by a single block, so the atomics are uncontended).
template <int NT>
__device__ void scan_tiles(const PeelArgs& a, i32 l, i32 r, i32 na, const i32* __restrict__ A, i32* __restrict__ Aout,
                           i32* __restrict__ curr, i64 tile0, i64 tstride, i32& mn, i64* tmp, i64* cnt, i32* sbase) {
  const i64 tile = (i64)NT * SCAN_ITEMS;
  for (i64 t0 = tile0 * tile; t0 < na; t0 += tstride * tile) {
    u32 tk = 0, kp = 0;
    i32 ev[SCAN_ITEMS];
    i32 wv[SCAN_ITEMS];
    // all loads first (no branch between them), then classify
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      const i64 i = t0 + (i64)k * NT + threadIdx.x;
      ev[k] = (i < na) ? A[i] : -1;
    }
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) wv[k] = a.sw[ev[k] < 0 ? 0 : ev[k]];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      if (ev[k] >= 0 && sw_st(wv[k]) == ST_ALIVE) {
        if (sw_sup(wv[k]) == l) {
          tk |= 1u << k;
        } else {
          kp |= 1u << k;
          mn = min(mn, sw_sup(wv[k]));
        }
      }
    }
    i32 pt[SCAN_ITEMS], pk[SCAN_ITEMS], nt, nk;
    stable_tile<NT>(tk, kp, pt, pk, &nt, &nk, cnt, tmp);
    if (threadIdx.x == 0) {
      sbase[0] = nt ? atomicAdd(&a.ctl->nfound, nt) : 0;
      sbase[1] = nk ? atomicAdd(&a.ctl->nalive_out, nk) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      if ((tk >> k) & 1u) {
        curr[sbase[0] + pt[k]] = ev[k];
        a.sw[ev[k]] = sw_make(l, round_tag(r));  // alive at l: nothing else writes it during a scan
        if (a.order) a.order[ev[k]] = r;
      } else if ((kp >> k) & 1u) {
        Aout[sbase[1] + pk[k]] = ev[k];
      }
    }
    __syncthreads();
  }
}

// The previous round's frontier turns processed (its tag is handed out again by
// the next round); every block of a round takes a strided share.
__device__ __forceinline__ void mark_prev(const PeelArgs& a, int sel, i32 r, i32 nprev, i64 tid, i64 stride) {
  const i32* prev = prev_of(a, sel);
  const i32 flip = (i32)(round_tag(r + 2) ^ ST_PROC);
  for (i64 i = tid; i < nprev; i += stride) atomicXor(&a.sw[prev[i]], flip);
}

// Rows of the frontier edges of a fused round, kept in LDS so that an item
// reads its edge from there instead of three dependent global loads.
struct EdgeRows {
  i64 sb[SMALL_FRONTIER], lb[SMALL_FRONTIER];
  i32 e1[SMALL_FRONTIER], L[SMALL_FRONTIER], slen[SMALL_FRONTIER];
};

// Exclusive prefix of the work of frontier edges [0, nc) into LDS P[0..nc]
// (nc <= SMALL_FRONTIER); returns the total.  With er, also each edge's rows.
// Every thread of the block calls it.
template <int NT>
__device__ i64 lds_work_prefix(const PeelArgs& a, const Csr& c, const i32* curr, i32 nc, i32 l, int variant, i64* P,
                               i64* tmp, EdgeRows* er = nullptr) {
  constexpr int PER = SMALL_FRONTIER / NT;
  const int i0 = threadIdx.x * PER;
  i64 w[PER];
  i64 sum = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = i0 + k;
    w[k] = 0;
    if (i < nc && l > 0) {  // level 0: no items (work_of)
      const i32 e1 = curr[i];
      const Rows r = rows_of(c, a.el[e1]);
      const i64 ck = chunk_of(variant);
      w[k] = (r.slen + ck - 1) / ck;
      if (er) {
        er->e1[i] = e1;
        er->sb[i] = r.sb;
        er->lb[i] = r.lb;
        er->L[i] = (i32)(r.le - r.lb);
        er->slen[i] = (i32)r.slen;
      }
    }
    sum += w[k];
  }
  i64 tot;
  i64 run = block_excl_scan_i64<NT>(sum, tmp, &tot);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = i0 + k;
    if (i < nc) P[i] = run;
    run += w[k];
  }
  if (threadIdx.x == 0) P[nc] = tot;
  __syncthreads();
  return tot;
}

// Next-frontier appends of one block, gathered in LDS and written out once at
// the end of the block's tiles with a single reservation on the global counter
// (every wave of the grid appending to that one counter would queue its atomics
// at one address, on each tile's critical path).  Entries past the buffer go
// straight to the global list, one reservation per wave.
#define APPEND_LDS 512
struct BlockAppend {
  i32 buf[APPEND_LDS];
  i32 n, base;
  __device__ __forceinline__ void add1(i32 x, i32* next, i32* counter) {
    const u64 mask = __ballot(x >= 0);
    if (mask == 0) return;
    const int lane = lane_id(), leader = __ffsll((unsigned long long)mask) - 1;
    i32 b = 0;
    if (lane == leader) b = atomicAdd(&n, (i32)__popcll(mask));
    b = __shfl(b, leader);
    const i32 slot = b + (i32)__popcll(mask & ((1ull << lane) - 1ull));
    const bool spill = x >= 0 && slot >= APPEND_LDS;
    if (x >= 0 && !spill) buf[slot] = x;
    const i32 g = wave_append_slot(spill, counter);  // every active lane
    if (spill) next[g] = x;
  }
  __device__ __forceinline__ void add(i32 x0, i32 x1, i32* next, i32* counter) {
    add1(x0, next, counter);
    add1(x1, next, counter);
  }
  // Every thread of the block, after its last add.
  __device__ __forceinline__ void flush(i32* next, i32* counter) {
    __syncthreads();
    const i32 k = min(n, (i32)APPEND_LDS);
    if (threadIdx.x == 0 && k > 0) base = atomicAdd(counter, k);
    __syncthreads();
    for (i32 t = threadIdx.x; t < k; t += (i32)blockDim.x) next[base + t] = buf[t];
  }
};

// Items [base, total) with the given stride, pairs located through LDS P (and
// the edges' rows from LDS when er is given); appends through ba when given, and
// to `next` with the round's counter (Ctl::nnext unless given).
template <int NT>
__device__ void lds_items(const PeelArgs& a, const Csr& c, const i32* curr, i32 nc, i32 l, i32 r, int variant,
                          const i64* P, i64 total, i64 base, i64 stride, i32* next, const EdgeRows* er = nullptr,
                          BlockAppend* ba = nullptr, i32* counter = nullptr) {
  if (counter == nullptr) counter = &a.ctl->nnext;
  for (i64 b = base; b < total; b += stride) {
    const i64 g = b + threadIdx.x;
    i32 x0 = -1, x1 = -1;
    if (g < total) {
      const i64 i = upper_bound_dev(P, (i64)0, (i64)nc + 1, g) - 1;
      if (er) {
        Rows rw;
        rw.sb = er->sb[i];
        rw.slen = er->slen[i];
        rw.lb = er->lb[i];
        rw.le = rw.lb + er->L[i];
        psl_item_rows(a, c, er->e1[i], rw, g - P[i], l, r, variant, x0, x1, next, counter);
      } else {
        psl_item(a, c, curr[i], g - P[i], l, r, variant, x0, x1, next, counter);
      }
    }
    if (ba)
      ba->add(x0, x1, next, counter);
    else
      append_next(x0, x1, next, counter);
  }
}

// Item g of a small round taken by a group of G lanes (rounds with at most one item
// per group over the grid; search variant): the entry's place in the longer row found
// G ways at a time -- G evenly spaced entries of the range loaded at once, their
// ballot against the entry narrowing it G-fold -- instead of one lane's binary
// search, so the chain of dependent loads is about log_G of the row length long
// instead of log2.  The group's first lane applies the decrement rule; x0, x1 as
// psl_item_rows.  Called by all G lanes of the group with the same g.
template <int G>
__device__ void group_item(const PeelArgs& a, const Csr& c, const EdgeRows& er, const i64* P, i32 nc, i64 g, i32 l,
                           i32 r, i32& x0, i32& x1) {
  const int lane = lane_id(), k = lane & (G - 1), shift = lane & (PKT_WAVE - G);  // shift: the group's first lane
  const u64 gmask = (G == PKT_WAVE) ? ~0ull : (((1ull << G) - 1ull) << shift);
  const i64 i = upper_bound_dev(P, (i64)0, (i64)nc + 1, g) - 1;
  const i64 j = er.sb[i] + (g - P[i]);
  const i32 es = c.eid[j];
  const i32 ws = a.sw[es];
  if (is_processed(sw_st(ws), r)) return;
  const i32 w = c.adj[j];
  const i64 le = er.lb[i] + er.L[i];
  // entries before lo are below w, entries from hi on are not
  i64 lo = er.lb[i], hi = le;
  while (hi - lo > G) {
    const i64 step = (hi - lo + G - 1) / G;
    const i64 q = lo + (i64)k * step;
    const i32 v = q < hi ? c.adj[q] : INT_MAX;
    const int below = __popcll(__ballot(v < w) & gmask);  // samples below w: a prefix of the group
    const i64 nhi = min(lo + (i64)below * step, hi);
    if (below > 0) lo += (i64)(below - 1) * step + 1;
    hi = nhi;
  }
  const i32 v = lo + k < hi ? c.adj[lo + k] : INT_MAX;
  const i64 p = lo + __popcll(__ballot(v < w) & gmask);  // first entry not below w
  if (k != 0 || p >= le || c.adj[p] != w) return;
  const i32 eo = c.eid[p];
  const i32 wo = a.sw[eo];
  if (is_processed(sw_st(wo), r)) return;
  psl_tri(es, ws, eo, wo, er.e1[i], l, r, a.sw, a.order, a.owner_higher, x0, x1);
}

// Items of a small round by groups of G lanes, one item per group (total <= groups).
template <int G>
__device__ __forceinline__ void group_items(const PeelArgs& a, const Csr& c, const EdgeRows& er, const i64* P, i32 nc,
                                            i64 total, i32 l, i32 r, i32& x0, i32& x1) {
  const i64 g = ((i64)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (g < total) group_item<G>(a, c, er, P, nc, g, l, r, x0, x1);
}

// Snapshot of the control block shared through LDS by one block.
struct CtlView {
  i32 done, ncurr, level, sel, csel, nalive, asel, variant, choice, r, nprev, round_done;
};

__device__ __forceinline__ void load_view(const Ctl* ctl, CtlView* v) {
  if (threadIdx.x == 0) {
    v->done = ctl->done;
    v->ncurr = ctl->ncurr;
    v->level = ctl->level;
    v->sel = ctl->sel;
    v->csel = ctl->csel;
    v->nalive = ctl->nalive;
    v->asel = ctl->asel;
    v->variant = ctl->variant;
    v->choice = ctl->choice;
    v->r = ctl->sublevels;
    v->nprev = ctl->nprev;
    v->round_done = ctl->round_done;
  }
  __syncthreads();
}

// Last-arriving-block detection among nblk blocks (each calls it once, all
// threads).
__device__ __forceinline__ bool arrive_last(Ctl* ctl, int* slast, int nblk) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    *slast = (atomicAdd(&ctl->arrive, 1u) == (u32)nblk - 1);
  }
  __syncthreads();
  const bool last = *slast;
  if (last) __threadfence();  // see every block's writes
  return last;
}

}  // namespace

// ---------------------------------------------------------------- single block

namespace {

// Loop state for the host: two self-tagged 64-bit words with system-scope
// stores into the host-mapped slot of sequence seq.
__device__ __forceinline__ void publish_snap(const PeelArgs& a, const Ctl* ctl, LoopSnap* snap, i64 seq) {
  LoopSnap* slot = snap + (seq & (LOOP_SNAP_SLOTS - 1));
  const i32 compact = needs_compact(a.m - ctl->processed, ctl->csr_edges);
  __hip_atomic_store(&slot->w0, snap_w0(seq, ctl->ncurr, ctl->choice, ctl->done, compact), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(&slot->w1, snap_w1(seq, ctl->nalive), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// LDS of a block that may go on alone (P: work prefix of a small frontier).
template <int NT>
struct AloneLds {
  i64 P[SMALL_FRONTIER + 1];
  i64 tmp[NT / PKT_WAVE];
  i64 cnt[SCAN_ITEMS * (NT / PKT_WAVE)];
  i32 sbase[2];
  i32 nn;
  CtlView v;
};

// The last block of a round or level scan goes on alone while the work stays
// small: rounds of at most PeelArgs::alone_frontier edges and alone_items items,
// and level scans of at most alone_alive entries.  It stops at once with
// single_round.
// On return the control block says what is left (ncurr > 0: a frontier whose
// launch is still to be picked; ncurr == 0: a level scan; or done).
template <int NT>
__device__ void go_alone(const PeelArgs& a, AloneLds<NT>& s) {
  Ctl* ctl = a.ctl;
  if (a.single_round) return;
  for (int iter = 0; iter < (1 << 20); ++iter) {
    load_view(ctl, &s.v);
    if (s.v.done) break;
    const i32 l = s.v.level, sel = s.v.sel, r = s.v.r;
    i32* curr = cur_of(a, sel);
    if (s.v.ncurr == 0) {
      if (s.v.nalive > a.alone_alive) break;
      const i32* A = s.v.asel ? a.A1 : a.A0;
      i32* Aout = s.v.asel ? a.A0 : a.A1;
      i32 mn = INT_MAX;
      scan_tiles<NT>(a, l, r, s.v.nalive, A, Aout, curr, 0, 1, mn, s.tmp, s.cnt, s.sbase);
      mn = wave_min_i32(mn);
      if (lane_id() == 0 && mn != INT_MAX) atomicMin(&ctl->min_above, mn);
      __syncthreads();  // every wave's minimum is in before thread 0 reads it
      if (threadIdx.x == 0)
        ctl_after_scan(ctl, atomicAdd(&ctl->nfound, 0), atomicAdd(&ctl->nalive_out, 0),
                       atomicAdd(&ctl->min_above, 0), s.v.asel);
      __syncthreads();
      continue;
    }
    if (s.v.ncurr > a.alone_frontier) break;
    const Csr c = a.csr.pick(s.v.csel);
    i32* next = next_of(a, sel);
    const i64 total = lds_work_prefix<NT>(a, c, curr, s.v.ncurr, l, s.v.variant, s.P, s.tmp);
    if (total > a.alone_items) break;
    mark_prev(a, sel, r, s.v.nprev, threadIdx.x, NT);
    lds_items<NT>(a, c, curr, s.v.ncurr, l, r, s.v.variant, s.P, total, 0, NT, next);
    __syncthreads();  // every wave's appends are counted before the count is read
    if (threadIdx.x == 0) ctl_after_sublevel(ctl, s.v.ncurr, atomicAdd(&ctl->nnext, 0), sel);
    __syncthreads();
  }
}

// End of a round or level scan in its last block: go on alone, then pick the
// launch of the frontier left, if any.
template <int NT>
__device__ void leave(const PeelArgs& a, AloneLds<NT>& s) {
  if (a.alone_frontier > 0 || a.alone_alive > 0) {  // else s.v is current already
    go_alone<NT>(a, s);
    load_view(a.ctl, &s.v);
  }
  __shared__ float sx[8], sy[MLP_OUT], ha[MLP_H], hb[MLP_H];
  __shared__ int schoice;
  if (!s.v.done && s.v.ncurr > 0) decide(a, sx, sy, ha, hb, &schoice);
}

}  // namespace

// ---------------------------------------------------------------- kernels

// Level scan in two launches, with no contended atomics: every block counts the
// taken and kept entries of its contiguous chunk of the alive list, and the last
// block to finish turns the counts into offsets (k_scan_count); every block then
// writes its entries at its offset, and the last one updates the control block
// and goes on (k_scan_write).  Chunks: gridDim.x blocks of ceil(na / gridDim.x)
// entries, tile-aligned; blocks past the end count nothing.
namespace {
__device__ __forceinline__ void scan_chunk(i32 na, int G, i64* c0, i64* c1) {
  const i64 tile = (i64)PKT_BLOCK * SCAN_ITEMS;
  const i64 chunk = ((na + G - 1) / G + tile - 1) / tile * tile;
  *c0 = min((i64)na, (i64)blockIdx.x * chunk);
  *c1 = min((i64)na, *c0 + chunk);
}

// Classifies the PKT_BLOCK * SCAN_ITEMS entries of the alive list from t0 (below
// end): bit k of tk / kp set when entry t0 + k * PKT_BLOCK + threadIdx.x is taken /
// kept.
__device__ __forceinline__ void classify(const PeelArgs& a, i32 l, const i32* __restrict__ A, i64 t0, i64 end,
                                         i32* ev, u32& tk, u32& kp, i32& mn) {
  i32 wv[SCAN_ITEMS];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const i64 i = t0 + (i64)k * PKT_BLOCK + threadIdx.x;
    ev[k] = (i < end) ? A[i] : -1;
  }
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) wv[k] = a.sw[ev[k] < 0 ? 0 : ev[k]];
  tk = kp = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (ev[k] >= 0 && sw_st(wv[k]) == ST_ALIVE) {
      if (sw_sup(wv[k]) == l) {
        tk |= 1u << k;
      } else {
        kp |= 1u << k;
        mn = min(mn, sw_sup(wv[k]));
      }
    }
  }
}
}  // namespace

// With tbits, the count pass keeps every tile's classification (taken bits in
// the low half, kept bits in the high half of one word per thread), so that the
// write pass gathers no support word again.
__global__ __launch_bounds__(PKT_BLOCK) void k_scan_count(PeelArgs a, i64* __restrict__ part, i32* __restrict__ bmin,
                                                         u32* __restrict__ tbits) {
  Ctl* ctl = a.ctl;
  if (ctl->done || ctl->ncurr != 0 || ctl->scan_pending) return;
  const int G = gridDim.x;
  const i32 l = ctl->level, na = ctl->nalive;
  const i32* A = ctl->asel ? a.A1 : a.A0;
  i64 c0, c1;
  scan_chunk(na, G, &c0, &c1);
  i64 packed = 0;
  i32 mn = INT_MAX;
  for (i64 t0 = c0; t0 < c1; t0 += (i64)PKT_BLOCK * SCAN_ITEMS) {
    i32 ev[SCAN_ITEMS];
    u32 tk, kp;
    classify(a, l, A, t0, c1, ev, tk, kp, mn);
    if (tbits) tbits[t0 / SCAN_ITEMS + threadIdx.x] = tk | (kp << 16);
    packed += ((i64)__popc(tk) << 32) | (i64)__popc(kp);
  }
  __shared__ i64 sp[PKT_BLOCK / PKT_WAVE];
  __shared__ i32 sm[PKT_BLOCK / PKT_WAVE];
  __shared__ int last;
  packed = wave_sum_i64(packed);
  mn = wave_min_i32(mn);
  if (lane_id() == 0) {
    sp[threadIdx.x / PKT_WAVE] = packed;
    sm[threadIdx.x / PKT_WAVE] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    i64 t = 0;
    i32 m = INT_MAX;
    for (int w = 0; w < PKT_BLOCK / PKT_WAVE; ++w) {
      t += sp[w];
      m = min(m, sm[w]);
    }
    part[blockIdx.x] = t;
    bmin[blockIdx.x] = m;
  }
  if (!arrive_last(ctl, &last, G)) return;
  // last block: chunk counts -> offsets; totals and the minimum kept support
  i64 running = 0;
  mn = INT_MAX;
  for (int base = 0; base < G; base += PKT_BLOCK) {
    const int i = base + threadIdx.x;
    const i64 v = (i < G) ? part[i] : 0;
    if (i < G) mn = min(mn, bmin[i]);
    i64 tot;
    const i64 ex = block_excl_scan_i64(v, sp, &tot);
    if (i < G) part[i] = running + ex;
    running += tot;
  }
  mn = wave_min_i32(mn);
  if (lane_id() == 0) sm[threadIdx.x / PKT_WAVE] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < PKT_BLOCK / PKT_WAVE; ++w) mn = min(mn, sm[w]);
    ctl->nfound = (i32)(running >> 32);
    ctl->nalive_out = (i32)(running & 0xffffffffll);
    ctl->min_above = mn;
    ctl->scan_pending = 1;
    ctl->arrive = 0;
  }
}

__global__ __launch_bounds__(PKT_BLOCK) void k_scan_write(PeelArgs a, const i64* __restrict__ part,
                                                         const u32* __restrict__ tbits) {
  Ctl* ctl = a.ctl;
  if (ctl->done || !ctl->scan_pending) return;
  const int G = gridDim.x;
  const i32 l = ctl->level, na = ctl->nalive, asel = ctl->asel, r = ctl->sublevels;
  const i32* A = asel ? a.A1 : a.A0;
  i32* Aout = asel ? a.A0 : a.A1;
  i32* curr = cur_of(a, ctl->sel);
  __shared__ i64 tmp[PKT_BLOCK / PKT_WAVE];
  __shared__ i64 cnt[SCAN_ITEMS * (PKT_BLOCK / PKT_WAVE)];
  __shared__ int last;
  i64 c0, c1;
  scan_chunk(na, G, &c0, &c1);
  const i64 base = part[blockIdx.x];
  i32 bt = (i32)(base >> 32), bk = (i32)(base & 0xffffffffll);
  i32 mn = INT_MAX;
  for (i64 t0 = c0; t0 < c1; t0 += (i64)PKT_BLOCK * SCAN_ITEMS) {
    i32 ev[SCAN_ITEMS];
    u32 tk, kp;
    if (tbits) {
#pragma unroll
      for (int k = 0; k < SCAN_ITEMS; ++k) {
        const i64 i = t0 + (i64)k * PKT_BLOCK + threadIdx.x;
        ev[k] = (i < c1) ? A[i] : -1;
      }
      const u32 b = tbits[t0 / SCAN_ITEMS + threadIdx.x];
      tk = b & 0xffffu;
      kp = b >> 16;
    } else {
      classify(a, l, A, t0, c1, ev, tk, kp, mn);
    }
    i32 pt[SCAN_ITEMS], pk[SCAN_ITEMS], nt, nk;
    stable_tile<PKT_BLOCK>(tk, kp, pt, pk, &nt, &nk, cnt, tmp);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      if ((tk >> k) & 1u) {
        curr[bt + pt[k]] = ev[k];
        a.sw[ev[k]] = sw_make(l, round_tag(r));  // alive at l: nothing else writes it during a scan
        if (a.order) a.order[ev[k]] = r;
      } else if ((kp >> k) & 1u) {
        Aout[bk + pk[k]] = ev[k];
      }
    }
    bt += nt;
    bk += nk;
  }
  if (!arrive_last(ctl, &last, G)) return;
  if (threadIdx.x == 0) {
    ctl_after_scan(ctl, ctl->nfound, ctl->nalive_out, ctl->min_above, asel);
    ctl->scan_pending = 0;
    ctl->choice = CHOICE_NONE;  // k_decide follows
    ctl->arrive = 0;
  }
}

// A whole round of a frontier of at most SMALL_FRONTIER edges: every block
// builds the frontier's work prefix in LDS and takes its share of the items
// (k_decide follows and ends the round).
// TRUSS_CHOICE_FUSED_NARROW uses the first FUSED_NARROW_BLOCKS blocks of the grid.
__global__ __launch_bounds__(SMALL_THREADS) void k_psl_small(PeelArgs a) {
  Ctl* ctl = a.ctl;
  __shared__ i64 P[SMALL_FRONTIER + 1];
  __shared__ i64 tmp[SMALL_THREADS / PKT_WAVE];
  __shared__ EdgeRows er;
  __shared__ CtlView v;
  __shared__ BlockAppend ba;
  load_view(ctl, &v);
  if (v.done || v.ncurr == 0 || v.ncurr > SMALL_FRONTIER || !is_fused(v.choice)) return;
  const int nblk = v.choice == TRUSS_CHOICE_FUSED_NARROW ? min((int)gridDim.x, FUSED_NARROW_BLOCKS) : gridDim.x;
  if ((int)blockIdx.x >= nblk) return;
  const i32 nc = v.ncurr, l = v.level, sel = v.sel, r = v.r;
  const Csr c = a.csr.pick(v.csel);
  const i32* curr = cur_of(a, sel);
  i32* next = next_of(a, sel);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->round_done = 1;
  if (threadIdx.x == 0) ba.n = 0;  // visible after the prefix's barrier
  mark_prev(a, sel, v.r, v.nprev, (i64)blockIdx.x * SMALL_THREADS + threadIdx.x, (i64)nblk * SMALL_THREADS);
  const i64 total = lds_work_prefix<SMALL_THREADS>(a, c, curr, nc, l, v.variant, P, tmp, &er);
  // few items: a group of lanes per item, as wide as the grid allows (the group
  // searches G ways at a time); otherwise one lane per item
  const i64 lanes = (i64)nblk * SMALL_THREADS;
  if (v.variant == TRUSS_VARIANT_BSEARCH && total * 8 <= lanes) {
    i32 x0 = -1, x1 = -1;
    if (total * 64 <= lanes)
      group_items<64>(a, c, er, P, nc, total, l, r, x0, x1);
    else if (total * 32 <= lanes)
      group_items<32>(a, c, er, P, nc, total, l, r, x0, x1);
    else if (total * 16 <= lanes)
      group_items<16>(a, c, er, P, nc, total, l, r, x0, x1);
    else
      group_items<8>(a, c, er, P, nc, total, l, r, x0, x1);
    ba.add(x0, x1, next, &ctl->nnext);
  } else {
    lds_items<SMALL_THREADS>(a, c, curr, nc, l, r, v.variant, P, total, (i64)blockIdx.x * SMALL_THREADS,
                             (i64)nblk * SMALL_THREADS, next, &er, &ba);
  }
  ba.flush(next, &ctl->nnext);
}

// Grid barrier of a cooperative launch (every block resident): release this
// block's writes, arrive, wait for the generation to move on, acquire everyone
// else's.  The wait is bounded: after MULTI_SPIN polls the block gives up and sets
// Ctl::bar_timeout, which the host turns into an error, so a kernel can never spin
// for good.  Every thread of every block calls it; returns false after a timeout.
#define MULTI_SPIN (1 << 22)
__device__ __forceinline__ bool grid_barrier(Ctl* ctl, u32 nblk, int* sflag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const u32 g = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    if (atomicAdd(&ctl->bar_count, 1u) == nblk - 1) {
      __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->bar_gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int spins = 0;
      while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > MULTI_SPIN) {
          atomicExch(&ctl->bar_timeout, 1);
          ok = 0;
          break;
        }
      }
    }
    __threadfence();
    *sflag = ok && atomic_load_relaxed(&ctl->bar_timeout) == 0;
  }
  __syncthreads();
  return *sflag != 0;
}

// Consecutive rounds of small frontiers (at most SMALL_FRONTIER edges, launch choice
// TRUSS_CHOICE_FUSED) in one cooperative launch of MULTI_BLOCKS blocks: every round
// runs as in k_psl_small on the blocks' share of the items, then all blocks meet at
// a grid barrier instead of a kernel boundary.  Every block reads the next
// frontier's size after the barrier and keeps its own copy of the loop state; the
// next-frontier counter of round r is Ctl::mcnt[r % 3] (zeroed by the decision
// before the launch, and by block 0 a round ahead: round r + 1's counter was last
// read before barrier r - 1).  The loop stops when the next frontier is empty (the
// level is done) or too large for a fused round; block 0 then writes the loop state
// to the control block and k_decide picks the next launch.
#ifndef MULTI_BLOCKS
#define MULTI_BLOCKS 64
#endif
__global__ __launch_bounds__(SMALL_THREADS) void k_psl_multi(PeelArgs a) {
  Ctl* ctl = a.ctl;
  __shared__ i64 P[SMALL_FRONTIER + 1];
  __shared__ i64 tmp[SMALL_THREADS / PKT_WAVE];
  __shared__ EdgeRows er;
  __shared__ CtlView v;
  __shared__ BlockAppend ba;
  __shared__ int sflag;
  load_view(ctl, &v);  // every block sees the same state: nothing writes it before the end
  if (v.done || v.ncurr == 0 || v.ncurr > SMALL_FRONTIER || v.choice != TRUSS_CHOICE_FUSED) return;
  const u32 nblk = gridDim.x;
  const i32 l = v.level;
  const Csr c = a.csr.pick(v.csel);
  i32 nc = v.ncurr, sel = v.sel, r = v.r, nprev = v.nprev, rounds = 0, processed = 0;
  for (;;) {
    const i32* curr = cur_of(a, sel);
    i32* next = next_of(a, sel);
    i32* counter = &ctl->mcnt[r % 3];
    if (threadIdx.x == 0) ba.n = 0;  // visible after the prefix's barrier
    mark_prev(a, sel, r, nprev, (i64)blockIdx.x * SMALL_THREADS + threadIdx.x, (i64)nblk * SMALL_THREADS);
    const i64 total = lds_work_prefix<SMALL_THREADS>(a, c, curr, nc, l, v.variant, P, tmp, &er);
    lds_items<SMALL_THREADS>(a, c, curr, nc, l, r, v.variant, P, total, (i64)blockIdx.x * SMALL_THREADS,
                             (i64)nblk * SMALL_THREADS, next, &er, &ba, counter);
    ba.flush(next, counter);
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->mcnt[(r + 1) % 3] = 0;
    const bool ok = grid_barrier(ctl, nblk, &sflag);
    const i32 nn = atomic_load_relaxed(counter);
    processed += nc;
    nprev = nc;
    sel = sel == 2 ? 0 : sel + 1;
    ++r;
    ++rounds;
    nc = nn;
    if (!ok || nn == 0 || nn > SMALL_FRONTIER) break;
    __syncthreads();  // ba and the LDS prefix are rewritten by the next round
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->processed += processed;
    ctl->ncurr = nc;
    ctl->nnext = 0;
    ctl->nprev = nprev;
    ctl->sel = sel;
    ctl->sublevels += rounds;
    ctl->chosen[TRUSS_CHOICE_FUSED] += rounds - 1;
    if (nc == 0) ctl->level += 1;
    ctl->choice = CHOICE_NONE;  // k_decide picks the next launch
    ctl->round_done = 0;
  }
}

// Work of frontier edge i for the device-wide scan (wide rounds above level 0).
struct WideLen {
  PeelArgs a;
  __device__ bool active() const {
    const Ctl* c = a.ctl;
    return !c->done && c->ncurr > 0 && c->level > 0 && is_wide(c->choice);
  }
  __device__ i64 count() const { return a.ctl->ncurr; }
  __device__ i64 len(i64 i) const {
    const Ctl* c = a.ctl;
    const i32* curr = cur_of(a, c->sel);
    return work_of(a, a.csr.pick(c->csel), curr[i], c->level, c->variant);
  }
};

// Tile of the wide round whose items all belong to one frontier edge (search
// variant: one shorter-row entry per item).  The block stages NSAMP evenly
// spaced entries of the longer row in LDS (the whole row when it is at most
// NSAMP long, as for most of the work on skewed graphs); a lane finds the bracket of its entry among the samples in LDS and
// binary-searches only that bracket, at most `step` contiguous entries, in
// memory.  A block's next tile of the same edge keeps the staged samples.
#ifndef NSAMP
#define NSAMP 4096
#endif

struct TileEdge {
  i64 i0;            // frontier index of the staged edge (-1: none)
  i64 sb, lb, step;  // shorter-row start, longer-row start, sample spacing
  i32 e1, L, ns;     // edge id, longer-row length, samples staged
};

__device__ void tile_one_edge(const PeelArgs& a, const Csr& c, const i32* curr, const i64* __restrict__ P, i64 i0,
                              i64 base, i64 total, i32 l, i32 r, i32* next, TileEdge& te, i32* samp,
                              BlockAppend& ba) {
  if (te.i0 != i0) {  // block-uniform
    __syncthreads();  // the previous tile's lanes are done with samp
    if (threadIdx.x == 0) {
      const i32 e1 = curr[i0];
      const Rows rw = rows_of(c, a.el[e1]);
      const i64 L = rw.le - rw.lb;
      const i64 step = L > NSAMP ? (L + NSAMP - 1) / NSAMP : 1;
      te.i0 = i0;
      te.e1 = e1;
      te.sb = rw.sb;
      te.lb = rw.lb;
      te.L = (i32)L;
      te.step = step;
      te.ns = (i32)((L + step - 1) / step);
    }
    __syncthreads();
    for (i32 k = threadIdx.x; k < te.ns; k += WIDE_THREADS) samp[k] = c.adj[te.lb + (i64)k * te.step];
    __syncthreads();
  }
  const i64 g = base + threadIdx.x;
  i32 x0 = -1, x1 = -1;
  if (g < total) {
    // The entry's edge id and state are read only once a triangle is found: most
    // entries find none, and the search here costs no memory access past the
    // entry itself (LDS, or one line of the longer row).
    const i64 j = te.sb + (g - P[i0]);
    const i32 w = c.adj[j];
    i32 lo = 0, hi = te.ns;  // first sample >= w
    while (lo < hi) {
      const i32 mid = (lo + hi) >> 1;
      if (samp[mid] < w)
        lo = mid + 1;
      else
        hi = mid;
    }
    i64 p = -1;
    if (lo < te.ns && samp[lo] == w) {
      p = te.lb + (i64)lo * te.step;
    } else if (te.step > 1) {  // between samples lo - 1 and lo: positions ((lo-1)*step, lo*step)
      const i64 q0 = lo > 0 ? (i64)(lo - 1) * te.step + 1 : 0;
      const i64 q1 = min((i64)lo * te.step, (i64)te.L);
      const i64 q = lower_bound_dev(c.adj, te.lb + q0, te.lb + q1, w);
      if (q < te.lb + q1 && c.adj[q] == w) p = q;
    }
    if (p >= 0) {
      const i32 es = c.eid[j], eo = c.eid[p];
      const i32 ws = a.sw[es], wo = a.sw[eo];
      if (!is_processed(sw_st(ws), r) && !is_processed(sw_st(wo), r)) {
        psl_tri(es, ws, eo, wo, te.e1, l, r, a.sw, a.order, a.owner_higher, x0, x1);
      }
    }
  }
  ba.add(x0, x1, next, &a.ctl->nnext);
}

// Wide round: one thread per intersection item over the whole grid, items
// located through the device-wide work prefix P (not read at level 0, where
// there are no items); k_decide follows and ends the round.  Block b takes tiles
// of PKT_BLOCK items b, b + blocks, b + 2 blocks, ... (strided: the items' cost
// grows along the frontier, whose edges come in edge-id order, so fixed contiguous
// ranges would leave the last blocks with the dearest tiles); a tile inside one edge's items
// takes the staged-sample path (tile_one_edge), any other tile locates every
// item's edge and searches the longer row directly.  TRUSS_CHOICE_WIDE_NARROW
// uses the first WIDE_NARROW_BLOCKS blocks.  Kept lean: its register count sets
// the occupancy of the item loop, and no block fences or counts arrivals (a
// device-scope fence per block costs more than the kernel boundary that orders
// the round's end).
__global__ __launch_bounds__(WIDE_THREADS) void k_psl_bsearch(PeelArgs a, const i64* __restrict__ P) {
  Ctl* ctl = a.ctl;
  __shared__ CtlView v;
  __shared__ i64 sp[2];
  __shared__ TileEdge te;
  __shared__ i32 samp[NSAMP];
  __shared__ BlockAppend ba;
  load_view(ctl, &v);
  if (v.done || v.ncurr == 0 || !is_wide(v.choice)) return;
  const int nblk = v.choice == TRUSS_CHOICE_WIDE_NARROW ? min((int)gridDim.x, WIDE_NARROW_BLOCKS) : gridDim.x;
  if ((int)blockIdx.x >= nblk) return;
  const i32 nc = v.ncurr, l = v.level, sel = v.sel, r = v.r;
  const i64 npairs = nc;
  const i64 total = l > 0 ? P[npairs] : 0;
  const int variant = v.variant;
  const i32* curr = cur_of(a, sel);
  i32* next = next_of(a, sel);
  const Csr c = a.csr.pick(v.csel);
  mark_prev(a, sel, v.r, v.nprev, (i64)blockIdx.x * WIDE_THREADS + threadIdx.x, (i64)nblk * WIDE_THREADS);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->round_done = 1;
    if (total > 0) {  // accounting for the roofline report
      ctl->wide_items += total;
      ctl->wide_frontier += npairs;
      ctl->wide_launches += 1;
    }
  }
  if (threadIdx.x == 0) {
    te.i0 = -1;
    ba.n = 0;
  }
  const i64 tiles = (total + WIDE_THREADS - 1) / WIDE_THREADS;
  for (i64 tile = blockIdx.x; tile < tiles; tile += nblk) {
    const i64 base = tile * WIDE_THREADS;
    if (threadIdx.x == 0) sp[0] = upper_bound_dev(P, (i64)0, npairs + 1, base) - 1;
    if (threadIdx.x == PKT_WAVE)
      sp[1] = upper_bound_dev(P, (i64)0, npairs + 1, min(base + WIDE_THREADS, total) - 1) - 1;
    __syncthreads();
    const i64 s0 = sp[0], s1 = sp[1];
    if (s0 == s1 && variant == TRUSS_VARIANT_BSEARCH) {
      tile_one_edge(a, c, curr, P, s0, base, total, l, r, next, te, samp, ba);
    } else {
      const i64 g = base + threadIdx.x;
      i32 x0 = -1, x1 = -1;
      if (g < total) {
        const i64 i = upper_bound_dev(P, s0, s1 + 1, g) - 1;
        psl_item(a, c, curr[i], g - P[i], l, r, variant, x0, x1, next, &ctl->nnext);
      }
      ba.add(x0, x1, next, &ctl->nnext);
    }
    __syncthreads();
  }
  ba.flush(next, &ctl->nnext);
}

// Round of one wave per frontier edge (TRUSS_CHOICE_WAVE): no work prefix and no
// scan launches; wave g of the grid takes frontier edges g, g + waves, ... and
// merges (or, for skewed rows, searches) the edge's two rows itself (wave_edge:
// coalesced row loads, the 64-entry chunks located among each other by lane
// shuffles).  k_decide follows and ends the round.
struct WaveAppend {
  BlockAppend* ba;
  i32* next;
  i32* counter;
  __device__ __forceinline__ void add(i32 x0, i32 x1) { ba->add(x0, x1, next, counter); }
};

__global__ __launch_bounds__(WIDE_THREADS) void k_psl_wave(PeelArgs a) {
  Ctl* ctl = a.ctl;
  __shared__ CtlView v;
  __shared__ BlockAppend ba;
  load_view(ctl, &v);
  if (v.done || v.ncurr == 0 || !is_wave(v.choice)) return;
  const i32 nc = v.ncurr, l = v.level, sel = v.sel, r = v.r;
  const i32* curr = cur_of(a, sel);
  i32* next = next_of(a, sel);
  const Csr c = a.csr.pick(v.csel);
  mark_prev(a, sel, r, v.nprev, (i64)blockIdx.x * WIDE_THREADS + threadIdx.x, (i64)gridDim.x * WIDE_THREADS);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->round_done = 1;
  if (threadIdx.x == 0) ba.n = 0;
  __syncthreads();
  WaveAppend app{&ba, next, &ctl->nnext};
  if (l > 0) {  // level 0: frontier edges lie in no triangle
    constexpr int WPB = WIDE_THREADS / PKT_WAVE;
    const i64 waves = (i64)gridDim.x * WPB;
    for (i64 i = (i64)blockIdx.x * WPB + threadIdx.x / PKT_WAVE; i < nc; i += waves) {
      const i32 e1 = curr[i];
      wave_edge(c, rows_of(c, a.el[e1]), e1, l, r, a.sw, a.order, a.owner_higher, app);
    }
  }
  ba.flush(next, &ctl->nnext);
}

// Round of one wave per frontier edge with the longer row hashed into LDS
// (TRUSS_CHOICE_HASH): workgroups of one wave, HASH_BLOCKS of them; workgroup g
// takes frontier edges g, g + HASH_BLOCKS, ...  No work prefix, no scan launches.
#define HASH_BLOCKS 8192
__global__ __launch_bounds__(PKT_WAVE) void k_psl_hash(PeelArgs a) {
  Ctl* ctl = a.ctl;
  __shared__ CtlView v;
  __shared__ BlockAppend ba;
  __shared__ i32 keys[WAVE_HASH_SLOTS];
  __shared__ unsigned short pos[WAVE_HASH_SLOTS];
  load_view(ctl, &v);
  if (v.done || v.ncurr == 0 || !is_hash(v.choice)) return;
  const i32 nc = v.ncurr, l = v.level, sel = v.sel, r = v.r;
  const i32* curr = cur_of(a, sel);
  i32* next = next_of(a, sel);
  const Csr c = a.csr.pick(v.csel);
  mark_prev(a, sel, r, v.nprev, (i64)blockIdx.x * PKT_WAVE + threadIdx.x, (i64)gridDim.x * PKT_WAVE);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->round_done = 1;
  if (threadIdx.x == 0) ba.n = 0;
  __syncthreads();
  WaveAppend app{&ba, next, &ctl->nnext};
  if (l > 0) {  // level 0: frontier edges lie in no triangle
    for (i64 i = blockIdx.x; i < nc; i += gridDim.x) {
      const i32 e1 = curr[i];
      wave_edge_hash(c, rows_of(c, a.el[e1]), e1, l, r, a.sw, a.order, a.owner_higher, app, keys, pos);
    }
  }
  ba.flush(next, &ctl->nnext);
}

// One block after a level scan or a round: ends the round the previous launch
// ran (Ctl::round_done), goes on alone while the work stays small, then picks
// the launch of the frontier left, if any (only when none is picked yet).
// With publish set, writes the loop state to the host-mapped slots Ctl::snap
// under number seq (every path, also when there was nothing to do).  The slots'
// address sits in device memory rather than in the arguments: a kernel whose
// arguments point at host memory gets a system-scope release at its end.
__global__ __launch_bounds__(DECIDE_THREADS) void k_decide(PeelArgs a, i64 seq, int publish) {
  Ctl* ctl = a.ctl;
  __shared__ AloneLds<DECIDE_THREADS> s;
  load_view(ctl, &s.v);  // block-uniform copy: thread 0 rewrites round_done below
  bool go = !s.v.done && (s.v.round_done || s.v.choice == CHOICE_NONE);
  if (go && s.v.round_done) {
    if (threadIdx.x == 0) {
      const i32 nn = ctl->nnext;
      ctl_after_sublevel(ctl, s.v.ncurr, nn, s.v.sel);
      ctl->round_done = 0;
      ctl->choice = CHOICE_NONE;
      s.v.ncurr = nn;  // the view's fields leave() reads
      s.v.choice = CHOICE_NONE;
    }
    __syncthreads();
  }
  if (go) leave<DECIDE_THREADS>(a, s);
  if (publish) {
    __syncthreads();
    if (threadIdx.x == 0) publish_snap(a, ctl, ctl->snap, seq);
  }
}


// k_decide for runs that need no continuation, no features and no cost model
// (heuristic or forced launch choices, no trace): the same round end and choice,
// made by one lane of one wave, with no LDS.
__global__ __launch_bounds__(PKT_WAVE) void k_decide_lite(PeelArgs a, i64 seq, int publish) {
  if (threadIdx.x != 0) return;
  Ctl* ctl = a.ctl;
  const i32 rd = ctl->round_done;
  if (!ctl->done && (rd || ctl->choice == CHOICE_NONE)) {
    if (rd) {
      ctl_after_sublevel(ctl, ctl->ncurr, ctl->nnext, ctl->sel);
      ctl->round_done = 0;
      ctl->choice = CHOICE_NONE;
    }
    const i32 nc = ctl->ncurr;
    if (nc > 0) {
      const int policy = ctl->policy;
      int c = heuristic_choice(policy, nc);
      if (policy == TRUSS_VARIANT_FIXED) {
        const int f = ctl->force_choice;
        if (f >= 0 && f < TRUSS_NUM_CHOICES && (!is_fused(f) || nc <= SMALL_FRONTIER)) c = f;
      }
      ctl->choice = c;
      ctl->chosen[c] += 1;
      for (int k = 0; k < 3; ++k) ctl->mcnt[k] = 0;
      ctl->variant = (policy == TRUSS_VARIANT_MERGE || c == TRUSS_CHOICE_WIDE_GALLOP) ? TRUSS_VARIANT_MERGE
                                                                                       : TRUSS_VARIANT_BSEARCH;
      ctl->feat[0] = log2f(1.f + (float)nc);
      for (int i = 1; i < 8; ++i) ctl->feat[i] = 0.f;
    }
  }
  if (publish) publish_snap(a, ctl, ctl->snap, seq);
}

// ---------------------------------------------------------------- host side

namespace pkt {

namespace {

inline int grid_for(i64 count, int cap) {
  i64 g = (count + PKT_BLOCK - 1) / PKT_BLOCK;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

struct Timer {
  hipEvent_t ev[8];
  int k = 0;
  bool on = false;
  hipStream_t s;
  void init(bool enable, hipStream_t st) {
    on = enable;
    s = st;
    if (on)
      for (int i = 0; i < 8; ++i) (void)hipEventCreateWithFlags(&ev[i], hipEventDisableSystemFence);
  }
  void mark() {
    if (on && k < 8) (void)hipEventRecord(ev[k++], s);
  }
  float ms(int a, int b) {
    float t = 0.f;
    if (on && b < k) (void)hipEventElapsedTime(&t, ev[a], ev[b]);
    return t;
  }
  ~Timer() {
    if (on)
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(ev[i]);
  }
};

thread_local Ctl* h_ctl_pinned = nullptr;

truss_status read_ctl(const Work& w, Ctl* out, hipStream_t s) {
  if (w.no_alloc) {  // pageable destination: nothing allocated
    PKT_HIP(hipMemcpyAsync(out, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    return TRUSS_OK;
  }
  if (!h_ctl_pinned) PKT_HIP(hipHostMalloc((void**)&h_ctl_pinned, sizeof(Ctl), hipHostMallocDefault));
  PKT_HIP(hipMemcpyAsync(h_ctl_pinned, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  *out = *h_ctl_pinned;
  return TRUSS_OK;
}

// Device time of every launch of the wide round kernel (event pairs).
// Timing events stay with the calling thread for its later runs, one pool per
// device: creating and destroying two events per timed launch costs far more host
// time than recording them.
#define CLOCK_DEVICES 16
thread_local std::vector<hipEvent_t> clock_events[CLOCK_DEVICES];

struct KernelClock {
  std::vector<hipEvent_t>* ev = nullptr;
  size_t used = 0;
  hipError_t mark(hipStream_t s) {
    if (!ev) {
      int d = 0;
      const hipError_t r = hipGetDevice(&d);
      if (r != hipSuccess) return r;
      if (d < 0 || d >= CLOCK_DEVICES) return hipErrorInvalidDevice;
      ev = &clock_events[d];
    }
    if (used == ev->size()) {
      hipEvent_t e;
      // timing only: no system-scope fence (a cache writeback) at every record
      const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
      if (r != hipSuccess) return r;
      ev->push_back(e);
    }
    return hipEventRecord((*ev)[used++], s);
  }
  float total_ms() {
    float t = 0.f;
    for (size_t i = 0; i + 1 < used; i += 2) {
      float x = 0.f;
      if (hipEventElapsedTime(&x, (*ev)[i], (*ev)[i + 1]) == hipSuccess) t += x;
    }
    return t;
  }
};

}  // namespace

#ifndef PIPE_ALONE
#define PIPE_ALONE 0  // 1: the continuation with the pipelined loop too (tuning builds)
#endif

// The round's decision: the one-lane kernel when the run needs nothing more.
static inline hipError_t launch_decide(const PeelArgs& a, i64 seq, int publish, hipStream_t s) {
  if (a.lite)
    hipLaunchKernelGGL(k_decide_lite, dim3(1), dim3(PKT_WAVE), 0, s, a, seq, publish);
  else
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(DECIDE_THREADS), 0, s, a, seq, publish);
  return hipGetLastError();
}

// Cooperative launch of the multi-round kernel: every block resident at once, as its
// grid barrier needs.
static truss_status launch_multi(PeelArgs a, hipStream_t s) {
  void* args[] = {&a};
  PKT_HIP(hipLaunchCooperativeKernel((const void*)k_psl_multi, dim3(MULTI_BLOCKS), dim3(SMALL_THREADS), args, 0, s));
  return TRUSS_OK;
}

PeelArgs peel_args(const Work& w, const truss_options& opt) {
  PeelArgs a;
  a.ctl = w.ctl;
  for (int k = 0; k < 3; ++k) a.F[k] = w.F[k];
  a.A0 = w.A[0];
  a.A1 = w.A[1];
  a.el = w.el;
  a.csr = csr_set(w);
  a.sw = w.sw;
  a.order = opt.peel_round;
  a.m = w.m;
  // The single-block continuation saves host round trips; with launch sequences
  // guessed ahead (pipelined loop) there are none to save and the full grid is
  // faster, so it is off there.
  const bool cont = PIPE_ALONE || opt.device_loop != 3 || opt.trace != nullptr;
  a.alone_frontier = cont ? ALONE_FRONTIER : 0;
  a.alone_items = cont ? ALONE_ITEMS : 0;
  a.alone_alive = cont ? ALONE_ALIVE : 0;
  a.owner_higher = opt.owner_rule == 1;
  a.single_round = opt.single_round != 0;
  a.mlp = opt.mlp_weights;
  a.want_features = opt.trace != nullptr ? 2 : (opt.variant == TRUSS_VARIANT_LEARNED ? 1 : 0);
  // consecutive fused rounds in one cooperative launch (truss_options::multi_round), for
  // the host-driven and pipelined loops (the device-driven steps and captured graphs
  // keep one launch per round; tracing and single_round time every round on its own)
  a.multi = opt.multi_round != 0 && !opt.single_round && opt.trace == nullptr &&
            (opt.device_loop == 0 || opt.device_loop == 3);
  a.lite = a.alone_frontier == 0 && a.alone_items == 0 && a.alone_alive == 0 && a.want_features == 0 &&
           opt.variant != TRUSS_VARIANT_LEARNED;
  return a;
}

// Grid of a level scan over nalive entries: one block per tile, at most SCAN_BLOCKS.
// Scratch for the level scan's tile classification: the working-CSR flag array,
// when it holds one word per thread of every tile of the longest alive list.
inline u32* scan_bits(const Work& w) {
  const i64 tiles = (w.m + (i64)PKT_BLOCK * SCAN_ITEMS - 1) / ((i64)PKT_BLOCK * SCAN_ITEMS);
  return tiles * PKT_BLOCK * (i64)sizeof(u32) <= w.two_m ? (u32*)w.flag : nullptr;
}

inline int scan_grid(i64 nalive) {
  const i64 tiles = (nalive + (i64)PKT_BLOCK * SCAN_ITEMS - 1) / ((i64)PKT_BLOCK * SCAN_ITEMS);
  return (int)(tiles < 1 ? 1 : (tiles > SCAN_BLOCKS ? SCAN_BLOCKS : tiles));
}

// Host-driven loop: the launch sequence for the current loop state (read into
// hc): a level scan, or the round of the current frontier as its launch choice
// says.
static truss_status launch_round(const Work& w, const PeelArgs& a, const Ctl& hc, hipStream_t s, int* kind,
                                 KernelClock* prof) {
  if (hc.ncurr == 0) {
    *kind = 0;
    const int G = scan_grid(hc.nalive);
    hipLaunchKernelGGL(k_scan_count, dim3(G), dim3(PKT_BLOCK), 0, s, a, w.partial, w.bmin, scan_bits(w));
    hipLaunchKernelGGL(k_scan_write, dim3(G), dim3(PKT_BLOCK), 0, s, a, (const i64*)w.partial,
                       (const u32*)scan_bits(w));
    PKT_HIP(launch_decide(a, 0, 0, s));
  } else if (hc.choice == CHOICE_NONE) {
    *kind = 0;
    PKT_HIP(launch_decide(a, 0, 0, s));
  } else if (hc.choice == TRUSS_CHOICE_FUSED || hc.choice == TRUSS_CHOICE_FUSED_NARROW) {
    *kind = 1;
    if (a.multi && hc.choice == TRUSS_CHOICE_FUSED) {
      truss_status st = launch_multi(a, s);
      if (st) return st;
    } else {
      const int blocks = hc.choice == TRUSS_CHOICE_FUSED ? FUSED_BLOCKS : FUSED_NARROW_BLOCKS;
      hipLaunchKernelGGL(k_psl_small, dim3(blocks), dim3(SMALL_THREADS), 0, s, a);
    }
    PKT_HIP(launch_decide(a, 0, 0, s));
  } else if (hc.choice == TRUSS_CHOICE_WAVE) {
    *kind = 3;
    hipLaunchKernelGGL(k_psl_wave, dim3(WIDE_BLOCKS), dim3(WIDE_THREADS), 0, s, a);
    PKT_HIP(launch_decide(a, 0, 0, s));
  } else if (hc.choice == TRUSS_CHOICE_HASH) {
    *kind = 4;
    hipLaunchKernelGGL(k_psl_hash, dim3(HASH_BLOCKS), dim3(PKT_WAVE), 0, s, a);
    PKT_HIP(launch_decide(a, 0, 0, s));
  } else {
    *kind = 2;
    // level 0: frontier edges lie in no triangle, nothing to intersect or scan
    if (hc.level > 0) PKT_HIP((scan_launch<WideLen, true>(WideLen{a}, w.partial, w.X, &w.ctl->scan_arrive, s)));
    const int blocks = hc.choice == TRUSS_CHOICE_WIDE_NARROW ? WIDE_NARROW_BLOCKS : WIDE_BLOCKS;
    const bool timed = prof && hc.level > 0;
    if (timed) PKT_HIP(prof->mark(s));
    hipLaunchKernelGGL(k_psl_bsearch, dim3(blocks), dim3(WIDE_THREADS), 0, s, a, (const i64*)w.X);
    if (timed) PKT_HIP(prof->mark(s));
    PKT_HIP(launch_decide(a, 0, 0, s));
  }
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

// Device-driven loop: one step is every launch any loop state can need, each
// gated on the control block, so a step advances the loop by a level scan
// and/or a round (more when a last block goes on alone) without the host
// reading anything.  Launches whose gate is closed return at once.  The first
// k_decide ends the previous step's wide round.
static truss_status enqueue_step(const Work& w, const PeelArgs& a, int G, hipStream_t s, KernelClock* prof) {
  PKT_HIP(launch_decide(a, 0, 0, s));
  hipLaunchKernelGGL(k_scan_count, dim3(G), dim3(PKT_BLOCK), 0, s, a, w.partial, w.bmin, scan_bits(w));
  hipLaunchKernelGGL(k_scan_write, dim3(G), dim3(PKT_BLOCK), 0, s, a, (const i64*)w.partial,
                       (const u32*)scan_bits(w));
  PKT_HIP(launch_decide(a, 0, 0, s));
  hipLaunchKernelGGL(k_psl_small, dim3(FUSED_BLOCKS), dim3(SMALL_THREADS), 0, s, a);
  PKT_HIP(launch_decide(a, 0, 0, s));
  PKT_HIP((scan_launch<WideLen, true>(WideLen{a}, w.partial, w.X, &w.ctl->scan_arrive, s)));
  if (prof) PKT_HIP(prof->mark(s));
  hipLaunchKernelGGL(k_psl_bsearch, dim3(WIDE_BLOCKS), dim3(WIDE_THREADS), 0, s, a, (const i64*)w.X);
  if (prof) PKT_HIP(prof->mark(s));
  hipLaunchKernelGGL(k_psl_wave, dim3(WIDE_BLOCKS), dim3(WIDE_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_psl_hash, dim3(HASH_BLOCKS), dim3(PKT_WAVE), 0, s, a);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

// ---- pipelined host loop
// The host keeps a few launch sequences in flight beyond the last loop state it
// saw, guessed from that state.  Each sequence ends in k_decide, which
// publishes the loop state to host-mapped memory; the host polls for it instead
// of synchronizing the stream.  A wrong guess costs only its launches: every
// kernel gates itself on the control block, and the data a kernel reads (the
// work prefix of a wide round, the chunk offsets of a level scan) comes from the
// launch just before it in the same sequence, under the same loop state.

enum SeqKind { SEQ_SCAN = 0, SEQ_DECIDE = 1, SEQ_FUSED = 2, SEQ_WIDE = 3, SEQ_WAVE = 4, SEQ_HASH = 5 };

#define PIPE_DEPTH 2  // sequences in flight beyond the last state seen (default; measured best)
#define PIPE_MAX 6
static_assert(PIPE_MAX < LOOP_SNAP_SLOTS, "a slot must outlive the sequences in flight after it");

inline int seq_kind(i32 ncurr, i32 choice) {
  if (ncurr == 0) return SEQ_SCAN;
  if (choice == CHOICE_NONE) return SEQ_DECIDE;
  if (choice == TRUSS_CHOICE_FUSED || choice == TRUSS_CHOICE_FUSED_NARROW) return SEQ_FUSED;
  if (choice == TRUSS_CHOICE_WAVE) return SEQ_WAVE;
  if (choice == TRUSS_CHOICE_HASH) return SEQ_HASH;
  return SEQ_WIDE;
}

// One sequence; the grids follow `choice` (its kind's full grid when it is not
// of that kind) and the level-scan grid `nalive`.  The work scan of a wide round
// is always launched (it gates itself on the level), so the round never reads a
// stale prefix whatever state it meets.
static truss_status enqueue_seq(const Work& w, const PeelArgs& a, int kind, int choice, i32 nalive, hipStream_t s,
                                KernelClock* prof, i64 seq) {
  if (kind == SEQ_SCAN) {
    const int G = scan_grid(nalive);
    hipLaunchKernelGGL(k_scan_count, dim3(G), dim3(PKT_BLOCK), 0, s, a, w.partial, w.bmin, scan_bits(w));
    hipLaunchKernelGGL(k_scan_write, dim3(G), dim3(PKT_BLOCK), 0, s, a, (const i64*)w.partial,
                       (const u32*)scan_bits(w));
  } else if (kind == SEQ_FUSED) {
    if (a.multi && choice == TRUSS_CHOICE_FUSED) {
      truss_status st = launch_multi(a, s);
      if (st) return st;
    } else {
      const int blocks = choice == TRUSS_CHOICE_FUSED_NARROW ? FUSED_NARROW_BLOCKS : FUSED_BLOCKS;
      hipLaunchKernelGGL(k_psl_small, dim3(blocks), dim3(SMALL_THREADS), 0, s, a);
    }
  } else if (kind == SEQ_WAVE) {
    hipLaunchKernelGGL(k_psl_wave, dim3(WIDE_BLOCKS), dim3(WIDE_THREADS), 0, s, a);
  } else if (kind == SEQ_HASH) {
    hipLaunchKernelGGL(k_psl_hash, dim3(HASH_BLOCKS), dim3(PKT_WAVE), 0, s, a);
  } else if (kind == SEQ_WIDE) {
    PKT_HIP((scan_launch<WideLen, true>(WideLen{a}, w.partial, w.X, &w.ctl->scan_arrive, s)));
    const int blocks = choice == TRUSS_CHOICE_WIDE_NARROW ? WIDE_NARROW_BLOCKS : WIDE_BLOCKS;
    if (prof) PKT_HIP(prof->mark(s));
    hipLaunchKernelGGL(k_psl_bsearch, dim3(blocks), dim3(WIDE_THREADS), 0, s, a, (const i64*)w.X);
    if (prof) PKT_HIP(prof->mark(s));
  }
  PKT_HIP(launch_decide(a, seq, 1, s));
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

thread_local LoopSnap* h_snap = nullptr;  // host-mapped, coherent
thread_local LoopSnap* d_snap = nullptr;  // its device address
thread_local i64 snap_seq = 0;            // sequence numbers, never reused in a thread

truss_status snap_buffers() {
  if (h_snap) return TRUSS_OK;
  PKT_HIP(hipHostMalloc((void**)&h_snap, sizeof(LoopSnap) * LOOP_SNAP_SLOTS,
                        hipHostMallocMapped | hipHostMallocCoherent));
  memset(h_snap, 0xff, sizeof(LoopSnap) * LOOP_SNAP_SLOTS);
  PKT_HIP(hipHostGetDevicePointer((void**)&d_snap, h_snap, 0));
  return TRUSS_OK;
}

// Waits for the state published by sequence k.  Polls the slot; checks now and
// then whether the stream has drained without it (an error, not a hang).
truss_status wait_snap(i64 k, hipStream_t s, LoopState* out) {
  LoopSnap* slot = h_snap + (k & (LOOP_SNAP_SLOTS - 1));
  const u64 tag = (u64)k & SNAP_TAG_MASK;
  auto t_check = std::chrono::steady_clock::now();
  for (;;) {
    const u64 w0 = __atomic_load_n(&slot->w0, __ATOMIC_ACQUIRE);
    const u64 w1 = __atomic_load_n(&slot->w1, __ATOMIC_ACQUIRE);
    if ((w0 & SNAP_TAG_MASK) == tag && (w1 & SNAP_TAG_MASK) == tag) {
      out->ncurr = (i32)((w0 >> 24) & 0x7FFFFFFFull);
      out->choice = (i32)((w0 >> 55) & 0xFull) - 1;
      out->done = (i32)((w0 >> 59) & 1ull);
      out->compact = (i32)((w0 >> 60) & 1ull);
      out->nalive = (i32)((w1 >> 24) & 0x7FFFFFFFull);
      return TRUSS_OK;
    }
    const auto now = std::chrono::steady_clock::now();
    if (now - t_check > std::chrono::microseconds(200)) {
      t_check = now;
      const hipError_t q = hipStreamQuery(s);
      if (q == hipSuccess) {
        const u64 v0 = __atomic_load_n(&slot->w0, __ATOMIC_ACQUIRE), v1 = __atomic_load_n(&slot->w1, __ATOMIC_ACQUIRE);
        if ((v0 & SNAP_TAG_MASK) == tag && (v1 & SNAP_TAG_MASK) == tag) continue;
        set_error("loop state %lld was not published", (long long)k);
        return TRUSS_E_INTERNAL;
      }
      if (q != hipErrorNotReady) return hip_fail(q, "hipStreamQuery", __FILE__, __LINE__);
    }
  }
}

inline LoopState state_of(const Ctl& c, i64 m) {
  LoopState x;
  x.ncurr = c.ncurr;
  x.choice = c.choice;
  x.done = c.done;
  x.nalive = c.nalive;
  x.compact = needs_compact(m - c.processed, c.csr_edges);
  return x;
}

#define GRAPH_STEPS 8  // steps per captured graph

// GRAPH_STEPS steps captured once into a hipGraph and replayed; recaptured when
// the level-scan grid it was built with no longer fits the alive list.
struct StepGraph {
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  int G = 0;
  truss_status ensure(const Work& w, const PeelArgs& a, int want) {
    if (exec && want <= G && G <= 4 * want) return TRUSS_OK;
    release();
    PKT_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    PKT_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    truss_status st = TRUSS_OK;
    for (int k = 0; k < GRAPH_STEPS && st == TRUSS_OK; ++k) st = enqueue_step(w, a, want, cap, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    PKT_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    PKT_HIP(ei);
    G = want;
    return TRUSS_OK;
  }
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cap) (void)hipStreamDestroy(cap);
    exec = nullptr;
    cap = nullptr;
    G = 0;
  }
  ~StepGraph() { release(); }
};

truss_status run_single(const Work& w, const truss_options& opt, truss_stats* stats, i32* trussness,
                        hipStream_t s, bool support_only) {
  Timer tm;
  tm.init(stats != nullptr && !w.no_alloc, s);  // phase times need events
  tm.mark();  // 0
  Ctl init;
  memset(&init, 0, sizeof(init));
  init.min_above = INT_MAX;
  init.nalive = (i32)w.m;
  init.csr_edges = (i32)w.m;
  init.policy = opt.variant;
  init.force_choice = opt.force_choice;
  init.variant = opt.variant == TRUSS_VARIANT_MERGE ? TRUSS_VARIANT_MERGE : TRUSS_VARIANT_BSEARCH;
  init.choice = CHOICE_NONE;
  if (opt.device_loop == 3 && !opt.trace) {
    truss_status sb = snap_buffers();
    if (sb) return sb;
    init.snap = d_snap;
  }
  PKT_HIP(hipMemcpyAsync(w.ctl, &init, sizeof(Ctl), hipMemcpyHostToDevice, s));
  if (opt.validate) {
    truss_status st = validate_input(w, s);
    if (st) return st;
  }
  tm.mark();  // 1
  if (w.m == 0) {
    if (stats) memset(stats, 0, sizeof(*stats));
    PKT_HIP(hipStreamSynchronize(s));
    return TRUSS_OK;
  }
  truss_status st = build_edges(w, s);
  if (st) return st;
  tm.mark();  // 2
  st = compute_support(w, s);
  if (st) return st;
  tm.mark();  // 3
  if (support_only) {
    st = write_support(w, trussness, s);
    if (st) return st;
    PKT_HIP(hipStreamSynchronize(s));
    return TRUSS_OK;
  }
  st = init_peel(w, s);
  if (st) return st;
  const PeelArgs a = peel_args(w, opt);
  truss_trace* trace = opt.trace;
  hipEvent_t tev[2];
  if (trace) {
    PKT_HIP(hipEventCreateWithFlags(&tev[0], hipEventDisableSystemFence));
    PKT_HIP(hipEventCreateWithFlags(&tev[1], hipEventDisableSystemFence));
  }
  KernelClock clock;
  Ctl hc;
  st = read_ctl(w, &hc, s);
  if (st) return st;
  i64 guard = 0;
  const i64 guard_max = 4 * w.m + 4096;  // bound on launch sequences / steps
  // Working-CSR rebuild when few of its edges are left (needs_compact).  Valid between
  // any two rounds: rows lose only processed edges, which every round skips.
  auto maybe_compact = [&]() -> truss_status {
    if (!opt.compact || !needs_compact(w.m - hc.processed, hc.csr_edges)) return TRUSS_OK;
    truss_status r = compact(w, s);
    if (r) return r;
    return read_ctl(w, &hc, s);
  };
  const int mode = trace ? 0 : opt.device_loop;  // a trace needs one sync per launch sequence
  if (mode == 3) {
    st = snap_buffers();
    if (st) return st;
    KernelClock* prof = opt.profile ? &clock : nullptr;
    const int depth = opt.steps_per_sync > 0 ? (opt.steps_per_sync < PIPE_MAX ? opt.steps_per_sync : PIPE_MAX)
                                             : PIPE_DEPTH;
    struct Flight {
      i64 seq;
      int kind;
    };
    Flight fl[PIPE_MAX];
    int nfl = 0;
    LoopState cur = state_of(hc, w.m);
    int after_scan = SEQ_WIDE;  // kind of the round that followed the last level scan
    // after a multi-round launch the level is usually done: a level scan follows
    auto guess_after = [&](int kind) {
      if (kind == SEQ_SCAN) return after_scan;
      if (kind == SEQ_DECIDE) return (int)SEQ_WIDE;
      if (kind == SEQ_FUSED && a.multi) return (int)SEQ_SCAN;
      return kind;
    };
    // Tops the pipeline up to `depth` sequences.  The sequences in flight are
    // replayed against the last state seen: one of the state's kind does its
    // round (what follows is guessed: the same kind again, or after a level scan
    // the kind that followed the last one); any other does nothing.  A sequence
    // for a state known exactly gets that state's grids.
    auto fill = [&]() -> truss_status {
      int ks = seq_kind(cur.ncurr, cur.choice);
      bool known = true;
      for (int j = 0; j < nfl; ++j)
        if (fl[j].kind == ks) {
          ks = guess_after(ks);
          known = false;
        }
      while (nfl < depth) {
        const i64 q = ++snap_seq;
        const int choice = known ? cur.choice
                                 : (ks == SEQ_FUSED  ? TRUSS_CHOICE_FUSED
                                    : ks == SEQ_WAVE ? TRUSS_CHOICE_WAVE
                                    : ks == SEQ_HASH ? TRUSS_CHOICE_HASH
                                                     : TRUSS_CHOICE_WIDE);
        truss_status r = enqueue_seq(w, a, ks, choice, cur.nalive, s, prof, q);
        if (r) return r;
        fl[nfl++] = Flight{q, ks};
        ks = guess_after(ks);
        known = false;
      }
      return TRUSS_OK;
    };
    st = fill();
    if (st) return st;
    for (;;) {
      const Flight f = fl[0];
      for (int i = 1; i < nfl; ++i) fl[i - 1] = fl[i];
      --nfl;
      const LoopState prev = cur;
      st = wait_snap(f.seq, s, &cur);
      if (st) return st;
      if (cur.done) break;
      if (++guard > guard_max) {
        set_error("level / sub-level count exceeded its bound");
        return TRUSS_E_INTERNAL;
      }
      if (f.kind == SEQ_SCAN && seq_kind(prev.ncurr, prev.choice) == SEQ_SCAN) {
        const int k = seq_kind(cur.ncurr, cur.choice);
        if (k == SEQ_FUSED || k == SEQ_WIDE || k == SEQ_WAVE || k == SEQ_HASH) after_scan = k;
      }
      if (opt.compact && cur.compact) {
        PKT_HIP(hipStreamSynchronize(s));  // lets the sequences in flight finish
        nfl = 0;
        st = read_ctl(w, &hc, s);
        if (st) return st;
        st = maybe_compact();
        if (st) return st;
        cur = state_of(hc, w.m);
        if (cur.done) break;
      }
      st = fill();
      if (st) return st;
    }
    PKT_HIP(hipStreamSynchronize(s));
    st = read_ctl(w, &hc, s);
    if (st) return st;
  } else if (mode == 0) {
    while (!hc.done) {
      if (++guard > guard_max) {
        set_error("level / sub-level count exceeded its bound");
        return TRUSS_E_INTERNAL;
      }
      st = maybe_compact();
      if (st) return st;
      const Ctl before = hc;
      int kind = 0;
      if (trace) PKT_HIP(hipEventRecord(tev[0], s));
      st = launch_round(w, a, hc, s, &kind, opt.profile ? &clock : nullptr);
      if (st) return st;
      if (trace) PKT_HIP(hipEventRecord(tev[1], s));
      st = read_ctl(w, &hc, s);
      if (st) return st;
      if (trace && trace->count < trace->capacity) {
        truss_trace_record& r = trace->records[trace->count++];
        memset(&r, 0, sizeof(r));
        r.level = before.level;
        r.kind = kind;
        r.choice = kind == 0 ? -1 : before.choice;
        r.rounds = hc.sublevels - before.sublevels;
        r.round_index = before.sublevels;
        r.frontier = before.ncurr;
        r.items = -1;
        if (kind == 2 && before.level > 0)
          PKT_HIP(hipMemcpy(&r.items, w.X + before.ncurr, sizeof(i64), hipMemcpyDeviceToHost));
        for (int i = 0; i < 8; ++i) r.features[i] = before.feat[i];
        PKT_HIP(hipEventElapsedTime(&r.ms, tev[0], tev[1]));
      }
    }
  } else {
    // Device-driven: batches of steps between host checks (GRAPH_STEPS, doubling
    // up to 8 * GRAPH_STEPS, or steps_per_sync); with mode 2 the steps replay a
    // captured hipGraph (not with profile, whose events sit between launches).
    StepGraph graph;
    const bool use_graph = mode == 2 && !opt.profile;
    int batch = 1;
    while (!hc.done) {
      st = maybe_compact();
      if (st) return st;
      const int G = scan_grid(hc.nalive);
      const int graphs = opt.steps_per_sync > 0 ? (opt.steps_per_sync + GRAPH_STEPS - 1) / GRAPH_STEPS : batch;
      const int steps = opt.steps_per_sync > 0 ? opt.steps_per_sync : batch * GRAPH_STEPS;
      guard += use_graph ? (i64)graphs * GRAPH_STEPS : steps;
      if (guard > guard_max) {
        set_error("level / sub-level count exceeded its bound");
        return TRUSS_E_INTERNAL;
      }
      if (use_graph) {
        st = graph.ensure(w, a, G);
        if (st) return st;
        for (int k = 0; k < graphs; ++k) PKT_HIP(hipGraphLaunch(graph.exec, s));
      } else {
        for (int k = 0; k < steps; ++k) {
          st = enqueue_step(w, a, G, s, opt.profile ? &clock : nullptr);
          if (st) return st;
        }
      }
      st = read_ctl(w, &hc, s);
      if (st) return st;
      if (batch < 8) batch *= 2;
    }
  }
  if (trace) {
    (void)hipEventDestroy(tev[0]);
    (void)hipEventDestroy(tev[1]);
  }
  tm.mark();  // 4
  st = write_output(w, trussness, s);
  if (st) return st;
  tm.mark();  // 5
  st = read_ctl(w, &hc, s);
  if (st) return st;
  if (hc.bar_timeout) {
    set_error("a grid barrier of the multi-round launch timed out");
    return TRUSS_E_INTERNAL;
  }
  if (hc.processed != w.m) {
    set_error("peeling ended with %lld of %lld edges processed", (long long)hc.processed, (long long)w.m);
    return TRUSS_E_INTERNAL;
  }
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->m = w.m;
    stats->levels = hc.levels;
    stats->sublevels = hc.sublevels;
    stats->triangles = hc.tri3 / 3;
    stats->t_max = hc.tmax_s;
    stats->compactions = hc.compactions;
    stats->ms_validate = tm.ms(0, 1);
    stats->ms_build = tm.ms(1, 2);
    stats->ms_support = tm.ms(2, 3);
    stats->ms_peel = tm.ms(3, 4);
    stats->ms_total = tm.ms(0, 5);
    for (int k = 0; k < TRUSS_NUM_CHOICES; ++k) stats->choice_count[k] = hc.chosen[k];
    stats->wide_launches = hc.wide_launches;
    stats->wide_items = hc.wide_items;
    stats->wide_frontier = hc.wide_frontier;
    stats->wide_ms = opt.profile ? clock.total_ms() : 0.f;
    stats->wide_timed = opt.profile ? (i32)(clock.used / 2) : 0;
  }
  return TRUSS_OK;
}

}  // namespace pkt
