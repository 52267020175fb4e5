// Sub-level processing device routines shared by the level loop (peel.hip) and
// the persistent batched kernel (persist.hip): the decrement rule of a triangle
// (Kabir and Madduri, arXiv:1707.02000, Algorithm 5 and the text on concurrent
// triangle processing that follows it) and the wave-level intersection of a
// frontier edge's two rows.
#pragma once
#include <limits.h>

#include "truss.h"

// Decrement rule for edge x of a triangle whose other non-frontier-edge is y,
// seen from frontier edge e1 in round r: x loses one unit if its support is
// above l and e1 owns the triangle (y is not in the frontier, or e1 has the
// lower id -- the higher id with owner_higher).  The atomic's old value decides:
// l + 1 means x now sits at l and joins the next frontier (tag of round r + 1);
// <= l means the decrement overshot (another thread got there first) and is
// undone.  The caller's earlier read of x's word may be stale: while the support
// is > l every older value is > l too, and once it is <= l it stays <= l for the
// level, so a stale read can only cause a decrement that is then undone.  Whether
// y is current comes from the same earlier read of y's word: during a round a
// state only changes between values that are not the round's tag (alive -> next,
// previous round -> processed), so that read answers for the whole round.  The
// next-frontier tag written here reads as "not current" and "not processed" to
// every other thread.
//
// Applied to both other edges es, eo of one triangle (words ws, wo as read by the
// caller): (x, y) = (es, eo) and (eo, es), both atomics issued before either
// result is used, so their round trips overlap.  xa / xb get es / eo if they
// joined the next frontier, else -1.  sw may point to global memory or to LDS.
__device__ __forceinline__ void psl_tri(i32 es, i32 ws, i32 eo, i32 wo, i32 e1, i32 l, i32 r, i32* sw, i32* order,
                                        int owner_higher, i32& xa, i32& xb) {
  const u8 tcur = round_tag(r);
  const bool own_s = sw_st(wo) != tcur || (owner_higher ? (e1 > eo) : (e1 < eo));
  const bool own_o = sw_st(ws) != tcur || (owner_higher ? (e1 > es) : (e1 < es));
  const bool ds = own_s && sw_sup(ws) > l, dd = own_o && sw_sup(wo) > l;
  const i32 as = ds ? sw_sup(atomicSub(&sw[es], SW_ONE)) : 0;
  const i32 ao = dd ? sw_sup(atomicSub(&sw[eo], SW_ONE)) : 0;
  xa = xb = -1;
  if (ds) {
    if (as == l + 1) {
      atomicOr(&sw[es], (i32)round_tag(r + 1));
      if (order) order[es] = r + 1;
      xa = es;
    } else if (as <= l) {
      atomicAdd(&sw[es], SW_ONE);
    }
  }
  if (dd) {
    if (ao == l + 1) {
      atomicOr(&sw[eo], (i32)round_tag(r + 1));
      if (order) order[eo] = r + 1;
      xb = eo;
    } else if (ao <= l) {
      atomicAdd(&sw[eo], SW_ONE);
    }
  }
}

// Shorter and longer working rows of frontier edge e1 = (u, v).
struct Rows {
  i64 sb, slen, lb, le;
};

__device__ __forceinline__ Rows rows_of(const Csr& c, int2 uv) {
  const i64 ub = c.off[uv.x], ue = c.off[uv.x + 1], vb = c.off[uv.y], ve = c.off[uv.y + 1];
  Rows r;
  if (ue - ub <= ve - vb) {
    r.sb = ub; r.slen = ue - ub; r.lb = vb; r.le = ve;
  } else {
    r.sb = vb; r.slen = ve - vb; r.lb = ub; r.le = ue;
  }
  return r;
}

// ---------------------------------------------------------------- one wave per edge

// The longer row is merged when it is at most WAVE_MERGE_RATIO times the
// shorter one (a merge reads both rows once, (a + b) / 64 steps of the wave);
// beyond that every lane binary-searches its shorter-row entry in the part of
// the longer row its chunk can reach ((a / 64) log b probes per lane).
#ifndef WAVE_MERGE_RATIO
#define WAVE_MERGE_RATIO 8
#endif

// Position in [0, 63] of s among the wave's 64 ascending register values lv (one
// per lane): the number of values below s, capped at 63.  s is present iff the
// value at that position equals s.  Lanes may ask for different s.  Called by the
// whole wave (a shuffle reads only lanes that execute it).
__device__ __forceinline__ int wave_rank(i32 lv, i32 s) {
  int pos = 0;
#pragma unroll
  for (int step = PKT_WAVE / 2; step >= 1; step >>= 1) {
    const i32 v = __shfl(lv, pos + step - 1);
    if (v < s) pos += step;
  }
  return pos;
}

// The triangle {e1, es, eo} found by a lane: rule set of the round when neither
// other edge is processed.
__device__ __forceinline__ void wave_triangle(i32 es, i32 eo, i32 e1, i32 l, i32 rd, i32* sw, i32* order,
                                              int owner_higher, i32& x0, i32& x1) {
  const i32 ws = sw[es], wo = sw[eo];
  if (!is_processed(sw_st(ws), rd) && !is_processed(sw_st(wo), rd))
    psl_tri(es, ws, eo, wo, e1, l, rd, sw, order, owner_higher, x0, x1);
}

// Every common entry of the shorter row adj[r.sb, r.sb + r.slen) and the longer
// row adj[r.lb, r.le), found by the calling wave: hit(ok, js, jl) is called by the
// whole wave once per step, with ok set on the lanes that found one (js, jl: its
// slots in the two rows).  Every common entry is reported exactly once.  The rows
// are merged when the longer one is at most WAVE_MERGE_RATIO times the shorter;
// otherwise every lane binary-searches its entry inside the longer-row bracket of
// its 64-entry chunk.  Every argument is wave-uniform.
template <class Hit>
__device__ void wave_intersect(const i32* __restrict__ adj, const Rows& r, Hit& hit) {
  const int lane = lane_id();
  const i64 a = r.slen, b = r.le - r.lb;
  if (a == 0 || b == 0) return;
  if (b <= (i64)WAVE_MERGE_RATIO * a) {
    // merge path in chunks of 64: i, j are the first unresolved entries of the rows
    i64 i = 0, j = 0;
    while (i < a && j < b) {
      const bool sv = i + lane < a;
      const i32 s = sv ? adj[r.sb + i + lane] : INT_MAX;
      const i32 lv = (j + lane < b) ? adj[r.lb + j + lane] : INT_MAX;
      const int pos = wave_rank(lv, s);
      const i32 at = __shfl(lv, pos);  // every lane takes part: a shuffle reads only active lanes
      hit(sv && at == s, r.sb + i + lane, r.lb + j + pos);
      const i32 s_last = __shfl(s, PKT_WAVE - 1), l_last = __shfl(lv, PKT_WAVE - 1);
      if (s_last <= l_last) {  // every entry of this S chunk is resolved; L entries <= s_last are spent
        j += (i64)__popcll(__ballot(lv <= s_last));
        i += PKT_WAVE;
      } else {  // S entries <= l_last are resolved; the whole L chunk is spent
        i += (i64)__popcll(__ballot(sv && s <= l_last));
        j += PKT_WAVE;
      }
    }
  } else {
    // skewed rows: per-lane binary search inside the bracket of the chunk
    for (i64 i = 0; i < a; i += PKT_WAVE) {
      const bool sv = i + lane < a;
      const i32 s = sv ? adj[r.sb + i + lane] : INT_MAX;
      const int last = (int)min((i64)PKT_WAVE, a - i) - 1;
      i64 lo = 0, hi = 0;
      if (lane == 0) lo = lower_bound_dev(adj, r.lb, r.le, s);
      if (lane == last) hi = upper_bound_dev(adj, r.lb, r.le, s);
      lo = __shfl(lo, 0);
      hi = __shfl(hi, last);
      i64 p = hi;
      if (sv) p = lower_bound_dev(adj, lo, hi, s);
      hit(sv && p < hi && adj[p < hi ? p : lo] == s, r.sb + i + lane, p);
    }
  }
}

// Frontier edge e1 (rows r of the working CSR c) processed by the calling wave:
// every w in N(u) ∩ N(v) is found once, and the decrement rule runs on the
// triangle's two other edges.  app.add(x0, x1) receives the edges that reached
// the level; it is called by the whole wave, uniformly.  Every argument is
// wave-uniform.
template <class Append>
struct PeelHit {
  const i32* eid;
  i32 e1, l, rd;
  i32* sw;
  i32* order;
  int owner_higher;
  Append* app;
  __device__ __forceinline__ void operator()(bool ok, i64 js, i64 jl) {
    i32 x0 = -1, x1 = -1;
    if (ok) wave_triangle(eid[js], eid[jl], e1, l, rd, sw, order, owner_higher, x0, x1);
    app->add(x0, x1);
  }
};

template <class Append>
__device__ void wave_edge(const Csr& c, const Rows& r, i32 e1, i32 l, i32 rd, i32* sw, i32* order,
                          int owner_higher, Append& app) {
  PeelHit<Append> h{c.eid, e1, l, rd, sw, order, owner_higher, &app};
  wave_intersect(c.adj, r, h);
}

// LDS hash variant: the longer row (at most WAVE_HASH_CAP entries) goes into an
// open-addressing table in LDS (key = vertex, value = its position in the row;
// WAVE_HASH_SLOTS slots, linear probing, multiplicative hash), then every lane
// probes its shorter-row entries.  Longer rows take wave_intersect.  Called by a
// workgroup of exactly one wave (its barriers are the wave's own), every argument
// uniform; keys / pos are that workgroup's LDS.
#define WAVE_HASH_CAP 256
#define WAVE_HASH_SLOTS (2 * WAVE_HASH_CAP)
__device__ __forceinline__ u32 wave_hash_slot(i32 w) { return ((u32)w * 0x9E3779B1u) >> (32 - 9); }
static_assert(WAVE_HASH_SLOTS == 512, "wave_hash_slot takes the top 9 bits");

template <class Hit>
__device__ void wave_intersect_hash(const i32* __restrict__ adj, const Rows& r, Hit& hit, i32* keys,
                                    unsigned short* pos) {
  const int lane = lane_id();
  const i64 a = r.slen, b = r.le - r.lb;
  if (a == 0 || b == 0) return;
  if (b > WAVE_HASH_CAP) {
    wave_intersect(adj, r, hit);
    return;
  }
  for (int k = lane; k < WAVE_HASH_SLOTS; k += PKT_WAVE) keys[k] = -1;
  __syncthreads();
  for (i32 j = lane; j < (i32)b; j += PKT_WAVE) {
    const i32 w = adj[r.lb + j];
    u32 h = wave_hash_slot(w);
    for (;;) {  // b <= half the slots: a free slot is always found
      const i32 old = atomicCAS(&keys[h], -1, w);
      if (old == -1) {
        pos[h] = (unsigned short)j;
        break;
      }
      h = (h + 1) & (WAVE_HASH_SLOTS - 1);
    }
  }
  __syncthreads();
  for (i64 i = 0; i < a; i += PKT_WAVE) {
    const bool sv = i + lane < a;
    i64 jl = -1;
    if (sv) {
      const i32 s = adj[r.sb + i + lane];
      u32 h = wave_hash_slot(s);
      for (;;) {
        const i32 k = keys[h];
        if (k == s) {
          jl = r.lb + pos[h];
          break;
        }
        if (k == -1) break;
        h = (h + 1) & (WAVE_HASH_SLOTS - 1);
      }
    }
    hit(jl >= 0, r.sb + i + lane, jl);
  }
  __syncthreads();  // the table is the next edge's
}

template <class Append>
__device__ void wave_edge_hash(const Csr& c, const Rows& r, i32 e1, i32 l, i32 rd, i32* sw, i32* order,
                               int owner_higher, Append& app, i32* keys, unsigned short* pos) {
  PeelHit<Append> h{c.eid, e1, l, rd, sw, order, owner_higher, &app};
  wave_intersect_hash(c.adj, r, h, keys, pos);
}

// |N(u) ∩ N(v)| of the rows r, by the calling wave (every lane gets the count).
struct CountHit {
  i32 n = 0;
  __device__ __forceinline__ void operator()(bool ok, i64, i64) { n += ok ? 1 : 0; }
};

__device__ __forceinline__ i32 wave_common(const i32* __restrict__ adj, const Rows& r) {
  CountHit h;
  wave_intersect(adj, r, h);
  return (i32)wave_sum_i64(h.n);
}
