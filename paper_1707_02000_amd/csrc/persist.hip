// Batched decomposition in one persistent launch: every workgroup takes graphs
// from a queue ordered by decreasing edge count (longest-processing-time first)
// and decomposes each one alone -- edge ids, support, the whole level loop of
// the PKT section (Algorithm 4: level scans and sub-level rounds; Algorithm 5 in
// every round) -- with workgroup barriers where the single-graph path has kernel
// boundaries.  Small graphs keep their support words (support and state of every
// edge, the randomly read and atomically updated array) in LDS.  Graphs above
// PB_MAX_EDGES are left to the single-graph path after the launch.
//
// Inside a workgroup the support counts and every round work on chunks of up to
// PB_CH edges: the chunk's rows and the exclusive prefix of its shorter-row
// lengths go to LDS, and every lane takes one entry of a shorter row (an item),
// finds its edge in the prefix and binary-searches the entry in the longer row --
// the rounds' load spreads over the lanes whatever the degrees.
#include <limits.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "psl.h"

#define PB_THREADS 512
#define PB_WAVES (PB_THREADS / PKT_WAVE)
#ifndef PB_LDS_EDGES
#define PB_LDS_EDGES 8192  // support words in LDS for graphs up to this many edges (32 KB)
#endif
#define PB_CH 1024  // edges per chunk of items (rows and work prefix in LDS)
#define PB_MAX_EDGES (1 << 22)  // larger graphs go through the single-graph path
#ifndef PB_MIN_WAVES
#define PB_MIN_WAVES 4  // waves per SIMD the kernel's registers must allow (4: no spills)
#endif
#define PB_WG_PER_CU (PB_MIN_WAVES / 2)  // workgroups per compute unit (8 waves each, 4 SIMDs)

namespace pkt {
truss_status run_single(const Work& w, const truss_options& opt, truss_stats* stats, i32* trussness,
                        hipStream_t s, bool support_only);
truss_status prepare_off64(Work& w, const i32* off32, hipStream_t s);
}  // namespace pkt

using namespace pkt;

namespace {

enum : u32 { PB_ERR_RANGE = 1u, PB_ERR_NOT_SIMPLE = 2u, PB_ERR_NOT_SYMMETRIC = 4u, PB_ERR_INTERNAL = 8u };

struct PbArgs {
  const i64* __restrict__ vo;   // [G+1] offsets entries of each graph
  const i64* __restrict__ ao;   // [G+1] adjacency slots of each graph
  const i32* __restrict__ offs;  // packed local offsets
  const i32* __restrict__ adj;   // packed local ids
  const i32* __restrict__ order;  // the graphs of this launch, largest first
  i32 nq;                         // entries of order
  i32* queue;                     // next entry of order (atomic)
  i32* eb;                        // [total_vtx] first edge id of every row
  i32* eid;                       // [total_adj] edge id of every slot
  int2* el;                       // [total_adj / 2] endpoints of every edge
  i32* sw;                        // [total_adj / 2] support words (graphs above PB_LDS_EDGES)
  i32* fa;                        // [total_adj / 2] frontier buffers
  i32* fb;
  i32* al0;                       // [total_adj / 2] alive lists
  i32* al1;
  i32* out;                       // packed trussness
  u32* err;                       // error bits (PB_ERR_*)
  i32* bad_graph;                 // smallest graph index with an error (atomic min)
  i64* counters;                  // [4] levels, rounds, 3 x triangles, max trussness
  int owner_higher;
};

struct PbShared {
  i64 tmp[PB_WAVES];
  i32 P[PB_CH + 1];                      // exclusive prefix of the chunk's shorter-row lengths
  i32 sb[PB_CH], lb[PB_CH], ll[PB_CH];   // shorter-row start, longer-row start and length
  i32 e1[PB_CH];                         // the chunk's edges
  i32 g, n0, n1, mn, bad;
};

// Rows of the edges list[i] (i < cnt <= PB_CH; list NULL: edges first + i) into LDS,
// with the exclusive prefix of their shorter-row lengths (no items with nowork).
// Returns the chunk's items.  Every thread calls it.
__device__ i32 pb_chunk(const i32* __restrict__ O, const int2* __restrict__ EL, const i32* __restrict__ list,
                        i32 first, i32 cnt, bool nowork, PbShared& sh) {
  constexpr int PER = PB_CH / PB_THREADS;
  i32 w[PER];
  i64 sum = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const i32 i = threadIdx.x * PER + k;
    w[k] = 0;
    if (i < cnt) {
      const i32 e = list ? list[i] : first + i;
      const int2 uv = EL[e];
      const i32 ub = O[uv.x], ue = O[uv.x + 1], vb = O[uv.y], ve = O[uv.y + 1];
      const bool us = ue - ub <= ve - vb;
      sh.e1[i] = e;
      sh.sb[i] = us ? ub : vb;
      sh.lb[i] = us ? vb : ub;
      sh.ll[i] = us ? ve - vb : ue - ub;
      w[k] = nowork ? 0 : (us ? ue - ub : ve - vb);
    }
    sum += w[k];
  }
  i64 tot;
  i64 run = block_excl_scan_i64<PB_THREADS>(sum, sh.tmp, &tot);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const i32 i = threadIdx.x * PER + k;
    if (i < cnt) sh.P[i] = (i32)run;
    run += w[k];
  }
  if (threadIdx.x == 0) sh.P[cnt] = (i32)tot;
  __syncthreads();
  return (i32)tot;
}

// Items g0 and g1 of the chunk, side by side so that their dependent loads overlap
// (a lane has two chains in flight): for each, its edge k (-1 when g >= items), the
// slot js of its shorter-row entry and the slot jl of the same vertex in the longer
// row (-1 if absent).  Both binary searches run in lockstep, one probe of each per
// step; a finished search keeps probing its row's first slot (always inside the
// row: b may have reached the row's end, which can be one past the graph).
__device__ __forceinline__ void pb_item2(const i32* __restrict__ A, const PbShared& sh, i32 cnt, i32 items, i32 g0,
                                         i32 g1, i32& k0, i32& js0, i32& jl0, i32& k1, i32& js1, i32& jl1) {
  const bool v0 = g0 < items, v1 = g1 < items;
  k0 = v0 ? (i32)upper_bound_dev(sh.P, (i32)0, cnt + 1, g0) - 1 : -1;
  k1 = v1 ? (i32)upper_bound_dev(sh.P, (i32)0, cnt + 1, g1) - 1 : -1;
  const i32 q0 = v0 ? k0 : 0, q1 = v1 ? k1 : 0;
  js0 = sh.sb[q0] + (v0 ? g0 - sh.P[q0] : 0);
  js1 = sh.sb[q1] + (v1 ? g1 - sh.P[q1] : 0);
  const i32 w0 = A[js0], w1 = A[js1];
  const i32 r0 = sh.lb[q0], r1 = sh.lb[q1];  // row starts: rows of edges hold >= 1 entry
  i32 b0 = r0, n0 = v0 ? sh.ll[q0] : 0;
  i32 b1 = r1, n1 = v1 ? sh.ll[q1] : 0;
  const i32 e0 = b0 + n0, e1 = b1 + n1;
  while (n0 > 0 || n1 > 0) {  // lower bound: b + n stays the end of the candidates
    const i32 h0 = n0 >> 1, h1 = n1 >> 1;
    const i32 x0 = A[n0 > 0 ? b0 + h0 : r0], x1 = A[n1 > 0 ? b1 + h1 : r1];
    if (n0 > 0) {
      if (x0 < w0) {
        b0 += h0 + 1;
        n0 -= h0 + 1;
      } else {
        n0 = h0;
      }
    }
    if (n1 > 0) {
      if (x1 < w1) {
        b1 += h1 + 1;
        n1 -= h1 + 1;
      } else {
        n1 = h1;
      }
    }
  }
  jl0 = (v0 && b0 < e0 && A[b0] == w0) ? b0 : -1;
  jl1 = (v1 && b1 < e1 && A[b1] == w1) ? b1 : -1;
}

// Appends of one round to the next frontier: per wave, one LDS reservation.
struct PbAppend {
  i32* next;
  i32* counter;  // LDS
  __device__ __forceinline__ void add1(i32 x) {
    const u64 mask = __ballot(x >= 0);
    if (mask == 0) return;
    const int lane = lane_id(), leader = __ffsll((unsigned long long)mask) - 1;
    i32 b = 0;
    if (lane == leader) b = atomicAdd(counter, (i32)__popcll(mask));
    b = __shfl(b, leader);
    if (x >= 0) next[b + (i32)__popcll(mask & ((1ull << lane) - 1ull))] = x;
  }
  __device__ __forceinline__ void add(i32 x0, i32 x1) {
    add1(x0);
    add1(x1);
  }
};

// Ends a checking phase: every thread's flag is in, the graph is dropped if any
// check failed (the error bits and the graph index are recorded).  Uniform.
__device__ __forceinline__ bool phase_failed(PbShared& sh, const PbArgs& p, i32 g, u32 bits) {
  if (bits) atomicOr((u32*)&sh.bad, bits);
  __syncthreads();
  const u32 b = (u32)sh.bad;
  __syncthreads();
  if (b && threadIdx.x == 0) {
    atomicOr(p.err, b);
    atomicMin(p.bad_graph, g);
  }
  return b != 0;
}

// The whole decomposition of graph g by the calling workgroup.
__device__ void pb_graph(const PbArgs& p, i32 g, PbShared& sh, i32* lsw) {
  const int tid = threadIdx.x, wave = tid / PKT_WAVE, lane = lane_id();
  const i64 v0 = p.vo[g], a0 = p.ao[g];
  const i32 n = (i32)(p.vo[g + 1] - v0 - 1);
  const i64 two_m = p.ao[g + 1] - a0;
  const i32 m = (i32)(two_m / 2);
  const i64 e0 = a0 / 2;
  const i32* __restrict__ O = p.offs + v0;
  const i32* __restrict__ A = p.adj + a0;
  i32* EB = p.eb + v0;
  i32* EID = p.eid + a0;
  int2* EL = p.el + e0;
  i32* SW = m <= PB_LDS_EDGES ? lsw : p.sw + e0;
  if (tid == 0) sh.bad = 0;
  __syncthreads();
  if (m == 0) return;

  // ---- rows: offsets in range and in order; upper entries per row
  u32 bits = 0;
  for (i32 u = tid; u < n; u += PB_THREADS) {
    const i32 b = O[u], e = O[u + 1];
    if (b < 0 || e < b || e > two_m || (u == 0 && b != 0) || (u == n - 1 && e != two_m)) {
      bits |= PB_ERR_RANGE;
      continue;
    }
    EB[u] = e - (i32)lower_bound_dev(A, (i64)b, (i64)e, u + 1);
  }
  if (phase_failed(sh, p, g, bits)) return;
  // first edge id of every row: exclusive prefix of the upper counts
  i64 run = 0;
  for (i32 base = 0; base < n; base += PB_THREADS) {
    const i32 u = base + tid;
    const i64 c = u < n ? EB[u] : 0;
    i64 tot;
    const i64 ex = block_excl_scan_i64<PB_THREADS>(c, sh.tmp, &tot);
    if (u < n) EB[u] = (i32)(run + ex);
    run += tot;
  }
  if (run != m) bits |= PB_ERR_NOT_SYMMETRIC;  // a symmetric simple graph has m upper entries
  if (phase_failed(sh, p, g, bits)) return;

  // ---- slots: ids in range, rows strictly increasing, no self-loop; upper slots numbered
  for (i32 u = wave; u < n; u += PB_WAVES) {
    const i32 b = O[u], e = O[u + 1];
    i64 us = 0;
    if (lane == 0) us = lower_bound_dev(A, (i64)b, (i64)e, u + 1);
    us = __shfl(us, 0);
    const i32 base = EB[u];
    for (i32 j = b + lane; j < e; j += PKT_WAVE) {
      const i32 x = A[j];
      if (x < 0 || x >= n) {
        bits |= PB_ERR_RANGE;
        continue;
      }
      if (x == u || (j > b && A[j - 1] >= x)) bits |= PB_ERR_NOT_SIMPLE;
      if (x > u) {
        const i64 id = base + (j - us);
        if (id < 0 || id >= m) {
          bits |= PB_ERR_NOT_SIMPLE;
        } else {
          EID[j] = (i32)id;
          EL[id] = make_int2(u, x);
        }
      }
    }
  }
  if (phase_failed(sh, p, g, bits)) return;
  // lower slots: the id of the mirror slot (an upper slot of the smaller endpoint)
  for (i32 u = wave; u < n; u += PB_WAVES) {
    const i32 b = O[u], e = O[u + 1];
    for (i32 j = b + lane; j < e; j += PKT_WAVE) {
      const i32 x = A[j];
      if (x >= u) continue;
      const i32 xb = O[x], xe = O[x + 1];
      const i32 q = (i32)lower_bound_dev(A, (i64)xb, (i64)xe, u);
      if (q == xe || A[q] != u)
        bits |= PB_ERR_NOT_SYMMETRIC;
      else
        EID[j] = EID[q];
    }
  }
  if (phase_failed(sh, p, g, bits)) return;

  // ---- support: per chunk of edges, one lane per shorter-row entry; the hits of the
  // lanes that share an edge are summed in the wave and added to its word at once
  for (i32 e = tid; e < m; e += PB_THREADS) SW[e] = 0;
  __syncthreads();
  i64 tri3 = 0;
  for (i32 c0 = 0; c0 < m; c0 += PB_CH) {
    const i32 cnt = min(PB_CH, m - c0);
    const i32 items = pb_chunk(O, EL, nullptr, c0, cnt, false, sh);
    for (i32 base = 0; base < items; base += 2 * PB_THREADS) {
      i32 k[2], js[2], jl[2];
      pb_item2(A, sh, cnt, items, base + tid, base + PB_THREADS + tid, k[0], js[0], jl[0], k[1], js[1], jl[1]);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        u64 todo = __ballot(k[h] >= 0);
        const u64 hits = __ballot(jl[h] >= 0);
        while (todo) {  // lanes' edges are non-decreasing: a few segments per wave
          const int lead = __ffsll((unsigned long long)todo) - 1;
          const i32 kl = __shfl(k[h], lead);
          const u64 same = __ballot(k[h] == kl);
          const i32 c = (i32)__popcll(hits & same);
          if (lane == lead && c) {
            atomicAdd(&SW[c0 + kl], c << SW_SHIFT);  // state bits stay ST_ALIVE
            tri3 += c;
          }
          todo &= ~same;
        }
      }
    }
    __syncthreads();  // the chunk's LDS is rewritten by the next one
  }

  // ---- level loop
  i32* AL = p.al0 + e0;
  i32* ALn = p.al1 + e0;
  i32* FA = p.fa + e0;
  i32* FB = p.fb + e0;
  i32 l = 0, r = 0, nal = m, levels = 0, rounds = 0;
  bool first = true;  // the first scan reads every edge, in order
  // every level scan finds a frontier or jumps to a support that has one, and
  // every round retires at least one edge: at most 2m + 2 steps (a watchdog)
  const i64 guard_max = 2 * (i64)m + 2;
  i64 guard = 0;
  for (;;) {
    if (++guard > guard_max) {  // uniform: every thread counts the same steps
      if (tid == 0) {
        atomicOr(p.err, PB_ERR_INTERNAL);
        atomicMin(p.bad_graph, g);
      }
      break;
    }
    // level scan: alive edges at support l form the frontier (tag of round r), the
    // others stay on the alive list
    if (tid == 0) {
      sh.n0 = 0;
      sh.n1 = 0;
      sh.mn = INT_MAX;
    }
    __syncthreads();
    i32 mn = INT_MAX;
    for (i32 base = 0; base < nal; base += PB_THREADS) {
      const i32 k = base + tid;
      i32 e = -1, w = 0;
      if (k < nal) {
        e = first ? k : AL[k];
        w = SW[e];
      }
      const bool alive = e >= 0 && sw_st(w) == ST_ALIVE;
      const bool take = alive && sw_sup(w) == l, keep = alive && !take;
      if (keep) mn = min(mn, sw_sup(w));
      const u64 mt = __ballot(take), mk = __ballot(keep);
      const int leader = 0;
      i32 bt = 0, bk = 0;
      if (lane == leader) {
        if (mt) bt = atomicAdd(&sh.n0, (i32)__popcll(mt));
        if (mk) bk = atomicAdd(&sh.n1, (i32)__popcll(mk));
      }
      bt = __shfl(bt, leader);
      bk = __shfl(bk, leader);
      const u64 below = (1ull << lane) - 1ull;
      if (take) {
        FA[bt + (i32)__popcll(mt & below)] = e;
        SW[e] = sw_make(l, round_tag(r));
      }
      if (keep) ALn[bk + (i32)__popcll(mk & below)] = e;
    }
    mn = wave_min_i32(mn);
    if (lane == 0 && mn != INT_MAX) atomicMin(&sh.mn, mn);
    __syncthreads();
    i32 nf = sh.n0;
    const i32 nk = sh.n1, kmin = sh.mn;
    __syncthreads();
    first = false;
    {
      i32* t = AL;
      AL = ALn;
      ALn = t;
    }
    nal = nk;
    ++levels;
    if (nf == 0) {
      if (nk == 0) break;
      l = kmin;  // no edge at this level: jump to the lowest support left
      continue;
    }
    // rounds of level l until no edge reaches it
    while (nf > 0 && guard <= guard_max) {
      ++guard;
      if (tid == 0) sh.n1 = 0;
      __syncthreads();
      PbAppend app{FB, &sh.n1};
      if (l > 0) {  // level 0: frontier edges lie in no triangle
        for (i32 c0 = 0; c0 < nf; c0 += PB_CH) {
          const i32 cnt = min(PB_CH, nf - c0);
          const i32 items = pb_chunk(O, EL, FA + c0, 0, cnt, false, sh);
          for (i32 base = 0; base < items; base += 2 * PB_THREADS) {
            i32 k[2], js[2], jl[2];
            pb_item2(A, sh, cnt, items, base + tid, base + PB_THREADS + tid, k[0], js[0], jl[0], k[1], js[1],
                     jl[1]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              i32 x0 = -1, x1 = -1;
              if (jl[h] >= 0)
                wave_triangle(EID[js[h]], EID[jl[h]], sh.e1[k[h]], l, r, SW, nullptr, p.owner_higher, x0, x1);
              app.add(x0, x1);
            }
          }
          __syncthreads();  // the chunk's LDS is rewritten by the next one
        }
      }
      __syncthreads();
      // the round's frontier is processed; its support stays l
      for (i32 k = tid; k < nf; k += PB_THREADS) SW[FA[k]] = sw_make(l, ST_PROC);
      const i32 nn = sh.n1;
      __syncthreads();
      i32* t = FA;
      FA = FB;
      FB = t;
      nf = nn;
      ++r;
      ++rounds;
    }
    l += 1;
  }

  // ---- output: trussness = support + 2
  i32 tmax = 0;
  i32* OUT = p.out + e0;
  for (i32 e = tid; e < m; e += PB_THREADS) {
    const i32 t = sw_sup(SW[e]) + 2;
    OUT[e] = t;
    tmax = max(tmax, t);
  }
  tmax = wave_max_i32(tmax);
  tri3 = wave_sum_i64(tri3);
  if (lane == 0) {
    atomicAdd((unsigned long long*)&p.counters[2], (unsigned long long)tri3);
    atomicMax((unsigned long long*)&p.counters[3], (unsigned long long)tmax);
  }
  if (tid == 0) {
    atomicAdd((unsigned long long*)&p.counters[0], (unsigned long long)levels);
    atomicAdd((unsigned long long*)&p.counters[1], (unsigned long long)rounds);
  }
  __syncthreads();  // SW (LDS) is reused by the next graph
}

__global__ __launch_bounds__(PB_THREADS, PB_MIN_WAVES) void k_batch_persist(PbArgs p) {
  extern __shared__ i32 lsw[];  // PB_LDS_EDGES support words
  __shared__ PbShared sh;
  for (;;) {
    if (threadIdx.x == 0) {
      const i32 q = atomicAdd(p.queue, 1);
      sh.g = q < p.nq ? p.order[q] : -1;
    }
    __syncthreads();
    const i32 g = sh.g;
    __syncthreads();
    if (g < 0) break;
    pb_graph(p, g, sh, lsw);
  }
}

__global__ void k_pb_zero(i32* queue, u32* err, i32* bad_graph, i64* counters) {
  if (threadIdx.x == 0) {
    *queue = 0;
    *err = 0;
    *bad_graph = INT_MAX;
    for (int k = 0; k < 4; ++k) counters[k] = 0;
  }
}

struct PbWork {
  i32 *order, *queue, *eb, *eid, *sw, *fa, *fb, *al0, *al1, *bad_graph;
  int2* el;
  u32* err;
  i64* counters;
};

size_t pb_layout(i32 G, i64 total_vtx, i64 total_adj, void* ws, PbWork* w) {
  Carver cv(ws);
  PbWork t;
  const size_t m = (size_t)(total_adj / 2);
  t.order = cv.take<i32>((size_t)G);
  t.queue = cv.take<i32>(1);
  t.err = cv.take<u32>(1);
  t.bad_graph = cv.take<i32>(1);
  t.counters = cv.take<i64>(4);
  t.eb = cv.take<i32>((size_t)total_vtx);
  t.eid = cv.take<i32>((size_t)total_adj);
  t.el = cv.take<int2>(m);
  t.sw = cv.take<i32>(m);
  t.fa = cv.take<i32>(m);
  t.fb = cv.take<i32>(m);
  t.al0 = cv.take<i32>(m);
  t.al1 = cv.take<i32>(m);
  if (w) *w = t;
  return cv.used;
}

}  // namespace

namespace pkt {

size_t persist_workspace_bytes(i32 G, i64 total_vtx, i64 total_adj) {
  return pb_layout(G, total_vtx, total_adj, nullptr, nullptr);
}

// Host side of the persistent mode.  vo, ao: the graph offset arrays on the host
// (already checked by the caller: start at 0, every graph with its offsets entry,
// even slot counts).  Graphs above PB_MAX_EDGES run afterwards, one by one, through
// the single-graph path in the same workspace.
truss_status run_persistent(i32 G, const i64* d_vo, const i64* d_ao, const i32* offs, const i32* adj, i32* out,
                            const std::vector<i64>& vo, const std::vector<i64>& ao, void* ws, const truss_options& opt,
                            truss_stats* stats, hipStream_t s) {
  const i64 total_vtx = vo[G], total_adj = ao[G];
  PbWork w;
  pb_layout(G, total_vtx, total_adj, ws, &w);
  std::vector<i32> order, big;
  order.reserve(G);
  for (i32 g = 0; g < G; ++g) {
    const i64 m = (ao[g + 1] - ao[g]) / 2;
    if (m > PB_MAX_EDGES)
      big.push_back(g);
    else if (m > 0)
      order.push_back(g);
  }
  // longest processing time first: decreasing edge count (ties by graph index)
  std::stable_sort(order.begin(), order.end(),
                   [&](i32 x, i32 y) { return ao[x + 1] - ao[x] > ao[y + 1] - ao[y]; });
  const i32 nq = (i32)order.size();
  // graphs with no edge: nothing to write
  hipLaunchKernelGGL(k_pb_zero, dim3(1), dim3(64), 0, s, w.queue, w.err, w.bad_graph, w.counters);
  PKT_LAUNCH_CHECK();
  if (nq > 0) {
    PKT_HIP(hipMemcpyAsync(w.order, order.data(), sizeof(i32) * (size_t)nq, hipMemcpyHostToDevice, s));
    int dev = 0, cus = 0;
    PKT_HIP(hipGetDevice(&dev));
    PKT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = std::min(nq, std::max(1, cus) * PB_WG_PER_CU);
    PbArgs p;
    p.vo = d_vo;
    p.ao = d_ao;
    p.offs = offs;
    p.adj = adj;
    p.order = w.order;
    p.nq = nq;
    p.queue = w.queue;
    p.eb = w.eb;
    p.eid = w.eid;
    p.el = w.el;
    p.sw = w.sw;
    p.fa = w.fa;
    p.fb = w.fb;
    p.al0 = w.al0;
    p.al1 = w.al1;
    p.out = out;
    p.err = w.err;
    p.bad_graph = w.bad_graph;
    p.counters = w.counters;
    p.owner_higher = opt.owner_rule == 1;
    hipLaunchKernelGGL(k_batch_persist, dim3(blocks), dim3(PB_THREADS), PB_LDS_EDGES * sizeof(i32), s, p);
    PKT_LAUNCH_CHECK();
  }
  u32 err = 0;
  i32 bad = 0;
  i64 cnt[4] = {0, 0, 0, 0};
  PKT_HIP(hipMemcpyAsync(&err, w.err, sizeof(u32), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipMemcpyAsync(&bad, w.bad_graph, sizeof(i32), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipMemcpyAsync(cnt, w.counters, sizeof(cnt), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (err & PB_ERR_INTERNAL) {
    set_error("batch graph %d: level / round count exceeded its bound", bad);
    return TRUSS_E_INTERNAL;
  }
  if (err) {
    set_error("batch graph %d: %s", bad,
              (err & PB_ERR_RANGE) ? "offsets or vertex ids out of range"
                                   : ((err & PB_ERR_NOT_SIMPLE) ? "a row not strictly increasing, or a self-loop"
                                                                : "(u, v) present without (v, u)"));
    return (err & PB_ERR_RANGE) ? TRUSS_E_RANGE : ((err & PB_ERR_NOT_SIMPLE) ? TRUSS_E_NOT_SIMPLE : TRUSS_E_NOT_SYMMETRIC);
  }
  if (stats) {
    stats->m = total_adj / 2;
    stats->levels = cnt[0];
    stats->sublevels = cnt[1];
    stats->triangles = cnt[2] / 3;
    stats->t_max = (i32)cnt[3];
  }
  for (const i32 g : big) {
    Work wg;
    work_layout((i32)(vo[g + 1] - vo[g] - 1), ao[g + 1] - ao[g], true, ws, &wg);
    wg.adj = adj + ao[g];
    truss_status st = prepare_off64(wg, offs + vo[g], s);
    if (st) return st;
    truss_stats gs;
    st = run_single(wg, opt, stats ? &gs : nullptr, out + ao[g] / 2, s, false);
    if (st) {
      set_error("graph %d: %s", g, truss_last_error());
      return st;
    }
    if (stats) {
      stats->levels += gs.levels;
      stats->sublevels += gs.sublevels;
      stats->triangles += gs.triangles;
      stats->t_max = gs.t_max > stats->t_max ? gs.t_max : stats->t_max;
    }
  }
  return TRUSS_OK;
}

}  // namespace pkt
