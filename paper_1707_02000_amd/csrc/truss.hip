// Single-graph truss decomposition on gfx950: input checks, edge ids,
// orientation, support, level-synchronous peeling and the host driver.
//
// Method: Kabir and Madduri, arXiv:1707.02000, PKT section -- support by
// oriented triangle counting with edge ids (Algorithm 3), level scan
// (Algorithm 4), sub-level processing with the lower-edge-id ownership rule and
// the clamp/restore of supports (Algorithm 5 and the text around it).
#include <limits.h>
#include <string.h>

#include <vector>

#include "peel.h"
#include "scan.h"

namespace {

inline int grid_for(i64 count, int cap = 8192) {
  i64 g = (count + PKT_BLOCK - 1) / PKT_BLOCK;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Row containing slot j: the last u with off[u] <= j, searched in [r0, r1].
__device__ __forceinline__ i32 row_of(const i64* __restrict__ off, i32 r0, i32 r1, i64 j) {
  return (i32)(upper_bound_dev(off, (i64)r0, (i64)r1 + 1, j) - 1);
}

// Narrows the row range of the slots [s0, s1] a block will visit (done by two
// lanes, shared through LDS).
__device__ __forceinline__ void block_rows(const i64* __restrict__ off, i32 n, i64 s0, i64 s1, i32* sr) {
  if (threadIdx.x == 0) sr[0] = (i32)(upper_bound_dev(off, (i64)0, (i64)n + 1, s0) - 1);
  if (threadIdx.x == PKT_WAVE) sr[1] = (i32)(upper_bound_dev(off, (i64)0, (i64)n + 1, s1) - 1);
  __syncthreads();
}

// Rank order used to orient edges: by degree, ties by id.
__device__ __forceinline__ bool rank_less(i32 du, i32 u, i32 dv, i32 v) {
  return du < dv || (du == dv && u < v);
}

// ------------------------------------------------------------------ checks

// One wave per row: offsets in range and monotone, ids in range, rows strictly
// ascending (sorted, no duplicates, no self-loop), every (u, v) mirrored.
__global__ __launch_bounds__(PKT_BLOCK) void k_validate(i32 n, const i64* __restrict__ off,
                                                       const i32* __restrict__ adj, i64 two_m,
                                                       u32* __restrict__ verr) {
  const int lane = lane_id();
  const i64 wave = ((i64)blockIdx.x * PKT_BLOCK + threadIdx.x) / PKT_WAVE;
  const i64 nwaves = (i64)gridDim.x * PKT_BLOCK / PKT_WAVE;
  u32 bits = 0;
  if (wave == 0 && lane == 0 && (off[0] != 0 || off[n] != two_m)) bits |= VERR_RANGE;
  for (i64 u = wave; u < n; u += nwaves) {
    const i64 b = off[u], e = off[u + 1];
    if (b < 0 || e < b || e > two_m) {
      bits |= VERR_RANGE;
      continue;
    }
    for (i64 j = b + lane; j < e; j += PKT_WAVE) {
      const i32 v = adj[j];
      if (v < 0 || v >= n) {
        bits |= VERR_RANGE;
        continue;
      }
      if (v == (i32)u || (j > b && adj[j - 1] >= v)) bits |= VERR_NOT_SIMPLE;
      const i64 vb = off[v], ve = off[v + 1];
      if (vb < 0 || ve < vb || ve > two_m) {
        bits |= VERR_RANGE;
        continue;
      }
      const i64 p = lower_bound_dev(adj, vb, ve, (i32)u);
      if (p == ve || adj[p] != (i32)u) bits |= VERR_NOT_SYMMETRIC;
    }
  }
  if (bits) atomicOr(verr, bits);  // only on malformed input
}

// ------------------------------------------------------------ edge ids etc.

// Per row: degree, neighbours below the vertex, and the count above it.  A degree
// whose edges could hold a support past SW_MAX_SUPPORT sets VERR_DEGREE.
__global__ __launch_bounds__(PKT_BLOCK) void k_rowinfo(i32 n, const i64* __restrict__ off,
                                                      const i32* __restrict__ adj, i32* __restrict__ deg,
                                                      i32* __restrict__ locnt, i32* __restrict__ upcnt,
                                                      u32* __restrict__ verr) {
  for (i64 u = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; u < n; u += (i64)gridDim.x * PKT_BLOCK) {
    const i64 b = off[u], e = off[u + 1];
    const i64 lo = lower_bound_dev(adj, b, e, (i32)u) - b;
    if (e - b > (i64)SW_MAX_SUPPORT + 1) atomicOr(verr, VERR_DEGREE);  // support <= degree - 1
    deg[u] = (i32)(e - b);
    locnt[u] = (i32)lo;
    upcnt[u] = (i32)(e - b - lo);
  }
}

// Per adjacency slot: edge id (rank of (min, max) in row-major order), the
// endpoint list, and the orientation flag (neighbour ranks above the row's
// vertex).
__global__ __launch_bounds__(PKT_BLOCK) void k_slots(i32 n, i64 two_m, const i64* __restrict__ off,
                                                    const i32* __restrict__ adj, const i32* __restrict__ deg,
                                                    const i32* __restrict__ locnt, const i64* __restrict__ ebase,
                                                    i32* __restrict__ eid, int2* __restrict__ el,
                                                    u8* __restrict__ oflag) {
  __shared__ i32 sr[2];
  for (i64 s0 = (i64)blockIdx.x * PKT_BLOCK; s0 < two_m; s0 += (i64)gridDim.x * PKT_BLOCK) {
    const i64 s1 = min(s0 + PKT_BLOCK, two_m) - 1;
    block_rows(off, n, s0, s1, sr);
    const i64 j = s0 + threadIdx.x;
    if (j <= s1) {
      const i32 u = row_of(off, sr[0], sr[1], j);
      const i32 v = adj[j];
      const i64 p = j - off[u];
      i64 e;
      if (p >= locnt[u]) {
        e = ebase[u] + (p - locnt[u]);
        el[e] = make_int2(u, v);
      } else {
        const i64 q = lower_bound_dev(adj, off[v], off[v + 1], u) - off[v];
        e = ebase[v] + (q - locnt[v]);
      }
      eid[j] = (i32)e;
      oflag[j] = rank_less(deg[u], u, deg[v], v) ? 1 : 0;
    }
    __syncthreads();
  }
}

// Oriented CSR: the slots flagged above, in their original (sorted-by-id)
// order; X is the exclusive scan of the flags.  Edge ids only when asked (with ids
// in rank order, slot d holds edge d).
__global__ __launch_bounds__(PKT_BLOCK) void k_orient(i32 n, i64 two_m, const i64* __restrict__ off,
                                                     const i32* __restrict__ adj, const i32* __restrict__ eid,
                                                     const u8* __restrict__ oflag, const i64* __restrict__ X,
                                                     i64* __restrict__ ooff, i32* __restrict__ oadj,
                                                     i32* __restrict__ oeid, int write_eid) {
  const i64 tid = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x, stride = (i64)gridDim.x * PKT_BLOCK;
  for (i64 j = tid; j < two_m; j += stride)
    if (oflag[j]) {
      const i64 d = X[j];
      oadj[d] = adj[j];
      if (write_eid) oeid[d] = eid[j];
    }
  for (i64 u = tid; u <= n; u += stride) ooff[u] = X[off[u]];
}

// ------------------------------------------------------------------ support

#define SUP_THREADS 256
#ifndef SUP_DMAX
#define SUP_DMAX 1024          // largest out-row hashed in LDS (16 KB of LDS per block: 8 blocks
#endif                         // per CU; 2048 measured 1.6x slower for the lost occupancy)
#ifndef SUP_BLOCKS
#define SUP_BLOCKS 2048        // workgroups of the support kernel (they drain a work queue)
#endif
#define SUP_TBL (2 * SUP_DMAX)  // hash slots (power of two)
#ifndef SUP_CHUNK
#define SUP_CHUNK 8             // vertices taken from the work queue at a time
#endif
#ifndef SUP_UNROLL
#define SUP_UNROLL 2            // out-row entries per lane in flight
#endif

// Support by oriented triangle counting (Algorithm 3's scheme, one workgroup per
// vertex instead of one thread): vertices are ranked by (degree, id) and every
// triangle is found once, from its lowest-rank vertex u and middle vertex v, as
// w in N+(u) ∩ N+(v).  The workgroup of u puts N+(u) in an LDS hash table
// (the role of the paper's mark array X: key w -> slot of w in N+(u)), walks
// N+(v) for every v in N+(u), and probes each w there.  Each triangle adds one
// to its three edges: edge (v, w) by a global atomic, edges (u, v) and (u, w)
// through LDS counters per slot of N+(u), flushed once per u.  Rows longer than
// SUP_DMAX take a path with binary searches instead.  Vertices come from
// an atomic work queue in chunks (dynamic scheduling); with ids in rank order (a
// relabelled graph) the queue runs from the highest id down, so the vertices with
// the most work start first and the light ones fill the tail.
// Edge id of oriented slot k: oeid[k], or k itself when the ids follow the rank
// (IDENT: the oriented CSR is then the rows' upper halves in edge order), which
// saves the support walk one of its two loads per entry.
template <bool IDENT>
__device__ __forceinline__ i32 oid(const i32* __restrict__ oeid, i64 k) {
  return IDENT ? (i32)k : oeid[k];
}

// Long out-row (more than SUP_DMAX entries): one wave per v in N+(u), lanes over
// N+(v), each w looked up by binary search in N+(u) -- staged sorted in LDS (the
// hash table's space) when it fits in 2 * SUP_DMAX entries, else in memory; all
// three edges by global atomics.
template <bool IDENT>
__device__ void support_long_row(i32 b_u, i64 b, i32 d, const i64* __restrict__ ooff, const i32* __restrict__ oadj,
                                 const i32* __restrict__ oeid, i32* __restrict__ sw, i32* lds) {
  const bool staged = d <= 2 * SUP_DMAX;
  if (staged) {
    for (int i = threadIdx.x; i < d; i += SUP_THREADS) lds[i] = oadj[b + i];
    __syncthreads();
  }
  const int lane = lane_id(), wid = threadIdx.x / PKT_WAVE;
  for (i32 i = wid; i < d; i += SUP_THREADS / PKT_WAVE) {
    const i32 v = oadj[b + i];
    const i64 vb = ooff[v], ve = ooff[v + 1];
    i32 c_uv = 0;
    for (i64 k = vb + lane; k < ve; k += PKT_WAVE) {
      const i32 w = oadj[k];
      i64 p;
      bool hit;
      if (staged) {
        const i32 q = lower_bound_dev(lds, (i32)0, d, w);
        hit = q < d && lds[q] == w;
        p = b + q;
      } else {
        p = lower_bound_dev(oadj, b, b + d, w);
        hit = p < b + d && oadj[p] == w;
      }
      if (hit) {
        atomicAdd(&sw[oid<IDENT>(oeid, p)], SW_ONE);  // edge (u, w)
        atomicAdd(&sw[oid<IDENT>(oeid, k)], SW_ONE);  // edge (v, w)
        ++c_uv;
      }
    }
    c_uv = (i32)wave_sum_i64(c_uv);
    if (lane == 0 && c_uv) atomicAdd(&sw[oid<IDENT>(oeid, b + i)], c_uv * SW_ONE);  // edge (u, v)
  }
  __syncthreads();  // the LDS is the next vertex's table
}

template <bool IDENT>
__global__ __launch_bounds__(SUP_THREADS) void k_support(i32 n, const i64* __restrict__ ooff,
                                                        const i32* __restrict__ oadj, const i32* __restrict__ oeid,
                                                        i32* __restrict__ sw, i32* __restrict__ queue) {
  __shared__ i32 keys[SUP_TBL];
  __shared__ unsigned short slot[SUP_TBL];
  __shared__ i32 cnt[SUP_DMAX];
  __shared__ i32 s_u0;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) s_u0 = atomicAdd(queue, SUP_CHUNK);
    __syncthreads();
    const i32 u0 = s_u0;
    __syncthreads();
    if (u0 >= n) break;
    const i32 u1 = min(n, u0 + SUP_CHUNK);
    for (i32 uq = u0; uq < u1; ++uq) {
      const i32 u = IDENT ? n - 1 - uq : uq;  // rank order: the heavy vertices first
      const i64 b = ooff[u];
      const i32 d = (i32)(ooff[u + 1] - b);
      if (d < 2) continue;
      if (d > SUP_DMAX) {
        support_long_row<IDENT>(u, b, d, ooff, oadj, oeid, sw, keys);
        continue;
      }
      int tbits = 6;
      while ((1 << tbits) < 2 * d) ++tbits;
      const int tsize = 1 << tbits;
      for (int i = tid; i < tsize; i += SUP_THREADS) keys[i] = -1;
      for (int i = tid; i < d; i += SUP_THREADS) cnt[i] = 0;
      __syncthreads();
      // N+(u) into the table
      for (int i = tid; i < d; i += SUP_THREADS) {
        const i32 w = oadj[b + i];
        u32 h = ((u32)w * 0x9E3779B1u) >> (32 - tbits);
        for (;;) {
          const i32 old = atomicCAS(&keys[h], -1, w);
          if (old == -1) {
            slot[h] = (unsigned short)i;
            break;
          }
          h = (h + 1) & (tsize - 1);
        }
      }
      __syncthreads();
      // one wave per v in N+(u); lanes walk N+(v) and probe the table.  The
      // wave's next v and the row bounds of the one after are loaded while the
      // current row is walked (two dependent loads per v, off the critical path).
      const int lane = lane_id(), wid = tid / PKT_WAVE;
      constexpr int NWV = SUP_THREADS / PKT_WAVE;
      i32 v1 = wid + NWV < d ? oadj[b + wid + NWV] : 0;
      i64 vb = 0, ve = 0;
      if (wid < d) {
        const i32 v0 = oadj[b + wid];
        vb = ooff[v0];
        ve = ooff[v0 + 1];
      }
      for (i32 i = wid; i < d; i += NWV) {
        const bool more1 = i + NWV < d, more2 = i + 2 * NWV < d;
        const i32 v2 = more2 ? oadj[b + i + 2 * NWV] : 0;
        const i64 vb1 = more1 ? ooff[v1] : 0, ve1 = more1 ? ooff[v1 + 1] : 0;
        i32 c_uv = 0;
        // SUP_UNROLL entries per lane in flight, each with its edge id (coalesced
        // loads, issued together; the id is not fetched after a hit)
        for (i64 k0 = vb + lane; k0 < ve; k0 += SUP_UNROLL * PKT_WAVE) {
          i32 wq[SUP_UNROLL], fq[SUP_UNROLL];
#pragma unroll
          for (int q = 0; q < SUP_UNROLL; ++q) {
            const i64 k = k0 + q * PKT_WAVE;
            wq[q] = k < ve ? oadj[k] : -1;
            fq[q] = k < ve ? oid<IDENT>(oeid, k) : -1;
          }
#pragma unroll
          for (int q = 0; q < SUP_UNROLL; ++q) {
            const i32 w = wq[q];
            if (w < 0) continue;
            u32 h = ((u32)w * 0x9E3779B1u) >> (32 - tbits);
            for (;;) {
              const i32 key = keys[h];
              if (key == w) {
                atomicAdd(&cnt[slot[h]], 1);  // edge (u, w)
                atomicAdd(&sw[fq[q]], SW_ONE);  // edge (v, w)
                ++c_uv;
                break;
              }
              if (key == -1) break;
              h = (h + 1) & (tsize - 1);
            }
          }
        }
        c_uv = (i32)wave_sum_i64(c_uv);
        if (lane == 0 && c_uv) atomicAdd(&cnt[i], c_uv);  // edge (u, v)
        vb = vb1;
        ve = ve1;
        v1 = v2;
      }
      __syncthreads();
      for (int i = tid; i < d; i += SUP_THREADS)
        if (cnt[i]) atomicAdd(&sw[oid<IDENT>(oeid, b + i)], cnt[i] * SW_ONE);
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(PKT_BLOCK) void k_fill_i32(i32* __restrict__ a, i64 n, i32 v) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < n; i += (i64)gridDim.x * PKT_BLOCK) a[i] = v;
}

__global__ __launch_bounds__(PKT_BLOCK) void k_iota(i32* __restrict__ a, i64 n) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < n; i += (i64)gridDim.x * PKT_BLOCK) a[i] = (i32)i;
}

// Sum of supports (3 x triangles) into ctl->tri3.
__global__ __launch_bounds__(PKT_BLOCK) void k_sum_support(const i32* __restrict__ sw, i64 m, Ctl* ctl) {
  i64 s = 0;
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < m; i += (i64)gridDim.x * PKT_BLOCK) s += sw_sup(sw[i]);
  s = wave_sum_i64(s);
  if (lane_id() == 0 && s) atomicAdd((unsigned long long*)&ctl->tri3, (unsigned long long)s);
}

// Working-CSR rebuild: keep the slots whose edge is not processed.
struct KeepLen {
  const u8* flag;
  i64 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 i) const { return flag[i]; }
};

__global__ __launch_bounds__(PKT_BLOCK) void k_keep_flags(Csr c, i64 slots, const i32* __restrict__ sw,
                                                         const Ctl* __restrict__ ctl, u8* __restrict__ flag) {
  const i32 r = ctl->sublevels;  // between rounds: the next round's index
  for (i64 j = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; j < slots; j += (i64)gridDim.x * PKT_BLOCK)
    flag[j] = !is_processed(sw_st(sw[c.eid[j]]), r);
}

__global__ __launch_bounds__(PKT_BLOCK) void k_compact(i32 n, Csr c, i64 slots, const u8* __restrict__ flag,
                                                      const i64* __restrict__ X, i64* __restrict__ doff,
                                                      i32* __restrict__ dadj, i32* __restrict__ deid) {
  const i64 tid = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x, stride = (i64)gridDim.x * PKT_BLOCK;
  for (i64 j = tid; j < slots; j += stride)
    if (flag[j]) {
      const i64 d = X[j];
      dadj[d] = c.adj[j];
      deid[d] = c.eid[j];
    }
  for (i64 u = tid; u <= n; u += stride) doff[u] = X[c.off[u]];
}


__global__ void k_after_compact(Ctl* ctl, i32 dst, i32 m) {
  ctl->csel = dst;
  ctl->csr_edges = m - ctl->processed;
  ctl->compactions += 1;
}

// trussness = final support + 2 (Algorithm 1's last step; Algorithm 4 output).
__global__ __launch_bounds__(PKT_BLOCK) void k_output(const i32* __restrict__ sw, i64 m, i32* __restrict__ out,
                                                     Ctl* ctl) {
  i32 mx = 0;
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < m; i += (i64)gridDim.x * PKT_BLOCK) {
    const i32 t = sw_sup(sw[i]) + 2;
    out[i] = t;
    mx = max(mx, t);
  }
  mx = wave_max_i32(mx);
  if (lane_id() == 0) atomicMax(&ctl->tmax_s, mx);
}

// Support alone (no peeling): the support field of every word.
__global__ __launch_bounds__(PKT_BLOCK) void k_support_out(const i32* __restrict__ sw, i64 m, i32* __restrict__ out) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < m; i += (i64)gridDim.x * PKT_BLOCK)
    out[i] = sw_sup(sw[i]);
}

__global__ void k_off32_to_64(const i32* __restrict__ a, i64* __restrict__ b, i64 n) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < n; i += (i64)gridDim.x * PKT_BLOCK) b[i] = a[i];
}

}  // namespace

// ------------------------------------------------------------------ host side

size_t work_layout(i32 n, i64 two_m, bool off32, void* base, Work* w) {
  Carver cv(base);
  const i64 m = two_m / 2;
  Work t;
  memset(&t, 0, sizeof(t));
  t.n = n;
  t.two_m = two_m;
  t.m = m;
  t.ctl = cv.take<Ctl>(1);
  t.verr = cv.take<u32>(4);
  t.partial = cv.take<i64>(SCAN_BLOCKS + 1);
  t.bmin = cv.take<i32>(SCAN_BLOCKS);
  if (off32) t.off64 = cv.take<i64>((size_t)n + 1);
  t.deg = cv.take<i32>((size_t)n);
  t.locnt = cv.take<i32>((size_t)n);
  t.upcnt = cv.take<i32>((size_t)n);
  t.ebase = cv.take<i64>((size_t)n + 1);
  t.eid = cv.take<i32>((size_t)two_m);
  t.el = cv.take<int2>((size_t)m);
  t.sw = cv.take<i32>((size_t)m);
  for (int k = 0; k < 3; ++k) t.F[k] = cv.take<i32>((size_t)m);
  for (int k = 0; k < 2; ++k) t.A[k] = cv.take<i32>((size_t)m);
  for (int k = 0; k < 2; ++k) {
    t.coff[k] = cv.take<i64>((size_t)n + 1);
    t.cadj[k] = cv.take<i32>((size_t)two_m);
    t.ceid[k] = cv.take<i32>((size_t)two_m);
  }
  t.flag = cv.take<u8>((size_t)two_m);
  t.X = cv.take<i64>((size_t)two_m + 1);
  t.ooff = t.coff[1];
  t.oadj = t.cadj[1];
  t.oeid = t.ceid[1];
  if (w) *w = t;
  return cv.used;
}

namespace pkt {

namespace {
inline i32 n_of(const Work& w) { return w.n; }
inline int grid_for_h(i64 count, int cap = 8192) {
  i64 g = (count + PKT_BLOCK - 1) / PKT_BLOCK;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}
}  // namespace

truss_status validate_input(const Work& w, hipStream_t s) {
  PKT_HIP(hipMemsetAsync(w.verr, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_validate, dim3(grid_for_h((i64)w.n * PKT_WAVE, 4096)), dim3(PKT_BLOCK), 0, s, w.n, w.off,
                     w.adj, w.two_m, w.verr);
  PKT_LAUNCH_CHECK();
  u32 bits = 0;
  PKT_HIP(hipMemcpyAsync(&bits, w.verr, sizeof(u32), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (bits & VERR_RANGE) {
    set_error("input CSR: offsets or vertex ids out of range");
    return TRUSS_E_RANGE;
  }
  if (bits & VERR_NOT_SIMPLE) {
    set_error("input CSR: a row is not strictly ascending or has a self-loop");
    return TRUSS_E_NOT_SIMPLE;
  }
  if (bits & VERR_NOT_SYMMETRIC) {
    set_error("input CSR: an edge (u, v) has no mirror (v, u)");
    return TRUSS_E_NOT_SYMMETRIC;
  }
  return TRUSS_OK;
}

// Edge ids, endpoint list and oriented CSR.
truss_status build_edges(const Work& w, hipStream_t s) {
  const i32 n = w.n;
  // Only a graph of more than SW_MAX_SUPPORT edges can hold an edge of larger
  // support (s triangles on one edge take 2 s + 1 edges); only then is the degree
  // check read back.
  const bool big = w.m > (i64)SW_MAX_SUPPORT;
  if (big) PKT_HIP(hipMemsetAsync(w.verr, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_rowinfo, dim3(grid_for_h(n)), dim3(PKT_BLOCK), 0, s, n, w.off, w.adj, w.deg, w.locnt,
                     w.upcnt, w.verr);
  if (big) {
    u32 bits = 0;
    PKT_HIP(hipMemcpyAsync(&bits, w.verr, sizeof(u32), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
    if (bits & VERR_DEGREE) {
      set_error("a vertex has degree above %d: its supports would not fit the 29-bit support field",
                SW_MAX_SUPPORT + 1);
      return TRUSS_E_RANGE;
    }
  }
  PKT_HIP(scan_launch(ArrayLen<i32>{(const i32*)w.upcnt, n}, w.partial, w.ebase, &w.ctl->scan_arrive, s));
  hipLaunchKernelGGL(k_slots, dim3(grid_for_h(w.two_m)), dim3(PKT_BLOCK), 0, s, n, w.two_m, w.off, w.adj, w.deg,
                     w.locnt, w.ebase, w.eid, w.el, w.flag);
  PKT_HIP(scan_launch(ArrayLen<u8>{w.flag, w.two_m}, w.partial, w.X, &w.ctl->scan_arrive, s));
  hipLaunchKernelGGL(k_orient, dim3(grid_for_h(w.two_m)), dim3(PKT_BLOCK), 0, s, n, w.two_m, w.off, w.adj, w.eid,
                     w.flag, w.X, w.ooff, w.oadj, w.oeid, w.id_order ? 0 : 1);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

truss_status compute_support(const Work& w, hipStream_t s) {
  // support 0, state ST_ALIVE
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for_h(w.m, 2048)), dim3(PKT_BLOCK), 0, s, w.sw, w.m, sw_make(0, ST_ALIVE));
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, s, &w.ctl->work_queue, (i64)1, 0);
  if (w.id_order)
    hipLaunchKernelGGL(k_support<true>, dim3(SUP_BLOCKS), dim3(SUP_THREADS), 0, s, n_of(w), (const i64*)w.ooff,
                       (const i32*)w.oadj, (const i32*)w.oeid, w.sw, &w.ctl->work_queue);
  else
    hipLaunchKernelGGL(k_support<false>, dim3(SUP_BLOCKS), dim3(SUP_THREADS), 0, s, n_of(w), (const i64*)w.ooff,
                       (const i32*)w.oadj, (const i32*)w.oeid, w.sw, &w.ctl->work_queue);
  hipLaunchKernelGGL(k_sum_support, dim3(grid_for_h(w.m, 2048)), dim3(PKT_BLOCK), 0, s, (const i32*)w.sw, w.m,
                     w.ctl);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

truss_status init_peel(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(grid_for_h(w.m, 2048)), dim3(PKT_BLOCK), 0, s, w.A[0], w.m);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

CsrSet csr_set(const Work& w) {
  CsrSet cs;
  cs.c[0] = Csr{w.off, w.adj, w.eid};
  cs.c[1] = Csr{w.coff[0], w.cadj[0], w.ceid[0]};
  cs.c[2] = Csr{w.coff[1], w.cadj[1], w.ceid[1]};
  return cs;
}

// Rebuilds the working CSR from the current one, dropping processed edges.
truss_status compact(const Work& w, hipStream_t s) {
  Ctl hc;
  PKT_HIP(hipMemcpyAsync(&hc, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  const CsrSet cs = csr_set(w);
  const Csr cur = cs.c[hc.csel];
  const int dst = (hc.csel == 1) ? 2 : 1;
  i64 slots = 0;
  PKT_HIP(hipMemcpyAsync(&slots, cur.off + w.n, sizeof(i64), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  hipLaunchKernelGGL(k_keep_flags, dim3(grid_for_h(slots)), dim3(PKT_BLOCK), 0, s, cur, slots,
                     (const i32*)w.sw, (const Ctl*)w.ctl, w.flag);
  PKT_HIP(scan_launch(KeepLen{w.flag, slots}, w.partial, w.X, &w.ctl->scan_arrive, s));
  hipLaunchKernelGGL(k_compact, dim3(grid_for_h(slots)), dim3(PKT_BLOCK), 0, s, w.n, cur, slots,
                     (const u8*)w.flag, (const i64*)w.X, w.coff[dst - 1], w.cadj[dst - 1], w.ceid[dst - 1]);
  hipLaunchKernelGGL(k_after_compact, dim3(1), dim3(1), 0, s, w.ctl, dst, (i32)w.m);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

truss_status write_output(const Work& w, i32* out, hipStream_t s) {
  hipLaunchKernelGGL(k_output, dim3(grid_for_h(w.m, 2048)), dim3(PKT_BLOCK), 0, s, (const i32*)w.sw, w.m, out,
                     w.ctl);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

truss_status write_support(const Work& w, i32* out, hipStream_t s) {
  hipLaunchKernelGGL(k_support_out, dim3(grid_for_h(w.m, 2048)), dim3(PKT_BLOCK), 0, s, (const i32*)w.sw, w.m, out);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

truss_status prepare_off64(Work& w, const i32* off32, hipStream_t s) {
  hipLaunchKernelGGL(k_off32_to_64, dim3(grid_for_h((i64)w.n + 1)), dim3(PKT_BLOCK), 0, s, off32, w.off64,
                     (i64)w.n + 1);
  PKT_LAUNCH_CHECK();
  w.off = w.off64;
  return TRUSS_OK;
}

}  // namespace pkt

namespace {
__global__ void k_split_el(const int2* __restrict__ el, i64 m, i32* __restrict__ a, i32* __restrict__ b) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < m; i += (i64)gridDim.x * PKT_BLOCK) {
    const int2 e = el[i];
    a[i] = e.x;
    b[i] = e.y;
  }
}
}  // namespace

namespace pkt {
truss_status run_edge_list(const Work& w, i32* el_u, i32* el_v, hipStream_t s) {
  if (w.m == 0) return TRUSS_OK;
  PKT_HIP(hipMemsetAsync(w.ctl, 0, sizeof(Ctl), s));  // zeroed counters for the scans
  truss_status st = build_edges(w, s);
  if (st) return st;
  hipLaunchKernelGGL(k_split_el, dim3(grid_for(w.m)), dim3(PKT_BLOCK), 0, s, (const int2*)w.el, w.m, el_u, el_v);
  PKT_LAUNCH_CHECK();
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}
}  // namespace pkt
