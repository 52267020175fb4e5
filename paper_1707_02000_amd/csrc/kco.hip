// Vertex reordering by increasing core number (KCO) before support, as in the
// support-computation study of the Performance Results section (Table 2): the new ids
// sort vertices by core number (ties by old id), the relabelled CSR keeps every
// row sorted, and the trussness computed on the relabelled graph is mapped back to
// the input's edge ids (trussness does not depend on the labels).
//
// Both sorts are one stable LSD radix sort of (u32 key, i32 value) pairs, eight
// key bits per pass.  A block ranks its tile of RS_TILE pairs stably by digit (a
// wave finds its lanes of equal digit with eight ballots; earlier sub-steps, then
// lower waves, then lower lanes come first): a first pass writes the tile's digit
// counts into a digit-major matrix, the device prefix of that matrix (scan.h)
// gives every (digit, tile) its first place, and a second pass stages the tile in
// LDS in digit order and writes it out in runs of consecutive places.  The
// order sorts (core, v) by core; the relabelled CSR sorts (new row, new neighbour)
// pairs, produced in increasing order of the neighbour, by row, which leaves every
// row sorted.
#include <limits.h>

#include "common.h"
#include "launch.h"
#include "scan.h"

namespace {

constexpr int RS_BINS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_ITEMS * PKT_BLOCK;
constexpr int RS_WAVES = PKT_BLOCK / PKT_WAVE;
static_assert(PKT_BLOCK == RS_BINS, "one thread per digit");

inline i64 rs_tiles(i64 cnt) { return (cnt + RS_TILE - 1) / RS_TILE; }

inline int bit_width(i64 x) {
  int b = 0;
  while (x > 0) {
    ++b;
    x >>= 1;
  }
  return b;
}

// Lanes of this wave whose digit equals this lane's (valid lanes only).
__device__ __forceinline__ u64 same_digit(bool valid, int d) {
  u64 same = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1;
    const u64 bb = __ballot(bit);
    same &= bit ? bb : ~bb;
  }
  return same;
}

// Digit counts of tile blockIdx.x into hist[digit * tiles + tile]: one LDS atomic
// per run of equal digits in a wave.
__global__ __launch_bounds__(PKT_BLOCK) void k_rs_count(i64 cnt, i64 tiles, const u32* __restrict__ keys, int shift,
                                                       i32* __restrict__ hist) {
  __shared__ i32 h[RS_BINS];
  const int tid = threadIdx.x, lane = lane_id();
  const i64 t = blockIdx.x;
  h[tid] = 0;
  __syncthreads();
  const u64 below = (1ull << lane) - 1ull;
  for (int sub = 0; sub < RS_ITEMS; ++sub) {
    const i64 i = t * RS_TILE + (i64)sub * PKT_BLOCK + tid;
    const bool valid = i < cnt;
    const int d = valid ? (int)((keys[i] >> shift) & (u32)(RS_BINS - 1)) : 0;
    const u64 same = same_digit(valid, d);
    if (valid && __popcll(same & below) == 0) atomicAdd(&h[d], __popcll(same));
  }
  __syncthreads();
  hist[(i64)tid * tiles + t] = h[tid];
}

// Scatter of tile blockIdx.x.  Every pair's stable rank among the tile's pairs of
// its digit (earlier sub-steps, then lower waves, then lower lanes first) puts it
// into LDS in digit order; the tile then leaves LDS in that order, so that the
// lanes of a wave write runs of consecutive places: pair p of digit d goes to
// start[d * tiles + tile] + (p - first LDS place of d).
__global__ __launch_bounds__(PKT_BLOCK) void k_rs_scatter(i64 cnt, i64 tiles, const u32* __restrict__ keys,
                                                         const i32* __restrict__ vals, int shift,
                                                         const i32* __restrict__ hist, const i64* __restrict__ start,
                                                         u32* __restrict__ okeys, i32* __restrict__ ovals) {
  __shared__ u32 lk[RS_TILE];
  __shared__ i32 lv[RS_TILE];
  __shared__ i32 wc[RS_WAVES][RS_BINS];  // this sub-step's count per wave and digit
  __shared__ i32 run[RS_BINS];           // the tile's pairs per digit before this sub-step
  __shared__ i32 lstart[RS_BINS];        // first LDS place of every digit
  __shared__ i64 base[RS_BINS];
  __shared__ i64 tmp[RS_WAVES];
  const int tid = threadIdx.x, wid = tid / PKT_WAVE, lane = lane_id();
  const i64 t = blockIdx.x;
  i64 total;
  lstart[tid] = (i32)block_excl_scan_i64((i64)hist[(i64)tid * tiles + t], tmp, &total);
  base[tid] = start[(i64)tid * tiles + t];
  run[tid] = 0;
  for (int w = 0; w < RS_WAVES; ++w) wc[w][tid] = 0;
  __syncthreads();
  const u64 below = (1ull << lane) - 1ull;
  for (int sub = 0; sub < RS_ITEMS; ++sub) {
    const i64 i = t * RS_TILE + (i64)sub * PKT_BLOCK + tid;
    const bool valid = i < cnt;
    const u32 key = valid ? keys[i] : 0u;
    const i32 val = valid ? vals[i] : 0;
    const int d = (int)((key >> shift) & (u32)(RS_BINS - 1));
    const u64 same = same_digit(valid, d);
    const int lower = __popcll(same & below);
    if (valid && lower == 0) wc[wid][d] = __popcll(same);
    __syncthreads();
    if (valid) {
      i32 r = lstart[d] + run[d] + lower;
      for (int w = 0; w < wid; ++w) r += wc[w][d];
      lk[r] = key;
      lv[r] = val;
    }
    __syncthreads();
    i32 tot = 0;
    for (int w = 0; w < RS_WAVES; ++w) {
      tot += wc[w][tid];
      wc[w][tid] = 0;
    }
    run[tid] += tot;
    __syncthreads();
  }
  for (i64 p = tid; p < total; p += PKT_BLOCK) {
    const u32 key = lk[p];
    const int d = (int)((key >> shift) & (u32)(RS_BINS - 1));
    const i64 pos = base[d] + (p - lstart[d]);
    okeys[pos] = key;
    ovals[pos] = lv[p];
  }
}

struct HistLen {
  const i32* h;
  i64 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 i) const { return h[i]; }
};

struct RsBufs {
  u32* k[2];
  i32* v[2];
  i32* hist;
  i64* start;
  i64* partial;
  u32* arrive;  // zeroed before the first pass; the prefix leaves it zeroed
};

void rs_take(Carver& cv, i64 cnt, RsBufs* b) {
  const i64 cells = rs_tiles(cnt) * RS_BINS;
  for (int q = 0; q < 2; ++q) b->k[q] = cv.take<u32>((size_t)cnt);
  for (int q = 0; q < 2; ++q) b->v[q] = cv.take<i32>((size_t)cnt);
  b->hist = cv.take<i32>((size_t)cells);
  b->start = cv.take<i64>((size_t)cells + 1);
  b->partial = cv.take<i64>(SCAN_BLOCKS + 1);
  b->arrive = cv.take<u32>(1);
}

// Sorts the cnt pairs in k[0], v[0] stably by their low `bits` key bits; *sel is
// the buffer that holds the result.
truss_status rs_sort(i64 cnt, int bits, const RsBufs& b, hipStream_t s, int* sel) {
  int q = 0;
  if (cnt > 0) {
    const i64 tiles = rs_tiles(cnt);
    if (tiles >= ((i64)1 << 24)) {  // a launch holds fewer than 2^32 work-items
      pkt::set_error("radix sort of %lld pairs: too many", (long long)cnt);
      return TRUSS_E_ARG;
    }
    for (int shift = 0; shift < bits; shift += 8) {
      hipLaunchKernelGGL(k_rs_count, dim3((unsigned)tiles), dim3(PKT_BLOCK), 0, s, cnt, tiles, (const u32*)b.k[q],
                         shift, b.hist);
      PKT_HIP(scan_launch(HistLen{b.hist, tiles * RS_BINS}, b.partial, b.start, b.arrive, s));
      hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)tiles), dim3(PKT_BLOCK), 0, s, cnt, tiles, (const u32*)b.k[q],
                         (const i32*)b.v[q], shift, (const i32*)b.hist, (const i64*)b.start, b.k[q ^ 1], b.v[q ^ 1]);
      PKT_LAUNCH_CHECK();
      q ^= 1;
    }
  }
  *sel = q;
  return TRUSS_OK;
}

struct KoFlags {
  u32 err;
  i32 kmax;
};

truss_status read_flags(const KoFlags* d, KoFlags* h, hipStream_t s) {
  PKT_HIP(hipMemcpyAsync(h, d, sizeof(KoFlags), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

// ---------------------------------------------------------------- the order

__global__ __launch_bounds__(PKT_BLOCK) void k_ko_init(i32 n, const i32* __restrict__ core, u32* __restrict__ keys,
                                                      i32* __restrict__ vals, KoFlags* fl) {
  i32 mx = 0;
  const i64 n_up = ((i64)n + PKT_WAVE - 1) / PKT_WAVE * PKT_WAVE;  // whole waves stay in the loop
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n_up; v += (i64)gridDim.x * PKT_BLOCK) {
    if (v < n) {
      const i32 c = core[v];
      if (c < 0) atomicOr(&fl->err, 1u);
      keys[v] = (u32)(c < 0 ? 0 : c);
      vals[v] = (i32)v;
      mx = max(mx, c);
    }
  }
  __shared__ i32 wm[RS_WAVES];
  mx = wave_max_i32(mx);
  if (lane_id() == 0) wm[threadIdx.x / PKT_WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {  // one atomic per block: per-wave ones on one address serialise
    for (int w = 1; w < RS_WAVES; ++w) mx = max(mx, wm[w]);
    if (mx > 0) atomicMax(&fl->kmax, mx);
  }
}

__global__ __launch_bounds__(PKT_BLOCK) void k_ko_out(i32 n, const i32* __restrict__ sorted, i32* __restrict__ order,
                                                     i32* __restrict__ new_id, KoFlags* fl) {
  for (i64 i = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; i < n; i += (i64)gridDim.x * PKT_BLOCK) {
    const i32 v = sorted[i];  // a permutation of 0..n-1: the values start as the ids
    order[i] = v;
    if (v >= 0 && v < n)
      new_id[v] = (i32)i;
    else
      atomicOr(&fl->err, 2u);
  }
}

size_t ko_layout(i32 n, void* ws, RsBufs* b, KoFlags** fl) {
  Carver cv(ws);
  RsBufs t;
  rs_take(cv, n, &t);
  KoFlags* f = cv.take<KoFlags>(1);
  if (b) *b = t;
  if (fl) *fl = f;
  return cv.used;
}

// ------------------------------------------------------ the relabelled CSR

// Offsets in order and inside the adjacency, and new_id a permutation with
// order its inverse: order[new_id[v]] == v for every v (new_id is read as an
// index only after its range check).
__global__ __launch_bounds__(PKT_BLOCK) void k_rl_check(i32 n, i64 two_m, const i64* __restrict__ off,
                                                       const i32* __restrict__ new_id, const i32* __restrict__ order,
                                                       KoFlags* fl) {
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK) {
    const i64 b = off[v], e = off[v + 1];
    if ((v == 0 && b != 0) || b < 0 || e < b || e > two_m) atomicOr(&fl->err, 1u);
    const i32 x = new_id[v];
    if (x < 0 || x >= n || order[x] != (i32)v) atomicOr(&fl->err, 2u);
  }
}

// Row length of new vertex y: the degree of the old vertex order[y].
struct RelabelRows {
  const i32* order;
  const i64* off;
  i32 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 y) const {
    const i32 u = order[y];
    return off[u + 1] - off[u];
  }
};

// Slot j of old row u becomes the pair (new_id[adj[j]], new_id[u]) at place
// off2[new_id[u]] + (j - off[u]): grouped by the new id of u, increasing.  A block
// takes PKT_BLOCK consecutive slots at a time and finds the rows of its first and
// last slot once, so every lane searches only the few rows in between.
__global__ __launch_bounds__(PKT_BLOCK) void k_rl_pairs(i32 n, i64 two_m, const i64* __restrict__ off,
                                                       const i32* __restrict__ adj, const i32* __restrict__ new_id,
                                                       const i64* __restrict__ off2, u32* __restrict__ keys,
                                                       i32* __restrict__ vals, KoFlags* fl) {
  __shared__ i64 rows[2];
  const i64 chunks = (two_m + PKT_BLOCK - 1) / PKT_BLOCK;
  for (i64 c = blockIdx.x; c < chunks; c += gridDim.x) {  // uniform over the block
    const i64 j0 = c * PKT_BLOCK;
    const i64 j1 = min(j0 + PKT_BLOCK, two_m) - 1;
    if (threadIdx.x < 2)
      rows[threadIdx.x] = upper_bound_dev(off, (i64)0, (i64)n + 1, threadIdx.x == 0 ? j0 : j1) - 1;
    __syncthreads();
    const i64 j = j0 + threadIdx.x;
    if (j <= j1) {
      const i32 u = (i32)(upper_bound_dev(off, rows[0], rows[1] + 1, j) - 1);
      const i32 w = adj[j];
      if (w < 0 || w >= n) {  // checked before any use as an index
        atomicOr(&fl->err, 4u);
      } else {
        const i32 y = new_id[u];
        const i64 pos = off2[y] + (j - off[u]);
        keys[pos] = (u32)new_id[w];
        vals[pos] = y;
      }
    }
    __syncthreads();  // rows[] is rewritten for the next chunk
  }
}

// Row x of the sorted pairs starts where off2 says: true of every symmetric CSR.
__global__ __launch_bounds__(PKT_BLOCK) void k_rl_rows(i32 n, i64 two_m, const u32* __restrict__ keys,
                                                      const i64* __restrict__ off2, KoFlags* fl) {
  for (i64 x = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; x < n; x += (i64)gridDim.x * PKT_BLOCK)
    if (lower_bound_dev(keys, (i64)0, two_m, (u32)x) != off2[x]) atomicOr(&fl->err, 8u);
}

// Every slot's mirror: entry y in row x of the sorted pairs needs x in row y.
// The row counts alone (k_rl_rows) pass an asymmetric CSR whose in- and
// out-degrees agree at every vertex (a directed cycle), whose sorted pairs are then
// its transpose; this check rejects it.  Rows are located per block chunk as in
// k_rl_pairs.
__global__ __launch_bounds__(PKT_BLOCK) void k_rl_mirror(i32 n, i64 two_m, const i64* __restrict__ off2,
                                                        const i32* __restrict__ adj2, KoFlags* fl) {
  __shared__ i64 rows[2];
  const i64 chunks = (two_m + PKT_BLOCK - 1) / PKT_BLOCK;
  for (i64 c = blockIdx.x; c < chunks; c += gridDim.x) {  // uniform over the block
    const i64 j0 = c * PKT_BLOCK;
    const i64 j1 = min(j0 + PKT_BLOCK, two_m) - 1;
    if (threadIdx.x < 2)
      rows[threadIdx.x] = upper_bound_dev(off2, (i64)0, (i64)n + 1, threadIdx.x == 0 ? j0 : j1) - 1;
    __syncthreads();
    const i64 j = j0 + threadIdx.x;
    if (j <= j1) {
      const i32 x = (i32)(upper_bound_dev(off2, rows[0], rows[1] + 1, j) - 1);
      const i32 y = adj2[j];  // a vertex id: every value of the pairs is some new_id[u]
      const i64 b = off2[y], e = off2[y + 1];
      const i64 q = lower_bound_dev(adj2, b, e, x);
      if (q == e || adj2[q] != x) atomicOr(&fl->err, 8u);
    }
    __syncthreads();  // rows[] is rewritten for the next chunk
  }
}

size_t rl_layout(i64 two_m, void* ws, RsBufs* b, KoFlags** fl) {
  Carver cv(ws);
  RsBufs t;
  rs_take(cv, two_m, &t);
  KoFlags* f = cv.take<KoFlags>(1);
  if (b) *b = t;
  if (fl) *fl = f;
  return cv.used;
}

// ---------------------------------------------------------------- mapping back

__global__ __launch_bounds__(PKT_BLOCK) void k_map_check(i32 n, i64 two_m, const i64* __restrict__ off2,
                                                        const i32* __restrict__ new_id, KoFlags* fl) {
  for (i64 v = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; v < n; v += (i64)gridDim.x * PKT_BLOCK) {
    const i64 b = off2[v], e = off2[v + 1];
    if ((v == 0 && b != 0) || b < 0 || e < b || e > two_m) atomicOr(&fl->err, 1u);
    const i32 x = new_id[v];
    if (x < 0 || x >= n) atomicOr(&fl->err, 2u);
  }
}

// First entry of row x of the relabelled graph above x: its canonical edges run
// from there to the row's end.
__global__ __launch_bounds__(PKT_BLOCK) void k_first_upper(i32 n, const i64* __restrict__ off2,
                                                          const i32* __restrict__ adj2, i64* __restrict__ fa) {
  for (i64 x = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; x < n; x += (i64)gridDim.x * PKT_BLOCK)
    fa[x] = upper_bound_dev(adj2, off2[x], off2[x + 1], (i32)x);
}

struct UpperRows {
  const i64* off2;
  const i64* fa;
  i32 n;
  __device__ bool active() const { return true; }
  __device__ i64 count() const { return n; }
  __device__ i64 len(i64 x) const { return off2[x + 1] - fa[x]; }
};

// tau[e] = tau2[edge id of (new_id[u], new_id[v]) in the relabelled graph]: the
// canonical edges of the rows before a, then the rank of b among row a's entries
// above a.
__global__ __launch_bounds__(PKT_BLOCK) void k_map(i32 n, i64 m, const i32* __restrict__ eu,
                                                  const i32* __restrict__ ev, const i32* __restrict__ new_id,
                                                  const i64* __restrict__ off2, const i32* __restrict__ adj2,
                                                  const i64* __restrict__ FA, const i64* __restrict__ U,
                                                  const i32* __restrict__ tau2, i32* __restrict__ tau, KoFlags* fl) {
  for (i64 e = (i64)blockIdx.x * PKT_BLOCK + threadIdx.x; e < m; e += (i64)gridDim.x * PKT_BLOCK) {
    const i32 u = eu[e], v = ev[e];
    i32 t = -1;
    if (u < 0 || u >= n || v < 0 || v >= n) {
      atomicOr(&fl->err, 4u);
    } else {
      const i32 x = new_id[u], y = new_id[v];
      const i32 a = min(x, y), b = max(x, y);
      const i64 end = off2[a + 1];
      const i64 fa = FA[a];
      const i64 pos = lower_bound_dev(adj2, fa, end, b);
      const i64 id = U[a] + (pos - fa);
      if (a == b || pos == end || adj2[pos] != b || id >= m)
        atomicOr(&fl->err, 8u);
      else
        t = tau2[id];
    }
    tau[e] = t;
  }
}

size_t map_layout(i32 n, void* ws, i64** FA, i64** U, i64** partial, u32** arrive, KoFlags** fl) {
  Carver cv(ws);
  i64* f0 = cv.take<i64>((size_t)n);
  i64* u = cv.take<i64>((size_t)n + 1);
  i64* p = cv.take<i64>(SCAN_BLOCKS + 1);
  u32* a = cv.take<u32>(1);
  KoFlags* f = cv.take<KoFlags>(1);
  if (FA) *FA = f0;
  if (U) *U = u;
  if (partial) *partial = p;
  if (arrive) *arrive = a;
  if (fl) *fl = f;
  return cv.used;
}

bool ws_ok(void* ws, size_t bytes, size_t need) {
  if (ws == nullptr || bytes < need || ((uintptr_t)ws & 255u)) {
    pkt::set_error("workspace: need %zu bytes at 256-byte alignment", need);
    return false;
  }
  return true;
}

}  // namespace

namespace pkt {

// Order and relabelled CSR for the library's own use (truss_decompose's relabelling):
// the inputs are known good (validated CSR, non-negative keys below 2^key_bits), so
// nothing is checked and nothing waits on the host.  The scratch (kco_scratch_bytes)
// is free again on return.
size_t kco_scratch_bytes(i32 n, i64 two_m) {
  const size_t a = ko_layout(n, nullptr, nullptr, nullptr), b = rl_layout(two_m, nullptr, nullptr, nullptr);
  return a > b ? a : b;
}

// new_id / order by increasing (keys[v], v).
truss_status kco_order_run(i32 n, const i32* keys, int key_bits, i32* new_id, i32* order, void* scratch,
                           hipStream_t s) {
  if (n == 0) return TRUSS_OK;
  RsBufs b;
  KoFlags* fl;
  ko_layout(n, scratch, &b, &fl);
  PKT_HIP(hipMemsetAsync(fl, 0, sizeof(KoFlags), s));
  PKT_HIP(hipMemsetAsync(b.arrive, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_ko_init, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, keys, b.k[0], b.v[0], fl);
  PKT_LAUNCH_CHECK();
  int q = 0;
  if (truss_status st = rs_sort(n, key_bits, b, s, &q)) return st;
  hipLaunchKernelGGL(k_ko_out, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, (const i32*)b.v[q], order, new_id, fl);
  PKT_LAUNCH_CHECK();
  return TRUSS_OK;
}

// The relabelled CSR (rows sorted) of a valid symmetric CSR.
truss_status kco_relabel_run(i32 n, i64 two_m, const i64* off, const i32* adj, const i32* new_id, const i32* order,
                             i64* off2, i32* adj2, void* scratch, hipStream_t s) {
  const i64 max_slots = (((i64)1 << 24) - 1) * RS_TILE;  // the radix sort's launch limit
  if (two_m > max_slots) {
    set_error("relabelling: %lld adjacency slots, above the radix sort's %lld", (long long)two_m,
              (long long)max_slots);
    return TRUSS_E_RANGE;
  }
  RsBufs b;
  KoFlags* fl;
  rl_layout(two_m, scratch, &b, &fl);
  PKT_HIP(hipMemsetAsync(fl, 0, sizeof(KoFlags), s));
  PKT_HIP(hipMemsetAsync(b.arrive, 0, sizeof(u32), s));
  PKT_HIP(scan_launch(RelabelRows{order, off, n}, b.partial, off2, b.arrive, s));
  if (two_m == 0) return TRUSS_OK;
  hipLaunchKernelGGL(k_rl_pairs, dim3(grid_items(two_m)), dim3(PKT_BLOCK), 0, s, n, two_m, off, adj, new_id,
                     (const i64*)off2, b.k[0], b.v[0], fl);
  PKT_LAUNCH_CHECK();
  int q = 0;
  if (truss_status st = rs_sort(two_m, bit_width((i64)n - 1), b, s, &q)) return st;
  PKT_HIP(hipMemcpyAsync(adj2, b.v[q], sizeof(i32) * (size_t)two_m, hipMemcpyDeviceToDevice, s));
  return TRUSS_OK;
}

int kco_bits(i64 x) { return bit_width(x); }

}  // namespace pkt

extern "C" truss_status truss_kco_order_workspace_bytes(int32_t n, size_t* bytes) {
  pkt::set_error("");
  if (n < 0 || bytes == nullptr) {
    pkt::set_error("bad arguments to truss_kco_order_workspace_bytes");
    return TRUSS_E_ARG;
  }
  *bytes = ko_layout(n, nullptr, nullptr, nullptr);
  return TRUSS_OK;
}

extern "C" truss_status truss_kco_order(int32_t n, const int32_t* core, int32_t* new_id, int32_t* order,
                                        void* workspace, size_t workspace_bytes, void* stream) {
  using namespace pkt;
  set_error("");
  if (n < 0 || (n > 0 && (core == nullptr || new_id == nullptr || order == nullptr))) {
    set_error("bad n or NULL core / new_id / order");
    return TRUSS_E_ARG;
  }
  if (!ws_ok(workspace, workspace_bytes, ko_layout(n, nullptr, nullptr, nullptr))) return TRUSS_E_WORKSPACE;
  if (n == 0) return TRUSS_OK;
  hipStream_t s = (hipStream_t)stream;
  RsBufs b;
  KoFlags* fl;
  ko_layout(n, workspace, &b, &fl);
  PKT_HIP(hipMemsetAsync(fl, 0, sizeof(KoFlags), s));
  PKT_HIP(hipMemsetAsync(b.arrive, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_ko_init, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, core, b.k[0], b.v[0], fl);
  PKT_LAUNCH_CHECK();
  KoFlags h;
  if (truss_status st = read_flags(fl, &h, s)) return st;
  if (h.err) {
    set_error("a negative core number");
    return TRUSS_E_RANGE;
  }
  int q = 0;
  if (truss_status st = rs_sort(n, bit_width(h.kmax), b, s, &q)) return st;
  hipLaunchKernelGGL(k_ko_out, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, (const i32*)b.v[q], order, new_id, fl);
  PKT_LAUNCH_CHECK();
  if (truss_status st = read_flags(fl, &h, s)) return st;
  if (h.err) {
    set_error("radix sort: output is not a permutation");
    return TRUSS_E_INTERNAL;
  }
  return TRUSS_OK;
}

extern "C" truss_status truss_kco_relabel_workspace_bytes(int32_t n, int64_t two_m, size_t* bytes) {
  pkt::set_error("");
  if (n < 0 || two_m < 0 || bytes == nullptr) {
    pkt::set_error("bad arguments to truss_kco_relabel_workspace_bytes");
    return TRUSS_E_ARG;
  }
  *bytes = rl_layout(two_m, nullptr, nullptr, nullptr);
  return TRUSS_OK;
}

extern "C" truss_status truss_kco_relabel(int32_t n, const int64_t* offsets, const int32_t* adj, const int32_t* new_id,
                                          const int32_t* order, int64_t* offsets2, int32_t* adj2, void* workspace,
                                          size_t workspace_bytes, void* stream) {
  using namespace pkt;
  set_error("");
  if (n < 0 || (n > 0 && (offsets == nullptr || new_id == nullptr || order == nullptr)) || offsets2 == nullptr) {
    set_error("bad n or NULL offsets / new_id / order / offsets2");
    return TRUSS_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  i64 two_m = 0;
  if (n > 0) {
    PKT_HIP(hipMemcpyAsync(&two_m, offsets + n, sizeof(i64), hipMemcpyDeviceToHost, s));
    PKT_HIP(hipStreamSynchronize(s));
  }
  const i64 max_slots = (((i64)1 << 24) - 1) * RS_TILE;  // the radix sort's launch limit
  if (two_m < 0 || two_m > max_slots) {
    set_error("offsets[n] = %lld is out of range [0, %lld]", (long long)two_m, (long long)max_slots);
    return TRUSS_E_RANGE;
  }
  if (two_m > 0 && (adj == nullptr || adj2 == nullptr)) {
    set_error("NULL adj / adj2");
    return TRUSS_E_ARG;
  }
  if (!ws_ok(workspace, workspace_bytes, rl_layout(two_m, nullptr, nullptr, nullptr))) return TRUSS_E_WORKSPACE;
  if (n == 0) {
    PKT_HIP(hipMemsetAsync(offsets2, 0, sizeof(i64), s));
    return TRUSS_OK;
  }
  RsBufs b;
  KoFlags* fl;
  rl_layout(two_m, workspace, &b, &fl);
  PKT_HIP(hipMemsetAsync(fl, 0, sizeof(KoFlags), s));
  PKT_HIP(hipMemsetAsync(b.arrive, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_rl_check, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, two_m, offsets, new_id, order, fl);
  PKT_LAUNCH_CHECK();
  KoFlags h;
  if (truss_status st = read_flags(fl, &h, s)) return st;
  if (h.err) {
    set_error(h.err & 1u ? "input CSR: offsets not starting at 0, out of order or past offsets[n]"
                         : "new_id is not a permutation with order its inverse");
    return TRUSS_E_RANGE;
  }
  PKT_HIP(scan_launch(RelabelRows{order, offsets, n}, b.partial, offsets2, b.arrive, s));
  hipLaunchKernelGGL(k_rl_pairs, dim3(grid_items(two_m)), dim3(PKT_BLOCK), 0, s, n, two_m, offsets, adj, new_id,
                     (const i64*)offsets2, b.k[0], b.v[0], fl);
  PKT_LAUNCH_CHECK();
  if (truss_status st = read_flags(fl, &h, s)) return st;
  if (h.err) {
    set_error("input CSR: a neighbour id outside [0, n)");
    return TRUSS_E_RANGE;
  }
  int q = 0;
  if (truss_status st = rs_sort(two_m, bit_width((i64)n - 1), b, s, &q)) return st;
  hipLaunchKernelGGL(k_rl_rows, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, two_m, (const u32*)b.k[q],
                     (const i64*)offsets2, fl);
  PKT_LAUNCH_CHECK();
  if (two_m > 0) PKT_HIP(hipMemcpyAsync(adj2, b.v[q], sizeof(i32) * (size_t)two_m, hipMemcpyDeviceToDevice, s));
  if (truss_status st = read_flags(fl, &h, s)) return st;
  if (!h.err && two_m > 0) {  // rows line up: every slot's mirror must be there too
    hipLaunchKernelGGL(k_rl_mirror, dim3(grid_items(two_m)), dim3(PKT_BLOCK), 0, s, n, two_m,
                       (const i64*)offsets2, (const i32*)adj2, fl);
    PKT_LAUNCH_CHECK();
    if (truss_status st = read_flags(fl, &h, s)) return st;
  }
  if (h.err) {
    set_error("input CSR: (u, v) present without (v, u)");
    return TRUSS_E_NOT_SYMMETRIC;
  }
  return TRUSS_OK;
}

extern "C" truss_status truss_kco_map_workspace_bytes(int32_t n, size_t* bytes) {
  pkt::set_error("");
  if (n < 0 || bytes == nullptr) {
    pkt::set_error("bad arguments to truss_kco_map_workspace_bytes");
    return TRUSS_E_ARG;
  }
  *bytes = map_layout(n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  return TRUSS_OK;
}

extern "C" truss_status truss_kco_map(int32_t n, int64_t m, const int32_t* el_u, const int32_t* el_v,
                                      const int32_t* new_id, const int64_t* offsets2, const int32_t* adj2,
                                      const int32_t* trussness2, int32_t* trussness, void* workspace,
                                      size_t workspace_bytes, void* stream) {
  using namespace pkt;
  set_error("");
  if (n < 0 || m < 0 || (n > 0 && (new_id == nullptr || offsets2 == nullptr)) ||
      (m > 0 && (n == 0 || el_u == nullptr || el_v == nullptr || adj2 == nullptr || trussness2 == nullptr ||
                 trussness == nullptr))) {
    set_error("bad n, m or a NULL argument");
    return TRUSS_E_ARG;
  }
  if (!ws_ok(workspace, workspace_bytes, map_layout(n, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr)))
    return TRUSS_E_WORKSPACE;
  if (m == 0) return TRUSS_OK;
  hipStream_t s = (hipStream_t)stream;
  i64 two_m = 0;
  PKT_HIP(hipMemcpyAsync(&two_m, offsets2 + n, sizeof(i64), hipMemcpyDeviceToHost, s));
  PKT_HIP(hipStreamSynchronize(s));
  if (two_m != 2 * m) {
    set_error("offsets2[n] = %lld, not 2m = %lld", (long long)two_m, (long long)(2 * m));
    return TRUSS_E_ARG;
  }
  i64 *FA, *U, *partial;
  u32* arrive;
  KoFlags* fl;
  map_layout(n, workspace, &FA, &U, &partial, &arrive, &fl);
  PKT_HIP(hipMemsetAsync(fl, 0, sizeof(KoFlags), s));
  PKT_HIP(hipMemsetAsync(arrive, 0, sizeof(u32), s));
  hipLaunchKernelGGL(k_map_check, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, two_m, offsets2, new_id, fl);
  PKT_LAUNCH_CHECK();
  KoFlags h;
  if (truss_status st = read_flags(fl, &h, s)) return st;
  if (h.err) {
    set_error(h.err & 1u ? "relabelled CSR: offsets not starting at 0, out of order or past offsets2[n]"
                         : "new_id: a value outside [0, n)");
    return TRUSS_E_RANGE;
  }
  hipLaunchKernelGGL(k_first_upper, dim3(grid_items(n)), dim3(PKT_BLOCK), 0, s, n, offsets2, adj2, FA);
  PKT_HIP(scan_launch(UpperRows{offsets2, FA, n}, partial, U, arrive, s));
  hipLaunchKernelGGL(k_map, dim3(grid_items(m)), dim3(PKT_BLOCK), 0, s, n, (i64)m, el_u, el_v, new_id, offsets2, adj2,
                     (const i64*)FA, (const i64*)U, trussness2, trussness, fl);
  PKT_LAUNCH_CHECK();
  if (truss_status st = read_flags(fl, &h, s)) return st;
  if (h.err) {
    set_error(h.err & 4u ? "edge list: an endpoint outside [0, n)"
                         : "an input edge has no image in the relabelled graph");
    return TRUSS_E_RANGE;
  }
  return TRUSS_OK;
}
