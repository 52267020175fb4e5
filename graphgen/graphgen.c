/*
 * Seeded synthetic graph generators: Erdos-Renyi, R-MAT, Chung-Lu with
 * planted cliques, 2-D random geometric graphs, and a packed batch of mixed
 * small graphs.  Every output is a simple undirected graph in CSR form:
 * rows strictly ascending (sorted, no duplicates), no self-loops, symmetric.
 *
 * This module only produces inputs.  It holds none of the truss
 * decomposition arithmetic and is shared by the tests, the benchmark and the
 * smoke check, which feed the same CSR to the GPU library and to the CPU
 * oracle.
 *
 * Randomness: a counter-based generator built from the SplitMix64 output
 * finalizer (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  Every draw is a pure function of
 * (seed, stream, counter), so results do not depend on the thread count.
 *
 * Memory returned through out-pointers is malloc'd; release it with gg_free.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG */

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* One 64-bit draw for (seed, stream, counter). */
static inline uint64_t rng3(uint64_t seed, uint64_t stream, uint64_t ctr) {
  uint64_t s = mix64(seed + 0x9e3779b97f4a7c15ULL);
  s = mix64(s ^ (stream * 0xd1b54a32d192ed03ULL));
  return mix64(s + ctr * 0x9e3779b97f4a7c15ULL);
}

/* Uniform double in [0, 1) from the top 53 bits. */
static inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, k) (k > 0), by 128-bit multiply-shift. */
static inline uint64_t below(uint64_t x, uint64_t k) {
  return (uint64_t)(((unsigned __int128)x * (unsigned __int128)k) >> 64);
}

/* --------------------------------------------------------- small sorts */

static void isort_i32(int32_t* a, int64_t n) {
  for (int64_t i = 1; i < n; ++i) {
    int32_t x = a[i];
    int64_t j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}

/* In-place LSD radix sort of non-negative int32 keys; tmp has n entries. */
static void rsort_i32(int32_t* a, int32_t* tmp, int64_t n) {
  if (n < 64) {
    isort_i32(a, n);
    return;
  }
  int32_t* src = a;
  int32_t* dst = tmp;
  for (int shift = 0; shift < 32; shift += 8) {
    int64_t cnt[256];
    memset(cnt, 0, sizeof(cnt));
    for (int64_t i = 0; i < n; ++i) cnt[((uint32_t)src[i] >> shift) & 255u]++;
    int64_t s = 0;
    for (int b = 0; b < 256; ++b) {
      int64_t c = cnt[b];
      cnt[b] = s;
      s += c;
    }
    for (int64_t i = 0; i < n; ++i) dst[cnt[((uint32_t)src[i] >> shift) & 255u]++] = src[i];
    int32_t* t = src;
    src = dst;
    dst = t;
  }
  /* four passes: the result is back in a */
}

/* Sort and dedup one row; returns the new length. */
static int64_t sort_unique_row(int32_t* row, int64_t len) {
  if (len <= 1) return len;
  if (len < 64) {
    isort_i32(row, len);
  } else {
    int32_t* tmp = (int32_t*)malloc((size_t)len * sizeof(int32_t));
    rsort_i32(row, tmp, len);
    free(tmp);
  }
  int64_t k = 1;
  for (int64_t i = 1; i < len; ++i)
    if (row[i] != row[k - 1]) row[k++] = row[i];
  return k;
}

/* ----------------------------------------------- pairs -> simple CSR */

/*
 * Build a simple symmetric CSR over n vertices from npairs endpoint pairs
 * (us[i], vs[i]).  Self-loops are dropped, each pair is inserted in both
 * directions, rows are sorted and deduplicated.  If perm is non-NULL, vertex
 * x is renamed perm[x] first.  Returns 0, or -1 on allocation failure.
 */
static int pairs_to_csr(int32_t n, int64_t npairs, const int32_t* us, const int32_t* vs,
                        const int32_t* perm, int64_t** off_out, int32_t** adj_out) {
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    int32_t u = us[i], v = vs[i];
    if (u == v) continue;
    if (perm) {
      u = perm[u];
      v = perm[v];
    }
    __atomic_fetch_add(&cnt[u + 1], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&cnt[v + 1], 1, __ATOMIC_RELAXED);
  }
  for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  int64_t total = cnt[n];
  int32_t* raw = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t) + 8);
  if (!raw || !fill) {
    free(cnt);
    free(raw);
    free(fill);
    return -1;
  }
  memcpy(fill, cnt, (size_t)n * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    int32_t u = us[i], v = vs[i];
    if (u == v) continue;
    if (perm) {
      u = perm[u];
      v = perm[v];
    }
    raw[__atomic_fetch_add(&fill[u], 1, __ATOMIC_RELAXED)] = v;
    raw[__atomic_fetch_add(&fill[v], 1, __ATOMIC_RELAXED)] = u;
  }
  free(fill);
  int64_t* ulen = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!ulen) {
    free(cnt);
    free(raw);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int32_t u = 0; u < n; ++u) ulen[u] = sort_unique_row(raw + cnt[u], cnt[u + 1] - cnt[u]);
  int64_t* off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!off) {
    free(cnt);
    free(raw);
    free(ulen);
    return -1;
  }
  off[0] = 0;
  for (int32_t u = 0; u < n; ++u) off[u + 1] = off[u] + ulen[u];
  int32_t* adj = (int32_t*)malloc((size_t)(off[n] > 0 ? off[n] : 1) * sizeof(int32_t));
  if (!adj) {
    free(cnt);
    free(raw);
    free(ulen);
    free(off);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int32_t u = 0; u < n; ++u) memcpy(adj + off[u], raw + cnt[u], (size_t)ulen[u] * sizeof(int32_t));
  free(cnt);
  free(raw);
  free(ulen);
  *off_out = off;
  *adj_out = adj;
  return 0;
}

/* Seeded uniform random permutation of [0, n) (Fisher-Yates). */
static int32_t* make_perm(int32_t n, uint64_t seed, uint64_t stream) {
  int32_t* p = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!p) return NULL;
  for (int32_t i = 0; i < n; ++i) p[i] = i;
  for (int64_t i = (int64_t)n - 1; i > 0; --i) {
    int64_t j = (int64_t)below(rng3(seed, stream, (uint64_t)i), (uint64_t)i + 1);
    int32_t t = p[i];
    p[i] = p[j];
    p[j] = t;
  }
  return p;
}

void gg_free(void* p) { free(p); }

/* ------------------------------------------------------------------ ER */

/*
 * G(n, p): every unordered pair independently with probability p, drawn by
 * geometric skipping over the n(n-1)/2 pairs in row-major upper order.
 */
int gg_er(int32_t n, double p, uint64_t seed, int64_t** off, int32_t** adj) {
  if (n < 0 || p < 0.0 || p > 1.0) return -2;
  int64_t npairs_all = (int64_t)n * (n - 1) / 2;
  int64_t cap = (int64_t)(npairs_all * p + 10.0 * sqrt(npairs_all * p + 1.0) + 16.0);
  if (cap > npairs_all) cap = npairs_all;
  int32_t* us = (int32_t*)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int32_t));
  int32_t* vs = (int32_t*)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int32_t));
  if (!us || !vs) {
    free(us);
    free(vs);
    return -1;
  }
  int64_t k = 0;
  if (p > 0.0 && npairs_all > 0) {
    double lq = (p < 1.0) ? log1p(-p) : 0.0;
    int64_t idx = -1;
    uint64_t ctr = 0;
    int32_t u = 0;
    int64_t row_start = 0; /* linear index of pair (u, u+1) */
    for (;;) {
      if (p >= 1.0) {
        idx += 1;
      } else {
        double r = u01(rng3(seed, 1, ctr++));
        double skip = floor(log1p(-r) / lq);
        if (skip > (double)npairs_all) break;
        idx += 1 + (int64_t)skip;
      }
      if (idx >= npairs_all) break;
      while (idx >= row_start + (n - 1 - u)) {
        row_start += n - 1 - u;
        ++u;
      }
      int32_t v = (int32_t)(u + 1 + (idx - row_start));
      if (k >= cap) {
        cap = cap * 2 + 16;
        us = (int32_t*)realloc(us, (size_t)cap * sizeof(int32_t));
        vs = (int32_t*)realloc(vs, (size_t)cap * sizeof(int32_t));
        if (!us || !vs) return -1;
      }
      us[k] = u;
      vs[k] = v;
      ++k;
    }
  }
  int rc = pairs_to_csr(n, k, us, vs, NULL, off, adj);
  free(us);
  free(vs);
  return rc;
}

/* ---------------------------------------------------------------- R-MAT */

/*
 * R-MAT: npairs endpoint pairs, each built bit by bit over `scale` levels by
 * picking quadrant (0,0), (0,1), (1,0), (1,1) with probabilities a, b, c,
 * 1-a-b-c.  Endpoints >= n are rejected (n <= 2^scale).  Pairs are
 * symmetrized, self-loops dropped, duplicates merged; ids are permuted if
 * `permute` is set.
 */
int gg_rmat(int32_t scale, int32_t n, int64_t npairs, double a, double b, double c, int32_t permute,
            uint64_t seed, int64_t** off, int32_t** adj) {
  if (scale < 0 || scale > 30 || n < 0 || (int64_t)n > ((int64_t)1 << scale) || npairs < 0) return -2;
  int32_t* us = (int32_t*)malloc((size_t)(npairs > 0 ? npairs : 1) * sizeof(int32_t));
  int32_t* vs = (int32_t*)malloc((size_t)(npairs > 0 ? npairs : 1) * sizeof(int32_t));
  if (!us || !vs) {
    free(us);
    free(vs);
    return -1;
  }
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < npairs; ++i) {
    uint32_t u = 0, v = 0;
    for (int32_t bit = 0; bit < scale; ++bit) {
      double r = u01(rng3(seed, 2, (uint64_t)i * 64u + (uint64_t)bit));
      uint32_t hi = 0, lo = 0;
      if (r < a) {
      } else if (r < ab) {
        lo = 1;
      } else if (r < abc) {
        hi = 1;
      } else {
        hi = 1;
        lo = 1;
      }
      u = (u << 1) | hi;
      v = (v << 1) | lo;
    }
    if ((int64_t)u >= n || (int64_t)v >= n) {
      u = 0;
      v = 0; /* rejected: encoded as a self-loop, dropped later */
    }
    us[i] = (int32_t)u;
    vs[i] = (int32_t)v;
  }
  int32_t* perm = NULL;
  if (permute) {
    perm = make_perm(n, seed, 3);
    if (!perm) {
      free(us);
      free(vs);
      return -1;
    }
  }
  int rc = pairs_to_csr(n, npairs, us, vs, perm, off, adj);
  free(perm);
  free(us);
  free(vs);
  return rc;
}

/* ------------------------------------------------------- Chung-Lu + cliques */

/*
 * Chung-Lu power-law graph: weights w_i = (i + i0)^(-1/(beta-1)), with i0
 * chosen by bisection so that the largest expected degree equals
 * sqrt(sum of expected degrees) for a target of `target_m` edges (the
 * admissibility bound of the Chung-Lu model).  `draws` endpoint pairs are
 * sampled proportionally to w (inverse CDF), then `ncliques` cliques with
 * sizes uniform in [cmin, cmax] are planted on uniformly random distinct
 * vertex sets.  Ids are permuted if `permute` is set.
 */
int gg_chunglu(int32_t n, double beta, double target_m, int64_t draws, int32_t ncliques, int32_t cmin,
               int32_t cmax, int32_t permute, uint64_t seed, int64_t** off, int32_t** adj) {
  if (n < 2 || beta <= 1.0 || draws < 0 || ncliques < 0 || cmin < 2 || cmax < cmin || cmax > n) return -2;
  const double gam = 1.0 / (beta - 1.0);
  const double want = 1.0 / sqrt(2.0 * target_m); /* w_0 / sum(w) */
  double lo = 0.0, hi = (double)n * 4.0;
  double* cdf = (double*)malloc((size_t)n * sizeof(double));
  if (!cdf) return -1;
  /* The weight sum of the bisection is the sum of two fixed halves, each summed in
   * index order, whatever the thread count (a parallel reduction's rounding would
   * depend on it, and the bisection's last steps with it). */
  const int32_t half = n - n / 2;
  for (int it = 0; it < 60; ++it) {
    double i0 = 0.5 * (lo + hi);
    double part[2] = {0.0, 0.0};
#pragma omp parallel for schedule(static, 1) num_threads(2)
    for (int h = 0; h < 2; ++h) {
      double t = 0.0;
      for (int32_t i = (h ? half : 0); i < (h ? n : half); ++i) t += pow((double)i + i0 + 1.0, -gam);
      part[h] = t;
    }
    double s = part[0] + part[1];
    double ratio = pow(i0 + 1.0, -gam) / s;
    if (ratio > want)
      lo = i0; /* head too heavy: shift further */
    else
      hi = i0;
  }
  double i0 = 0.5 * (lo + hi);
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    s += pow((double)i + i0 + 1.0, -gam);
    cdf[i] = s;
  }
  for (int32_t i = 0; i < n; ++i) cdf[i] /= s;
  cdf[n - 1] = 1.0;

  int64_t clique_pairs = 0;
  int32_t* csize = (int32_t*)malloc((size_t)(ncliques > 0 ? ncliques : 1) * sizeof(int32_t));
  if (!csize) {
    free(cdf);
    return -1;
  }
  for (int32_t q = 0; q < ncliques; ++q) {
    csize[q] = cmin + (int32_t)below(rng3(seed, 5, (uint64_t)q), (uint64_t)(cmax - cmin + 1));
    clique_pairs += (int64_t)csize[q] * (csize[q] - 1) / 2;
  }
  int64_t total = draws + clique_pairs;
  int32_t* us = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  int32_t* vs = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  if (!us || !vs) {
    free(cdf);
    free(csize);
    free(us);
    free(vs);
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < draws; ++i) {
    for (int side = 0; side < 2; ++side) {
      double r = u01(rng3(seed, 4, (uint64_t)i * 2u + (uint64_t)side));
      int32_t l = 0, h = n - 1; /* first index with cdf > r */
      while (l < h) {
        int32_t mid = l + (h - l) / 2;
        if (cdf[mid] > r)
          h = mid;
        else
          l = mid + 1;
      }
      if (side == 0)
        us[i] = l;
      else
        vs[i] = l;
    }
  }
  free(cdf);
  /* cliques: distinct members by rejection against a per-clique mark array */
  int64_t at = draws;
  uint8_t* mark = (uint8_t*)calloc((size_t)n, 1);
  int32_t* mem = (int32_t*)malloc((size_t)cmax * sizeof(int32_t));
  if (!mark || !mem) {
    free(mark);
    free(mem);
    free(csize);
    free(us);
    free(vs);
    return -1;
  }
  uint64_t ctr = 0;
  for (int32_t q = 0; q < ncliques; ++q) {
    int32_t k = 0;
    while (k < csize[q]) {
      int32_t x = (int32_t)below(rng3(seed, 6, ctr++), (uint64_t)n);
      if (mark[x]) continue;
      mark[x] = 1;
      mem[k++] = x;
    }
    for (int32_t i = 0; i < k; ++i) {
      mark[mem[i]] = 0;
      for (int32_t j = i + 1; j < k; ++j) {
        us[at] = mem[i];
        vs[at] = mem[j];
        ++at;
      }
    }
  }
  free(mark);
  free(mem);
  free(csize);
  int32_t* perm = NULL;
  if (permute) {
    perm = make_perm(n, seed, 7);
    if (!perm) {
      free(us);
      free(vs);
      return -1;
    }
  }
  int rc = pairs_to_csr(n, total, us, vs, perm, off, adj);
  free(perm);
  free(us);
  free(vs);
  return rc;
}

/* ------------------------------------------------------------------ RGG */

/*
 * 2-D random geometric graph: n points uniform in [0,1)^2 (float64), edge
 * iff Euclidean distance < r, with r = sqrt(k / (pi (n - 1))) for a target
 * mean degree k (ignoring the boundary).  Candidate pairs come from a grid
 * of cells of side >= r.
 */
int gg_rgg(int32_t n, double k, uint64_t seed, int64_t** off, int32_t** adj) {
  if (n < 1 || k < 0.0) return -2;
  double r = (n > 1) ? sqrt(k / (M_PI * (double)(n - 1))) : 0.0;
  double* x = (double*)malloc((size_t)n * sizeof(double));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  if (!x || !y) {
    free(x);
    free(y);
    return -1;
  }
  for (int32_t i = 0; i < n; ++i) {
    x[i] = u01(rng3(seed, 8, (uint64_t)i * 2u));
    y[i] = u01(rng3(seed, 8, (uint64_t)i * 2u + 1u));
  }
  int32_t g = (r > 0.0) ? (int32_t)floor(1.0 / r) : 1;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  int64_t cells = (int64_t)g * g;
  int64_t* cstart = (int64_t*)calloc((size_t)cells + 1, sizeof(int64_t));
  int32_t* cid = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* order = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!cstart || !cid || !order) {
    free(x);
    free(y);
    free(cstart);
    free(cid);
    free(order);
    return -1;
  }
  for (int32_t i = 0; i < n; ++i) {
    int32_t cx = (int32_t)(x[i] * g), cy = (int32_t)(y[i] * g);
    if (cx >= g) cx = g - 1;
    if (cy >= g) cy = g - 1;
    cid[i] = cy * g + cx;
    cstart[cid[i] + 1]++;
  }
  for (int64_t c = 0; c < cells; ++c) cstart[c + 1] += cstart[c];
  {
    int64_t* fill = (int64_t*)malloc((size_t)cells * sizeof(int64_t) + 8);
    if (!fill) return -1;
    memcpy(fill, cstart, (size_t)cells * sizeof(int64_t));
    for (int32_t i = 0; i < n; ++i) order[fill[cid[i]]++] = i;
    free(fill);
  }
  int64_t cap = (int64_t)(n * (k + 8.0)) + 64, cnt = 0;
  int32_t* us = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  int32_t* vs = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  if (!us || !vs) return -1;
  double r2 = r * r;
  for (int32_t i = 0; i < n; ++i) {
    int32_t cx = cid[i] % g, cy = cid[i] / g;
    for (int32_t dy = -1; dy <= 1; ++dy)
      for (int32_t dx = -1; dx <= 1; ++dx) {
        int32_t qx = cx + dx, qy = cy + dy;
        if (qx < 0 || qy < 0 || qx >= g || qy >= g) continue;
        int64_t c = (int64_t)qy * g + qx;
        for (int64_t t = cstart[c]; t < cstart[c + 1]; ++t) {
          int32_t j = order[t];
          if (j <= i) continue;
          double ddx = x[i] - x[j], ddy = y[i] - y[j];
          if (ddx * ddx + ddy * ddy < r2) {
            if (cnt >= cap) {
              cap = cap * 2;
              us = (int32_t*)realloc(us, (size_t)cap * sizeof(int32_t));
              vs = (int32_t*)realloc(vs, (size_t)cap * sizeof(int32_t));
              if (!us || !vs) return -1;
            }
            us[cnt] = i;
            vs[cnt] = j;
            ++cnt;
          }
        }
      }
  }
  free(x);
  free(y);
  free(cstart);
  free(cid);
  free(order);
  int rc = pairs_to_csr(n, cnt, us, vs, NULL, off, adj);
  free(us);
  free(vs);
  return rc;
}

/* --------------------------------------------------------------- batch */

/*
 * A packed batch of `ngraphs` independent graphs.  Graph g has n_g uniform
 * in [nmin, nmax] and a family uniform over {ER, R-MAT, RGG}:
 *   ER:    mean degree k uniform in [kmin, kmax], p = min(1, k / (n - 1));
 *   R-MAT: edge factor uniform in [efmin, efmax], scale ceil(log2 n),
 *          endpoints >= n rejected, ids permuted;
 *   RGG:   mean degree k uniform in [kmin, kmax].
 * Layout: offsets of graph g (int32, local, n_g + 1 entries) start at
 * vtx_off[g]; its adjacency (local ids) starts at adj_off[g].  vtx_off has
 * ngraphs + 1 entries with vtx_off[g+1] - vtx_off[g] = n_g + 1; adj_off has
 * ngraphs + 1 entries with adj_off[g+1] - adj_off[g] = 2 m_g.  family[g]
 * receives 0 (ER), 1 (R-MAT) or 2 (RGG).
 */
int gg_batch(int32_t ngraphs, int32_t nmin, int32_t nmax, double kmin, double kmax, int32_t efmin,
             int32_t efmax, uint64_t seed, int64_t** vtx_off_out, int64_t** adj_off_out,
             int32_t** offsets_out, int32_t** adj_out, int32_t** family_out) {
  if (ngraphs < 0 || nmin < 1 || nmax < nmin) return -2;
  int64_t** goff = (int64_t**)calloc((size_t)(ngraphs > 0 ? ngraphs : 1), sizeof(int64_t*));
  int32_t** gadj = (int32_t**)calloc((size_t)(ngraphs > 0 ? ngraphs : 1), sizeof(int32_t*));
  int32_t* gn = (int32_t*)malloc((size_t)(ngraphs > 0 ? ngraphs : 1) * sizeof(int32_t));
  int32_t* fam = (int32_t*)malloc((size_t)(ngraphs > 0 ? ngraphs : 1) * sizeof(int32_t));
  int* rcs = (int*)calloc((size_t)(ngraphs > 0 ? ngraphs : 1), sizeof(int));
  if (!goff || !gadj || !gn || !fam || !rcs) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t g = 0; g < ngraphs; ++g) {
    uint64_t gs = mix64(seed ^ (0x5851f42d4c957f2dULL * (uint64_t)(g + 1)));
    int32_t n = nmin + (int32_t)below(rng3(gs, 9, 0), (uint64_t)(nmax - nmin + 1));
    int32_t f = (int32_t)below(rng3(gs, 9, 1), 3);
    gn[g] = n;
    fam[g] = f;
    double k = kmin + (kmax - kmin) * u01(rng3(gs, 9, 2));
    if (f == 0) {
      double p = (n > 1) ? k / (double)(n - 1) : 0.0;
      if (p > 1.0) p = 1.0;
      rcs[g] = gg_er(n, p, gs, &goff[g], &gadj[g]);
    } else if (f == 1) {
      int32_t ef = efmin + (int32_t)below(rng3(gs, 9, 3), (uint64_t)(efmax - efmin + 1));
      int32_t sc = 0;
      while (((int64_t)1 << sc) < n) ++sc;
      rcs[g] = gg_rmat(sc, n, (int64_t)ef * n, 0.57, 0.19, 0.19, 1, gs, &goff[g], &gadj[g]);
    } else {
      rcs[g] = gg_rgg(n, k, gs, &goff[g], &gadj[g]);
    }
  }
  int rc = 0;
  for (int32_t g = 0; g < ngraphs; ++g)
    if (rcs[g]) rc = rcs[g];
  int64_t* vtx_off = (int64_t*)malloc(((size_t)ngraphs + 1) * sizeof(int64_t));
  int64_t* adj_off = (int64_t*)malloc(((size_t)ngraphs + 1) * sizeof(int64_t));
  if (!vtx_off || !adj_off) rc = -1;
  int32_t* offsets = NULL;
  int32_t* adjp = NULL;
  if (!rc) {
    vtx_off[0] = 0;
    adj_off[0] = 0;
    for (int32_t g = 0; g < ngraphs; ++g) {
      vtx_off[g + 1] = vtx_off[g] + gn[g] + 1;
      adj_off[g + 1] = adj_off[g] + goff[g][gn[g]];
    }
    offsets = (int32_t*)malloc((size_t)(vtx_off[ngraphs] > 0 ? vtx_off[ngraphs] : 1) * sizeof(int32_t));
    adjp = (int32_t*)malloc((size_t)(adj_off[ngraphs] > 0 ? adj_off[ngraphs] : 1) * sizeof(int32_t));
    if (!offsets || !adjp) rc = -1;
  }
  if (!rc) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t g = 0; g < ngraphs; ++g) {
      for (int32_t i = 0; i <= gn[g]; ++i) offsets[vtx_off[g] + i] = (int32_t)goff[g][i];
      memcpy(adjp + adj_off[g], gadj[g], (size_t)goff[g][gn[g]] * sizeof(int32_t));
    }
  }
  for (int32_t g = 0; g < ngraphs; ++g) {
    free(goff[g]);
    free(gadj[g]);
  }
  free(goff);
  free(gadj);
  free(gn);
  free(rcs);
  if (rc) {
    free(vtx_off);
    free(adj_off);
    free(offsets);
    free(adjp);
    free(fam);
    return rc;
  }
  *vtx_off_out = vtx_off;
  *adj_off_out = adj_off;
  *offsets_out = offsets;
  *adj_out = adjp;
  *family_out = fam;
  return 0;
}
