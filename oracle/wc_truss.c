/*
 * CPU ORACLE -- test infrastructure only.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load this.  It shares no code with the
 * GPU library.
 *
 * Serial truss decomposition in the style of Wang and Cheng (the serial
 * algorithm of the paper's Background section, Algorithm 1), plain and
 * unoptimised:
 *   1. edge ids: edge e = rank of (u, v), u < v, in row-major order of the
 *      input CSR (every edge once, from its smaller endpoint);
 *   2. support S[e] = |N(u) ∩ N(v)| by a sorted merge of the two rows (the
 *      definition of support in the Background section);
 *   3. a linear-time bin sort of the edges by support, with the constant-time
 *      "move to the front of its bin" reordering of Batagelj and Zaversnik;
 *   4. repeatedly take the edge e = (u, v) of lowest support k, visit every
 *      w in the shorter of N(u), N(v), and if both other edges of the
 *      triangle {u, v, w} are still present, lower the support of each one
 *      that is above k by one; then delete e; its trussness is k + 2.
 * The paper's hash table of vertex pairs is replaced by a binary search in
 * the sorted row (both rows are sorted), and both other edges must still be
 * present (the paper's listing tests only one of them; an edge already
 * deleted no longer closes a triangle).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ENOMEM -1
#define ORC_EINPUT -2

/* Position of x in the sorted slice a[lo, hi), or -1. */
static int64_t find_slot(const int32_t* a, int64_t lo, int64_t hi, int32_t x) {
  const int64_t end = hi;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < end && a[lo] == x) ? lo : -1;
}

/*
 * Checks the CSR: offsets start at 0 and do not decrease, ids are in range,
 * rows are strictly ascending (sorted, no duplicates), no self-loops, every
 * (u, v) has its mirror (v, u).  Returns ORC_OK or ORC_EINPUT.
 */
int oracle_check_csr(int32_t n, const int64_t* off, const int32_t* adj) {
  if (n < 0 || !off) return ORC_EINPUT;
  if (off[0] != 0) return ORC_EINPUT;
  for (int32_t u = 0; u < n; ++u)
    if (off[u + 1] < off[u]) return ORC_EINPUT;
  if (off[n] % 2 != 0) return ORC_EINPUT;
  for (int32_t u = 0; u < n; ++u) {
    for (int64_t j = off[u]; j < off[u + 1]; ++j) {
      int32_t v = adj[j];
      if (v < 0 || v >= n || v == u) return ORC_EINPUT;
      if (j > off[u] && adj[j - 1] >= v) return ORC_EINPUT;
    }
  }
  for (int32_t u = 0; u < n; ++u)
    for (int64_t j = off[u]; j < off[u + 1]; ++j) {
      int32_t v = adj[j];
      if (off[v + 1] == off[v] || find_slot(adj, off[v], off[v + 1], u) < 0) return ORC_EINPUT;
    }
  return ORC_OK;
}

/*
 * Edge ids.  el_u[e] < el_v[e] are the endpoints of edge e; slot_eid[j] is
 * the id of the edge at adjacency slot j (both directions).  Returns m or a
 * negative code.
 */
int64_t oracle_edge_ids(int32_t n, const int64_t* off, const int32_t* adj, int32_t* el_u, int32_t* el_v,
                        int32_t* slot_eid) {
  int64_t e = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int64_t j = off[u]; j < off[u + 1]; ++j)
      if (adj[j] > u) {
        if (el_u) el_u[e] = u;
        if (el_v) el_v[e] = adj[j];
        slot_eid[j] = (int32_t)e;
        ++e;
      }
  for (int32_t u = 0; u < n; ++u)
    for (int64_t j = off[u]; j < off[u + 1]; ++j) {
      int32_t v = adj[j];
      if (v < u) {
        int64_t k = find_slot(adj, off[v], off[v + 1], u);
        if (k < 0) return ORC_EINPUT;
        slot_eid[j] = slot_eid[k];
      }
    }
  return e;
}

/* Support of every edge: the number of common neighbours of its endpoints. */
static void support_by_merge(int64_t m, const int64_t* off, const int32_t* adj, const int32_t* el_u,
                             const int32_t* el_v, int32_t* S) {
  for (int64_t e = 0; e < m; ++e) {
    int64_t i = off[el_u[e]], ie = off[el_u[e] + 1];
    int64_t j = off[el_v[e]], je = off[el_v[e] + 1];
    int32_t c = 0;
    while (i < ie && j < je) {
      if (adj[i] < adj[j])
        ++i;
      else if (adj[i] > adj[j])
        ++j;
      else {
        ++c;
        ++i;
        ++j;
      }
    }
    S[e] = c;
  }
}

/* Support of every edge in canonical edge order.  Returns m or a negative code. */
int64_t oracle_support(int32_t n, const int64_t* off, const int32_t* adj, int32_t* S) {
  int rc = oracle_check_csr(n, off, adj);
  if (rc) return rc;
  int64_t two_m = off[n], m = two_m / 2;
  int32_t* el_u = (int32_t*)malloc((size_t)(m + 1) * sizeof(int32_t));
  int32_t* el_v = (int32_t*)malloc((size_t)(m + 1) * sizeof(int32_t));
  int32_t* eid = (int32_t*)malloc((size_t)(two_m + 1) * sizeof(int32_t));
  if (!el_u || !el_v || !eid) {
    free(el_u);
    free(el_v);
    free(eid);
    return ORC_ENOMEM;
  }
  int64_t mm = oracle_edge_ids(n, off, adj, el_u, el_v, eid);
  if (mm == m) support_by_merge(m, off, adj, el_u, el_v, S);
  free(el_u);
  free(el_v);
  free(eid);
  return mm;
}

/*
 * Trussness of every edge in canonical edge order (tau[e] >= 2).  If S0 is
 * non-NULL it receives the initial support; if rank is non-NULL, rank[e] is the
 * step at which edge e was removed (0 .. m-1, a peeling order).  Returns m or a
 * negative code.
 */
int64_t oracle_truss(int32_t n, const int64_t* off, const int32_t* adj, int32_t* tau, int32_t* S0,
                     int64_t* rank) {
  int rc = oracle_check_csr(n, off, adj);
  if (rc) return rc;
  int64_t two_m = off[n], m = two_m / 2;
  int32_t* el_u = (int32_t*)malloc((size_t)(m + 1) * sizeof(int32_t));
  int32_t* el_v = (int32_t*)malloc((size_t)(m + 1) * sizeof(int32_t));
  int32_t* eid = (int32_t*)malloc((size_t)(two_m + 1) * sizeof(int32_t));
  int32_t* S = (int32_t*)malloc((size_t)(m + 1) * sizeof(int32_t));
  int64_t* order = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
  int64_t* pos = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
  uint8_t* gone = (uint8_t*)calloc((size_t)(m + 1), 1);
  int64_t* bin = NULL;
  int64_t result = ORC_ENOMEM;
  if (!el_u || !el_v || !eid || !S || !order || !pos || !gone) goto out;
  if (oracle_edge_ids(n, off, adj, el_u, el_v, eid) != m) {
    result = ORC_EINPUT;
    goto out;
  }
  support_by_merge(m, off, adj, el_u, el_v, S);
  if (S0) memcpy(S0, S, (size_t)m * sizeof(int32_t));

  /* bin sort by support: bin[s] = index in `order` where support s starts */
  int32_t smax = 0;
  for (int64_t e = 0; e < m; ++e)
    if (S[e] > smax) smax = S[e];
  bin = (int64_t*)calloc((size_t)smax + 2, sizeof(int64_t));
  if (!bin) goto out;
  for (int64_t e = 0; e < m; ++e) bin[S[e] + 1]++;
  for (int32_t s = 0; s <= smax; ++s) bin[s + 1] += bin[s];
  {
    int64_t* fill = (int64_t*)malloc(((size_t)smax + 1) * sizeof(int64_t));
    if (!fill) goto out;
    memcpy(fill, bin, ((size_t)smax + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; ++e) {
      pos[e] = fill[S[e]]++;
      order[pos[e]] = e;
    }
    free(fill);
  }

  for (int64_t i = 0; i < m; ++i) {
    int64_t e = order[i];
    int32_t k = S[e];
    int32_t u = el_u[e], v = el_v[e];
    /* walk the shorter row, look the third vertex up in the other row */
    if (off[u + 1] - off[u] > off[v + 1] - off[v]) {
      int32_t t = u;
      u = v;
      v = t;
    }
    for (int64_t j = off[u]; j < off[u + 1]; ++j) {
      int32_t w = adj[j];
      if (w == v) continue;
      int64_t jv = find_slot(adj, off[v], off[v + 1], w);
      if (jv < 0) continue;
      int64_t f[2] = {eid[j], eid[jv]};
      if (gone[f[0]] || gone[f[1]]) continue;
      for (int t = 0; t < 2; ++t) {
        int64_t x = f[t];
        if (S[x] > k) {
          /* move x to the front of its bin, then shrink that bin by one */
          int32_t s = S[x];
          int64_t front = bin[s];
          int64_t y = order[front];
          if (y != x) {
            order[pos[x]] = y;
            pos[y] = pos[x];
            order[front] = x;
            pos[x] = front;
          }
          bin[s]++;
          S[x]--;
        }
      }
    }
    gone[e] = 1;
    tau[e] = k + 2;
    if (rank) rank[e] = i;
  }
  result = m;
out:
  free(el_u);
  free(el_v);
  free(eid);
  free(S);
  free(order);
  free(pos);
  free(gone);
  free(bin);
  return result;
}

/* Core numbers (k-core decomposition) by Batagelj and Zaversnik's bucket order:
 * vertices sorted by degree in bins; the vertex of least current degree is
 * removed, its core number is that degree, and every neighbour of larger degree
 * moves to the front of its bin and loses one.  Returns the largest core number,
 * or -1 on allocation failure. */
int64_t oracle_kcore(int32_t n, const int64_t* off, const int32_t* adj, int32_t* core) {
  if (n <= 0) return 0;
  int32_t md = 0;
  int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* vert = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!deg || !pos || !vert) {
    free(deg); free(pos); free(vert);
    return -1;
  }
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = (int32_t)(off[v + 1] - off[v]);
    if (deg[v] > md) md = deg[v];
  }
  int64_t* bin = (int64_t*)calloc((size_t)md + 2, sizeof(int64_t));
  if (!bin) {
    free(deg); free(pos); free(vert);
    return -1;
  }
  for (int32_t v = 0; v < n; ++v) bin[deg[v]] += 1;
  int64_t start = 0;
  for (int32_t d = 0; d <= md; ++d) {  /* bin[d] -> first position of degree d */
    const int64_t c = bin[d];
    bin[d] = start;
    start += c;
  }
  for (int32_t v = 0; v < n; ++v) {
    pos[v] = (int32_t)bin[deg[v]];
    vert[pos[v]] = v;
    bin[deg[v]] += 1;
  }
  for (int32_t d = md; d >= 1; --d) bin[d] = bin[d - 1];
  bin[0] = 0;
  int64_t kmax = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = vert[i];
    core[v] = deg[v];
    if (deg[v] > kmax) kmax = deg[v];
    for (int64_t j = off[v]; j < off[v + 1]; ++j) {
      const int32_t u = adj[j];
      if (deg[u] > deg[v]) {  /* u not yet removed: swap it to the front of its bin */
        const int32_t du = deg[u];
        const int32_t pu = pos[u];
        const int32_t pw = (int32_t)bin[du];
        const int32_t w = vert[pw];
        if (u != w) {
          pos[u] = pw;
          vert[pu] = w;
          pos[w] = pu;
          vert[pw] = u;
        }
        bin[du] += 1;
        deg[u] -= 1;
      }
    }
  }
  free(deg); free(pos); free(vert); free(bin);
  return kmax;
}

