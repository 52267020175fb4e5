"""CPU ORACLE -- test infrastructure only.

Pure-Python statements of what truss decomposition computes, for small graphs.
Edges are pairs (u, v) with u < v; the canonical order of the library's output is
the lexicographic order of these pairs (row-major upper triangle of the CSR).

* ``support_by_definition``: S(e, G) = number of triangles of G containing e
  (Background section).
* ``truss_by_definition``: H_k is the largest edge set in which every edge lies in at
  least k-2 triangles whose edges are all in H_k; tau(e) = max{k : e in H_k}
  (Background section: the k-truss definition and Cohen's deletion procedure,
  repeatedly removing edges in fewer than k-2 triangles).
* ``kcore_numbers``: vertex coreness by repeated removal of a minimum-degree vertex.
* ``hindex_estimates`` / ``hindex_truss``: the local iteration of Sariyuce et al.
  that the Background section cites as an alternative (each edge repeatedly
  takes the h-index of min(tau(f1), tau(f2)) over its triangles {e, f1, f2}, all
  edges at once per sweep); it converges to trussness - 2.  A second, independent
  oracle of the trussness, and the oracle of the GPU's sweeps.
"""
from __future__ import annotations

import heapq

import numpy as np


def canonical_edges(edges):
    """Sorted list of distinct (u, v), u < v, self-loops dropped."""
    s = set()
    for a, b in edges:
        a, b = int(a), int(b)
        if a == b:
            continue
        s.add((a, b) if a < b else (b, a))
    return sorted(s)


def edges_from_csr(g):
    """Canonical edge list of a CSR graph (pure Python)."""
    out = []
    for u in range(g.n):
        for j in range(int(g.offsets[u]), int(g.offsets[u + 1])):
            v = int(g.adj[j])
            if v > u:
                out.append((u, v))
    return out


def _adjacency(edges):
    adj = {}
    for u, v in edges:
        adj.setdefault(u, set()).add(v)
        adj.setdefault(v, set()).add(u)
    return adj


def support_by_definition(edges):
    """{(u, v): number of triangles containing (u, v)}."""
    adj = _adjacency(edges)
    return {(u, v): len(adj[u] & adj[v]) for (u, v) in edges}


def truss_by_definition(edges):
    """{(u, v): trussness}, by computing H_3, H_4, ... with simultaneous deletion rounds."""
    E = canonical_edges(edges)
    tau = {e: 2 for e in E}  # H_2 = E
    H = set(E)
    k = 2
    while H:
        k += 1
        # H_k is the largest subset of H_{k-1} closed under "support inside it >= k-2"
        while True:
            adj = _adjacency(H)
            drop = [e for e in H if len(adj[e[0]] & adj[e[1]]) < k - 2]
            if not drop:
                break
            H.difference_update(drop)
        for e in H:
            tau[e] = k
    return tau


def kcore_numbers(n, edges):
    """Coreness of every vertex 0..n-1 (heap-based minimum-degree peeling)."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    deg = [len(a) for a in adj]
    heap = [(deg[v], v) for v in range(n)]
    heapq.heapify(heap)
    removed = [False] * n
    core = [0] * n
    k = 0
    while heap:
        d, v = heapq.heappop(heap)
        if removed[v] or d != deg[v]:
            continue
        k = max(k, d)
        core[v] = k
        removed[v] = True
        for w in adj[v]:
            if not removed[w]:
                deg[w] -= 1
                heapq.heappush(heap, (deg[w], w))
    return np.array(core, dtype=np.int64)


def triangles_by_edge_ids(edges):
    """(T, 3) array of edge-index triples, one row per triangle (edges given in canonical order)."""
    E = canonical_edges(edges)
    index = {e: i for i, e in enumerate(E)}
    adj = _adjacency(E)
    tris = []
    for (u, v) in E:
        for w in adj[u] & adj[v]:
            if w > v:  # u < v < w: each triangle once
                tris.append((index[(u, v)], index[(u, w)], index[(v, w)]))
    return np.array(tris, dtype=np.int64).reshape(-1, 3)


def hindex_estimates(edges, sweeps=None):
    """Estimates of the local h-index iteration after `sweeps` sweeps (None: until none
    changes), in canonical edge order, and the number of sweeps that changed an edge.

    Sweep 0 is the support; every sweep gives each edge, all at once, the h-index of
    min(estimate(f1), estimate(f2)) over its triangles {e, f1, f2} under the previous
    sweep's estimates.  The fixed point is trussness - 2.
    """
    E = canonical_edges(edges)
    m = len(E)
    T = triangles_by_edge_ids(E)
    est = np.bincount(T.ravel(), minlength=m).astype(np.int64) if len(T) else np.zeros(m, np.int64)
    if len(T) == 0:
        return est, 0
    # every triangle gives each of its edges the value min(est of the other two)
    owner = np.concatenate([T[:, 0], T[:, 1], T[:, 2]])
    o1 = np.concatenate([T[:, 1], T[:, 0], T[:, 0]])
    o2 = np.concatenate([T[:, 2], T[:, 2], T[:, 1]])
    done = 0
    while sweeps is None or done < sweeps:
        val = np.minimum(est[o1], est[o2])
        order = np.lexsort((-val, owner))  # by owner, then value descending
        ow, vv = owner[order], val[order]
        starts = np.flatnonzero(np.r_[True, ow[1:] != ow[:-1]])
        rank = np.arange(len(ow)) - np.repeat(starts, np.diff(np.r_[starts, len(ow)]))
        cand = np.minimum(rank + 1, vv)
        h = np.zeros(m, np.int64)
        h[ow[starts]] = np.maximum.reduceat(cand, starts)
        if np.array_equal(h, est):
            break
        est = h
        done += 1
        if done > 10_000:
            raise RuntimeError("h-index iteration did not converge")
    return est, done


def hindex_truss(edges, max_iter=10_000):
    """Trussness by the local h-index iteration, as an array in canonical edge order."""
    est, _ = hindex_estimates(edges)
    return est + 2
