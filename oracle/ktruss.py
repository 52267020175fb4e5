"""CPU ORACLE (test infrastructure): the maximal k-trusses of a graph, given its trussness.

Introduction and Background sections: a k-truss is a maximal connected subgraph in which every edge
lies in at least k - 2 triangles of the subgraph.  The edges of trussness >= k form
the largest subgraph with that triangle property (H_k), and every k-truss lies in
it, so the k-trusses are exactly the connected components of H_k (two edges of H_k
that share a vertex belong to the same k-truss).

Each k-truss is named by its smallest edge id, which makes the labelling unique:
``labels(n, el, tau, k)[e]`` is that id for an edge of trussness >= k and -1 for
every other edge.  Two implementations, kept independent so that one pins the other:
``labels`` uses scipy's connected components of the vertex graph of H_k as its one
library step, ``labels_bfs`` walks H_k edge by edge in plain Python (small graphs).
"""
from __future__ import annotations

from collections import defaultdict, deque

import numpy as np


def labels(n: int, el, tau, k: int):
    """Smallest edge id of the k-truss of every edge (-1 below k), and the k-truss count."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    el = np.asarray(el, np.int64).reshape(-1, 2)
    tau = np.asarray(tau, np.int64)
    m = len(tau)
    out = np.full(m, -1, np.int64)
    keep = np.flatnonzero(tau >= k)
    if len(keep) == 0:
        return out.astype(np.int32), 0
    u, v = el[keep, 0], el[keep, 1]
    a = coo_matrix((np.ones(len(keep), np.int8), (u, v)), shape=(n, n))
    _, comp = connected_components(a, directed=False)
    c = comp[u]  # component of every kept edge (both endpoints share it)
    first = np.full(comp.max() + 1, np.iinfo(np.int64).max, np.int64)
    np.minimum.at(first, c, keep)
    out[keep] = first[c]
    return out.astype(np.int32), int(len(np.unique(c)))


def labels_bfs(n: int, el, tau, k: int):
    """The same by breadth-first search over the edges of H_k (plain Python)."""
    el = [tuple(map(int, p)) for p in np.asarray(el).reshape(-1, 2)]
    tau = [int(t) for t in tau]
    at = defaultdict(list)  # vertex -> edges of H_k at it
    for e, (u, v) in enumerate(el):
        if tau[e] >= k:
            at[u].append(e)
            at[v].append(e)
    out = [-1] * len(el)
    count = 0
    for e0 in range(len(el)):
        if tau[e0] < k or out[e0] != -1:
            continue
        count += 1  # e0 is the smallest id of a new k-truss: ids are visited in order
        out[e0] = e0
        queue = deque([e0])
        while queue:
            e = queue.popleft()
            for x in el[e]:
                for f in at[x]:
                    if out[f] == -1:
                        out[f] = e0
                        queue.append(f)
    return np.asarray(out, np.int32), count
