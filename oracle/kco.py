"""CPU ORACLE (test infrastructure): vertex reordering by increasing core number (KCO).

Performance Results section, the study of support computation (Table 2): before support,
every graph is relabelled so that vertex ids increase with the core number, which
cuts the oriented triangle-counting work sum_v d+(v)^2 on skewed graphs.  The
trussness of an edge does not depend on the labels, so the decomposition of the
relabelled graph, mapped back edge by edge, is the decomposition of the input.

* ``order(core)``: new id of every vertex and the vertex at every new id.  The
  paper fixes increasing core number; ties go by old id (our reading, which makes
  the order unique).
* ``relabel(offsets, adj, new_id)``: the CSR of the relabelled graph, rows sorted.
* ``map_back(el, new_id, offsets2, adj2, tau2)``: trussness per edge of the input
  (edge list ``el`` in its canonical order) from the trussness of the relabelled
  graph (canonical edge ids of ``offsets2, adj2``).
* ``wplus(offsets, adj)``: the work estimate sum_v d+(v)^2 with every edge oriented
  from the smaller id to the larger (Table 2's ordering-dependent estimate).
"""
from __future__ import annotations

import numpy as np


def order(core):
    """(new_id, order): vertices sorted by (core number, old id)."""
    core = np.asarray(core, np.int64)
    n = len(core)
    by = np.lexsort((np.arange(n), core))  # last key first: core, then id
    new_id = np.empty(n, np.int64)
    new_id[by] = np.arange(n)
    return new_id.astype(np.int32), by.astype(np.int32)


def relabel(offsets, adj, new_id):
    """(offsets2, adj2): vertex v becomes new_id[v]; every row sorted by the new ids."""
    offsets = np.asarray(offsets, np.int64)
    adj = np.asarray(adj, np.int64)
    new_id = np.asarray(new_id, np.int64)
    n = len(offsets) - 1
    src = np.repeat(np.arange(n), np.diff(offsets))
    a, b = new_id[src], new_id[adj]
    p = np.lexsort((b, a))
    off2 = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(a, minlength=n), out=off2[1:])
    return off2, b[p].astype(np.int32)


def canonical_pairs(offsets, adj):
    """(u, v) with u < v for every edge, in canonical (row-major) edge-id order."""
    offsets = np.asarray(offsets, np.int64)
    adj = np.asarray(adj, np.int64)
    n = len(offsets) - 1
    src = np.repeat(np.arange(n), np.diff(offsets))
    up = adj > src
    return np.stack([src[up], adj[up]], axis=1)


def map_back(el, new_id, offsets2, adj2, tau2):
    """Trussness of every input edge: that of its image in the relabelled graph."""
    el = np.asarray(el, np.int64).reshape(-1, 2)
    new_id = np.asarray(new_id, np.int64)
    n = len(new_id)
    pairs = canonical_pairs(offsets2, adj2)
    keys = pairs[:, 0] * n + pairs[:, 1]  # increasing: row-major order
    a, b = new_id[el[:, 0]], new_id[el[:, 1]]
    want = np.minimum(a, b) * n + np.maximum(a, b)
    idx = np.searchsorted(keys, want)
    if len(want) and (idx.max(initial=0) >= len(keys) or not np.array_equal(keys[idx], want)):
        raise ValueError("an input edge has no image in the relabelled graph")
    return np.asarray(tau2)[idx].astype(np.int32)


def wplus(offsets, adj):
    """sum_v d+(v)^2 with d+(v) = number of neighbours of larger id."""
    pairs = canonical_pairs(offsets, adj)
    n = len(offsets) - 1
    dplus = np.bincount(pairs[:, 0], minlength=n).astype(np.int64)
    return int((dplus * dplus).sum())
