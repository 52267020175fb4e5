"""CPU model of the degree-order relabelling inside truss_decompose (csrc/relabel.hip):
new ids by a stable sort of the degrees, the relabelled CSR with sorted rows, and the
map back in input edge order through the relabelled row of the lower-degree endpoint.
Also the property the support walk relies on for a relabelled graph: with ids in
(degree, id) order, the oriented CSR is the upper half of every row and its slot k
holds canonical edge k.  Trussness does not depend on the labels (Background section),
so the oracle's trussness of the relabelled graph, mapped back, is the oracle's
trussness of the input."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle


def relabel(g):
    deg = np.diff(g.offsets)
    order = np.argsort(deg, kind="stable").astype(np.int64)  # new id -> old id
    new_id = np.empty(g.n, np.int64)
    new_id[order] = np.arange(g.n)
    rows = []
    for y in range(g.n):
        u = order[y]
        rows.append(np.sort(new_id[g.adj[g.offsets[u]:g.offsets[u + 1]]]))
    off2 = np.zeros(g.n + 1, np.int64)
    off2[1:] = np.cumsum([len(r) for r in rows])
    adj2 = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return new_id, order, gg.Graph(n=g.n, offsets=off2, adj=adj2, name=g.name + "-relabelled")


def canonical_ids(off, adj):
    """Edge id of every slot: rank of (min, max) among the edges in row-major order."""
    n = len(off) - 1
    up = np.array([np.count_nonzero(adj[off[u]:off[u + 1]] > u) for u in range(n)], np.int64)
    eb = np.zeros(n + 1, np.int64)
    eb[1:] = np.cumsum(up)
    eid = np.empty(len(adj), np.int64)
    for u in range(n):
        row = adj[off[u]:off[u + 1]]
        lo = int(np.searchsorted(row, u))
        for k, v in enumerate(row):
            if v > u:
                eid[off[u] + k] = eb[u] + (k - lo)
            else:
                r = adj[off[v]:off[v + 1]]
                eid[off[u] + k] = eb[v] + int(np.searchsorted(r, u)) - int(np.searchsorted(r, v))
    return eid, eb


def graphs():
    yield gg.rmat(9, 8, seed=3)
    yield gg.er(300, mean_degree=7.0, seed=2)
    yield gg.chunglu(1 << 9, 2.1, 3.0e3, draws=2_500, ncliques=2, cmin=5, cmax=12, seed=4)
    yield gg.from_edges(12, itertools.combinations(range(12), 2))
    yield gg.from_edges(30, [(3, 7), (7, 9), (3, 9), (20, 21)])


@pytest.mark.parametrize("g", list(graphs()), ids=lambda g: g.name)
def test_ids_follow_the_rank_after_relabelling(g):
    _, _, h = relabel(g)
    deg = np.diff(h.offsets)
    assert np.all(np.diff(deg) >= 0)  # degrees never fall with the id
    eid, _ = canonical_ids(h.offsets, h.adj)
    k = 0
    for u in range(h.n):
        row = h.adj[h.offsets[u]:h.offsets[u + 1]]
        for j, v in enumerate(row):
            above = (deg[v], v) > (deg[u], u)  # the (degree, id) rank orientation
            assert above == (v > u)
            if above:  # oriented slot k: the next upper entry in row-major order
                assert eid[h.offsets[u] + j] == k
                k += 1
    assert k == g.m


@pytest.mark.parametrize("g", list(graphs()), ids=lambda g: g.name)
def test_map_back_gives_the_input_trussness(g):
    new_id, order, h = relabel(g)
    assert h.m == g.m and sorted(map(tuple, oracle.edge_list(h))) == sorted(
        tuple(sorted((int(new_id[a]), int(new_id[b])))) for a, b in oracle.edge_list(g))
    tau2 = oracle.truss(h)
    eid2, _ = canonical_ids(h.offsets, h.adj)
    # input side: first slot above x and first edge id of every row
    us = np.array([g.offsets[x] + np.searchsorted(g.adj[g.offsets[x]:g.offsets[x + 1]], x + 1)
                   for x in range(g.n)], np.int64)
    eb = np.zeros(g.n + 1, np.int64)
    eb[1:] = np.cumsum(g.offsets[1:] - us)
    out = np.full(g.m, -1, np.int64)
    for x in range(g.n):
        for j in range(us[x], g.offsets[x + 1]):
            y = int(g.adj[j])
            e = eb[x] + (j - us[x])
            a, b = int(new_id[x]), int(new_id[y])
            lo, hi = min(a, b), max(a, b)
            row = h.adj[h.offsets[lo]:h.offsets[lo + 1]]
            q = int(np.searchsorted(row, hi))
            assert q < len(row) and row[q] == hi
            out[e] = tau2[eid2[h.offsets[lo] + q]]
    assert np.all(out >= 0)
    assert np.array_equal(out, oracle.truss(g))
