"""Pins for the k-truss listing oracle (oracle/ktruss.py): the two independent
implementations agree, closed forms (cliques joined by a bridge, cliques sharing one
vertex, disjoint unions), and the definition of a k-truss (Background section) holds
for every component it returns: connected, every edge in >= k - 2 triangles of its
own component, and nothing of trussness >= k left out."""
import itertools
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import definition as D
from oracle import ktruss as KT


def graph(n, edges):
    return gg.from_edges(n, edges)


def clique(vs):
    return list(itertools.combinations(vs, 2))


def labelled(g, k):
    el = oracle.edge_list(g)
    tau = oracle.truss(g)
    return el, tau, KT.labels(g.n, el, tau, k)


def test_two_cliques_and_a_bridge():
    g = graph(10, clique(range(5)) + clique(range(5, 10)) + [(4, 5)])
    el = oracle.edge_list(g)
    bridge = [e for e, (u, v) in enumerate(el) if (u, v) == (4, 5)][0]
    for k in (3, 4, 5):
        (lab, cnt) = labelled(g, k)[2]
        assert cnt == 2 and lab[bridge] == -1
        left = [e for e, (u, v) in enumerate(el) if v < 5]
        right = [e for e, (u, v) in enumerate(el) if u >= 5]
        assert set(lab[left]) == {min(left)} and set(lab[right]) == {min(right)}
    lab, cnt = labelled(g, 2)[2]
    assert cnt == 1 and set(lab) == {0}
    lab, cnt = labelled(g, 6)[2]
    assert cnt == 0 and set(lab) == {-1}


def test_cliques_sharing_a_vertex_are_one_truss():
    # connected through the shared vertex, though no triangle spans both: one k-truss
    g = graph(7, clique(range(4)) + clique(range(3, 7)))
    lab, cnt = labelled(g, 4)[2]
    assert cnt == 1 and set(lab) == {0}


def test_disjoint_union_counts_components():
    edges = []
    for b in range(6):  # cliques of 3 .. 8 vertices, ten ids apart
        edges += clique(range(10 * b, 10 * b + 3 + b))
    g = graph(60, edges)
    for k, want in ((3, 6), (4, 5), (5, 4), (8, 1), (9, 0)):
        assert labelled(g, k)[2][1] == want


def random_graph(rng, n, p, planted=()):
    edges = {(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p}
    for vs in planted:
        edges |= set(clique(sorted(vs)))
    return graph(n, sorted(edges))


@pytest.mark.parametrize("seed", range(40))
def test_two_implementations_agree(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 40)
    planted = [rng.sample(range(n), min(n, rng.randint(3, 8))) for _ in range(rng.randint(0, 3))]
    g = random_graph(rng, n, rng.uniform(0.02, 0.3), planted)
    el = oracle.edge_list(g)
    tau = oracle.truss(g)
    tmax = int(tau.max()) if len(tau) else 2
    for k in range(2, tmax + 2):
        a = KT.labels(g.n, el, tau, k)
        b = KT.labels_bfs(g.n, el, tau, k)
        assert np.array_equal(a[0], b[0]) and a[1] == b[1]


@pytest.mark.parametrize("seed", range(15))
def test_components_are_k_trusses(seed):
    rng = random.Random(100 + seed)
    n = rng.randint(6, 24)
    planted = [rng.sample(range(n), rng.randint(4, min(n, 7))) for _ in range(2)]
    g = random_graph(rng, n, rng.uniform(0.1, 0.35), planted)
    el = oracle.edge_list(g)
    tau = oracle.truss(g)
    for k in range(3, int(tau.max()) + 1):
        lab, cnt = KT.labels(g.n, el, tau, k)
        assert np.array_equal(lab >= 0, tau >= k)  # every edge of trussness >= k, nothing else
        assert cnt == len(set(lab[lab >= 0]))
        for c in set(lab[lab >= 0]):
            comp = [tuple(el[e]) for e in np.flatnonzero(lab == c)]
            assert min(np.flatnonzero(lab == c)) == c
            sup = D.support_by_definition(comp)
            assert all(s >= k - 2 for s in sup.values())  # triangles inside the component
            verts = {x for p in comp for x in p}  # connected: one BFS reaches every vertex
            adj = {x: set() for x in verts}
            for u, v in comp:
                adj[u].add(v)
                adj[v].add(u)
            seen, stack = {comp[0][0]}, [comp[0][0]]
            while stack:
                for y in adj[stack.pop()]:
                    if y not in seen:
                        seen.add(y)
                        stack.append(y)
            assert seen == verts


def test_no_edges():
    lab, cnt = KT.labels(5, np.zeros((0, 2), np.int32), np.zeros(0, np.int32), 3)
    assert len(lab) == 0 and cnt == 0
