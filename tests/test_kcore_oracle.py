"""Pins for the oracle's core numbers (oracle/definition.py, kcore_numbers, and the
C bucket order behind oracle.kcore): the
k-core definition by brute force (repeated deletion of vertices of degree < k; the
core number of v is the largest k whose k-core holds v) on every graph with 5
vertices and on random graphs, and closed forms (isolated vertices, paths, stars,
trees, cycles, cliques, complete bipartite graphs, grids, disjoint unions)."""
import itertools
import random

import numpy as np
import pytest

from oracle import definition as D


def cores_by_definition(n, edges):
    adj = [set() for _ in range(n)]
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    core = [0] * n
    k = 1
    alive = set(range(n))
    while alive:
        changed = True
        while changed:  # the k-core: delete vertices of degree < k until none is left
            changed = False
            for v in list(alive):
                if len(adj[v] & alive) < k:
                    alive.discard(v)
                    changed = True
        for v in alive:
            core[v] = k
        k += 1
    return np.array(core, np.int64)


def test_every_graph_on_five_vertices():
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        edges = [p for i, p in enumerate(pairs) if mask >> i & 1]
        assert np.array_equal(D.kcore_numbers(5, edges), cores_by_definition(5, edges)), edges


@pytest.mark.parametrize("seed", range(30))
def test_random_graphs(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 60)
    p = rng.uniform(0.0, 0.4)
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    assert np.array_equal(D.kcore_numbers(n, edges), cores_by_definition(n, edges))


def test_closed_forms():
    assert D.kcore_numbers(4, []).tolist() == [0, 0, 0, 0]
    assert D.kcore_numbers(6, [(i, i + 1) for i in range(5)]).tolist() == [1] * 6  # path
    assert D.kcore_numbers(7, [(0, i) for i in range(1, 7)]).tolist() == [1] * 7  # star
    assert D.kcore_numbers(8, [(i, i // 2) for i in range(1, 8)]).tolist() == [1] * 8  # tree
    assert D.kcore_numbers(9, [(i, (i + 1) % 9) for i in range(9)]).tolist() == [2] * 9  # cycle
    for n in (2, 3, 7, 12):
        assert D.kcore_numbers(n, list(itertools.combinations(range(n), 2))).tolist() == [n - 1] * n
    a, b = 3, 6  # K_{3,6}: every vertex in the 3-core, none in a 4-core
    kab = [(i, a + j) for i in range(a) for j in range(b)]
    assert D.kcore_numbers(a + b, kab).tolist() == [3] * (a + b)
    grid = [(r * 5 + c, r * 5 + c + 1) for r in range(5) for c in range(4)] + \
           [(r * 5 + c, (r + 1) * 5 + c) for r in range(4) for c in range(5)]
    assert D.kcore_numbers(25, grid).tolist() == [2] * 25
    # K5 and a triangle joined by a pendant path: 4, 2 and 1
    edges = list(itertools.combinations(range(5), 2)) + [(5, 6), (6, 7), (5, 7), (4, 8), (8, 5)]
    assert D.kcore_numbers(9, edges).tolist() == [4, 4, 4, 4, 4, 2, 2, 2, 2]


@pytest.mark.parametrize("seed", range(25))
def test_bucket_order_in_c_matches_the_definition(seed):
    import graphgen as gg
    import oracle

    rng = random.Random(1000 + seed)
    n = rng.randint(1, 80)
    p = rng.uniform(0.0, 0.3)
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    for _ in range(rng.randint(0, 2)):  # planted cliques give deeper cores
        vs = sorted(rng.sample(range(n), min(n, rng.randint(3, 10))))
        edges += list(itertools.combinations(vs, 2))
    edges = sorted(set(edges))
    g = gg.from_edges(n, edges)
    assert np.array_equal(oracle.kcore(g), cores_by_definition(n, edges))


def test_bucket_order_on_a_medium_graph():
    import graphgen as gg
    import oracle

    g = gg.workload("rmat12", seed=4)
    edges = [tuple(map(int, p)) for p in oracle.edge_list(g)]
    assert np.array_equal(oracle.kcore(g), D.kcore_numbers(g.n, edges))


@pytest.mark.parametrize("seed", range(10))
def test_trussness_within_the_core_numbers(seed):
    # a k-truss lies in the (k-1)-core: every edge's trussness is at most one more than
    # the smaller core number of its endpoints (two oracles, one relation)
    import graphgen as gg
    import oracle

    rng = random.Random(2000 + seed)
    n = rng.randint(3, 120)
    p = rng.uniform(0.02, 0.3)
    edges = {(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p}
    for _ in range(rng.randint(0, 3)):
        vs = sorted(rng.sample(range(n), min(n, rng.randint(3, 12))))
        edges |= set(itertools.combinations(vs, 2))
    g = gg.from_edges(n, sorted(edges)) if seed else gg.workload("rmat12", seed=3)
    core = oracle.kcore(g)
    tau = oracle.truss(g)
    el = oracle.edge_list(g)
    if len(el):
        assert np.all(tau <= np.minimum(core[el[:, 0]], core[el[:, 1]]) + 1)
