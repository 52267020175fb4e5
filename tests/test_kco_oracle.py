"""Pins for the oracle's KCO reordering (oracle/kco.py): the order on graphs whose core
numbers are known in closed form, the order's defining properties on random core
vectors, the relabelled graph against the edge set by brute force, the trussness
mapped back against the trussness of the input (it does not depend on the labels),
and the work estimate sum_v d+(v)^2 in closed form and by brute force."""
import itertools
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import kco as K


def test_order_closed_form():
    # a path 0-1-2-3-4 (core 1), a K4 on 5..8 (core 3), a triangle on 9..11 (core 2),
    # an isolated vertex 12 (core 0)
    edges = [(i, i + 1) for i in range(4)] + list(itertools.combinations(range(5, 9), 2)) + \
        list(itertools.combinations(range(9, 12), 2))
    g = gg.from_edges(13, edges)
    core = oracle.kcore(g)
    assert core.tolist() == [1] * 5 + [3] * 4 + [2] * 3 + [0]
    new_id, by = K.order(core)
    assert by.tolist() == [12, 0, 1, 2, 3, 4, 9, 10, 11, 5, 6, 7, 8]
    assert new_id.tolist() == [1, 2, 3, 4, 5, 9, 10, 11, 12, 6, 7, 8, 0]


@pytest.mark.parametrize("seed", range(20))
def test_order_properties(seed):
    rng = random.Random(seed)
    n = rng.randint(0, 500)
    core = [rng.randint(0, rng.choice([0, 3, 300])) for _ in range(n)]
    new_id, by = K.order(core)
    assert sorted(by.tolist()) == list(range(n))  # a permutation ...
    assert all(new_id[by[i]] == i for i in range(n))  # ... and new_id is its inverse
    for i in range(n - 1):  # increasing core number, ties by increasing old id
        a, b = by[i], by[i + 1]
        assert core[a] < core[b] or (core[a] == core[b] and a < b)


def brute_relabel(n, edges, new_id):
    rows = [set() for _ in range(n)]
    for u, v in edges:
        rows[new_id[u]].add(new_id[v])
        rows[new_id[v]].add(new_id[u])
    return rows


@pytest.mark.parametrize("seed", range(15))
def test_relabel_by_brute_force(seed):
    rng = random.Random(100 + seed)
    n = rng.randint(1, 80)
    p = rng.uniform(0.0, 0.3)
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    g = gg.from_edges(n, edges)
    perm = list(range(n))
    rng.shuffle(perm)
    for new_id in (np.array(perm), K.order(oracle.kcore(g))[0]):
        off2, adj2 = K.relabel(g.offsets, g.adj, new_id)
        rows = brute_relabel(n, edges, new_id)
        for x in range(n):
            row = adj2[off2[x]:off2[x + 1]].tolist()
            assert row == sorted(rows[x]), x


def test_relabel_special_cases():
    g = gg.from_edges(6, [(i, i + 1) for i in range(5)])
    off, adj = K.relabel(g.offsets, g.adj, np.arange(6))  # identity: the same CSR
    assert np.array_equal(off, g.offsets) and np.array_equal(adj, g.adj)
    off, adj = K.relabel(g.offsets, g.adj, np.arange(6)[::-1].copy())  # reversal of a path
    assert np.array_equal(off, g.offsets) and np.array_equal(adj, g.adj)
    off, adj = K.relabel(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int64))
    assert off.tolist() == [0] and len(adj) == 0


def graphs():
    rng = random.Random(7)
    for i in range(6):
        n = rng.randint(5, 60)
        edges = {(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.2}
        vs = sorted(rng.sample(range(n), min(n, 8)))
        edges |= set(itertools.combinations(vs, 2))
        yield gg.from_edges(n, sorted(edges))
    yield gg.workload("rmat12", seed=2)


@pytest.mark.parametrize("g", list(graphs()))
def test_trussness_survives_the_relabelling(g):
    tau = oracle.truss(g)
    el = oracle.edge_list(g)
    rng = np.random.default_rng(3)
    for new_id in (K.order(oracle.kcore(g))[0], rng.permutation(g.n)):
        off2, adj2 = K.relabel(g.offsets, g.adj, new_id)
        g2 = gg.Graph(g.n, off2, adj2)
        assert np.array_equal(K.map_back(el, new_id, off2, adj2, oracle.truss(g2)), tau)


def test_map_back_identity_and_missing_edge():
    g = gg.from_edges(5, list(itertools.combinations(range(5), 2)))
    tau2 = np.arange(10, dtype=np.int32)
    el = oracle.edge_list(g)
    assert np.array_equal(K.map_back(el, np.arange(5), g.offsets, g.adj, tau2), tau2)
    h = gg.from_edges(5, [(0, 1)])
    with pytest.raises(ValueError):
        K.map_back(np.array([[0, 2]]), np.arange(5), h.offsets, h.adj, np.zeros(1, np.int32))


def test_wplus_closed_forms_and_brute_force():
    for n in (1, 2, 5, 9):
        g = gg.from_edges(n, list(itertools.combinations(range(n), 2)))
        assert K.wplus(g.offsets, g.adj) == (n - 1) * n * (2 * n - 1) // 6
    g = gg.from_edges(7, [(0, i) for i in range(1, 7)])  # star, centre smallest
    assert K.wplus(g.offsets, g.adj) == 36
    g = gg.from_edges(7, [(6, i) for i in range(6)])  # star, centre largest
    assert K.wplus(g.offsets, g.adj) == 6
    rng = random.Random(5)
    for _ in range(10):
        n = rng.randint(1, 40)
        edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < 0.3]
        g = gg.from_edges(n, edges)
        want = sum(sum(1 for (a, b) in edges if a == v) ** 2 for v in range(n))
        assert K.wplus(g.offsets, g.adj) == want


def test_kco_cuts_the_work_estimate_on_a_skewed_graph():
    # Table 2's effect on a skewed graph whose given labels are random (R-MAT ids are
    # permuted): increasing core order cuts sum d+^2 more than twofold
    g = gg.workload("rmat12", seed=1)
    new_id, _ = K.order(oracle.kcore(g))
    off2, adj2 = K.relabel(g.offsets, g.adj, new_id)
    assert K.wplus(off2, adj2) * 2 < K.wplus(g.offsets, g.adj)
