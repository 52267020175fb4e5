"""Pins for the oracle's sweeps of the local h-index iteration (oracle/definition.py,
hindex_estimates): sweep 0 is the support by definition, one sweep by brute force
(plain loops, h-index by sorting), closed forms (cliques need no sweep, two triangles
sharing an edge need one), and on random graphs at every sweep the invariants that
hold at any size: estimates never grow, never fall below trussness - 2 (trussness by
the deletion definition), and stop exactly there."""
import itertools
import random

import numpy as np
import pytest

from oracle import definition as D


def sweep_by_brute_force(edges, est):
    E = D.canonical_edges(edges)
    index = {e: i for i, e in enumerate(E)}
    adj = {}
    for u, v in E:
        adj.setdefault(u, set()).add(v)
        adj.setdefault(v, set()).add(u)
    out = []
    for u, v in E:
        vals = sorted((min(est[index[tuple(sorted((u, w)))]], est[index[tuple(sorted((v, w)))]])
                       for w in adj[u] & adj[v]), reverse=True)
        h = 0
        for i, x in enumerate(vals):  # h-index: the largest h with h values >= h
            if x >= i + 1:
                h = i + 1
        out.append(h)
    return np.array(out, np.int64)


def random_graph(seed, nmax=40):
    rng = random.Random(seed)
    n = rng.randint(3, nmax)
    p = rng.uniform(0.05, 0.5)
    edges = {(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p}
    for _ in range(rng.randint(0, 2)):
        vs = sorted(rng.sample(range(n), min(n, rng.randint(3, 8))))
        edges |= set(itertools.combinations(vs, 2))
    return sorted(edges)


def test_closed_forms():
    for n in (3, 4, 7):
        est, sweeps = D.hindex_estimates(list(itertools.combinations(range(n), 2)))
        assert est.tolist() == [n - 2] * (n * (n - 1) // 2) and sweeps == 0
    diamond = [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3)]  # two triangles sharing (0, 1)
    est0, _ = D.hindex_estimates(diamond, sweeps=0)
    assert est0.tolist() == [2, 1, 1, 1, 1]  # canonical order: 01 02 03 12 13
    est, sweeps = D.hindex_estimates(diamond)
    assert est.tolist() == [1] * 5 and sweeps == 1
    est, sweeps = D.hindex_estimates([(0, 1), (1, 2), (2, 3)])  # no triangle
    assert est.tolist() == [0, 0, 0] and sweeps == 0


@pytest.mark.parametrize("seed", range(25))
def test_sweeps_against_definitions(seed):
    edges = random_graph(seed)
    E = D.canonical_edges(edges)
    est0, _ = D.hindex_estimates(edges, sweeps=0)
    sup = D.support_by_definition(edges)
    assert np.array_equal(est0, [sup[e] for e in E])
    tau = D.truss_by_definition(edges)
    floor = np.array([tau[e] for e in E], np.int64) - 2
    prev = est0
    k = 0
    while True:
        k += 1
        est, done = D.hindex_estimates(edges, sweeps=k)
        want = sweep_by_brute_force(edges, prev)
        if done < k:  # converged before sweep k: the brute-force sweep changes nothing
            assert np.array_equal(want, prev) and np.array_equal(est, prev)
            break
        assert np.array_equal(est, want)
        assert np.all(est <= prev) and np.all(est >= floor)
        prev = est
    assert np.array_equal(prev, floor)
