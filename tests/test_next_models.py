"""Step-by-step models of the concurrency and search arguments behind the core-number and
h-index kernels, checked on the CPU against the oracle.

* Core-number rounds: every frontier lane reads its neighbour's degree, subtracts one
  atomically if it is above the level, keeps the neighbour if the old value was k + 1
  and undoes the subtraction if it was <= k.  The lanes' steps interleave at random;
  the model also drops the "not yet finished" test, as the kernel does, since a
  finished vertex sits at or below the level.  Result: the oracle's core numbers.
* The h-index search: 64 thresholds spread over [lo, hi] per pass, keeping the part
  where "count >= threshold" turns false, equals the h-index (capped at the old value).
* Active edges: a sweep that recomputes only the edges with a triangle neighbour that
  changed in the previous sweep equals the full synchronous sweep, sweep by sweep.
"""
import itertools
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import definition as D


def kcore_model(n, adj, rng):
    """Core numbers by level-synchronous rounds whose atomic steps interleave at random."""
    deg = [len(a) for a in adj]
    core = [-1] * n
    alive = set(range(n))
    k = 0
    while alive:
        frontier = [v for v in alive if deg[v] == k]
        if not frontier:
            k = min(deg[v] for v in alive)  # skip to the smallest degree left
            continue
        while frontier:
            for v in frontier:
                core[v] = k
                alive.discard(v)
            # one lane per (frontier vertex, neighbour): read -> subtract -> maybe undo
            lanes = [[w, "read", None] for u in frontier for w in adj[u]]
            nxt = []
            while lanes:
                i = rng.randrange(len(lanes))
                w, step, old = lanes[i]
                if step == "read":
                    if deg[w] > k:  # the only test: no "finished" flag
                        lanes[i][1] = "sub"
                    else:
                        lanes.pop(i)
                elif step == "sub":
                    old = deg[w]
                    deg[w] -= 1
                    if old == k + 1:
                        nxt.append(w)
                        lanes.pop(i)
                    elif old <= k:
                        lanes[i][1] = "undo"
                    else:
                        lanes.pop(i)
                else:  # undo
                    deg[w] += 1
                    lanes.pop(i)
            assert all(deg[v] >= k for v in alive)  # never below the level between rounds
            frontier = nxt
        k += 1
    return np.array(core, np.int64)


def adjacency(g):
    return [g.adj[g.offsets[u]:g.offsets[u + 1]].tolist() for u in range(g.n)]


@pytest.mark.parametrize("seed", range(12))
def test_kcore_rounds_under_random_interleavings(seed):
    rng = random.Random(seed)
    n = rng.randint(2, 60)
    p = rng.uniform(0.05, 0.4)
    edges = {(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p}
    for _ in range(rng.randint(0, 2)):
        vs = sorted(rng.sample(range(n), min(n, rng.randint(3, 9))))
        edges |= set(itertools.combinations(vs, 2))
    g = gg.from_edges(n, sorted(edges))
    want = oracle.kcore(g)
    for trial in range(5):
        assert np.array_equal(kcore_model(n, adjacency(g), random.Random(seed * 100 + trial)), want)


def hindex_search(values, old, lanes=64):
    """The kernel's bisection: the h-index of `values`, searched in [0, old]."""
    lo, hi = 0, old
    while lo < hi:
        span = hi - lo
        T = [lo + ((t + 1) * span + lanes - 1) // lanes for t in range(lanes)]
        ok = [sum(1 for x in values if x >= T[t]) >= T[t] for t in range(lanes)]
        q = sum(ok)
        assert ok == [True] * q + [False] * (lanes - q)  # a prefix of the lanes
        if q == 0:
            hi = T[0] - 1
        else:
            lo = T[q - 1]
            if q < lanes:
                hi = T[q] - 1
    return lo


def h_index(values):
    s = sorted(values, reverse=True)
    return max([0] + [i + 1 for i, x in enumerate(s) if x >= i + 1])


@pytest.mark.parametrize("seed", range(40))
def test_threshold_search_is_the_h_index(seed):
    rng = random.Random(seed)
    size = rng.choice([0, 1, 5, 63, 64, 65, 300, 5000])
    top = rng.choice([1, 10, 100, 10_000])
    values = [rng.randint(0, top) for _ in range(size)]
    h = h_index(values)
    for old in {0, 1, h, h + 1, max(h - 1, 0), h + 70, 5000}:
        assert hindex_search(values, old) == min(h, old)


def sweeps_with_active_edges(edges):
    """The iteration with the kernel's active-edge tracking; returns the estimates per sweep."""
    E = D.canonical_edges(edges)
    index = {e: i for i, e in enumerate(E)}
    adj = {}
    for u, v in E:
        adj.setdefault(u, set()).add(v)
        adj.setdefault(v, set()).add(u)
    tri = [[(index[tuple(sorted((u, w)))], index[tuple(sorted((v, w)))]) for w in adj[u] & adj[v]]
           for (u, v) in E]
    est = [len(t) for t in tri]
    act = [True] * len(E)
    out = [list(est)]
    while True:
        nxt, act_next, changed = list(est), [False] * len(E), 0
        for e in range(len(E)):
            if not act[e] or est[e] == 0:
                continue
            h = hindex_search([min(est[a], est[b]) for a, b in tri[e]], est[e])
            nxt[e] = h
            if h != est[e]:
                changed += 1
                for a, b in tri[e]:
                    act_next[a] = act_next[b] = True
        if changed == 0:
            return out
        est, act = nxt, act_next
        out.append(list(est))


@pytest.mark.parametrize("seed", range(15))
def test_active_edges_give_the_synchronous_sweeps(seed):
    rng = random.Random(500 + seed)
    n = rng.randint(4, 40)
    p = rng.uniform(0.1, 0.5)
    edges = sorted({(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p})
    got = sweeps_with_active_edges(edges)
    for k, est in enumerate(got):
        want, done = D.hindex_estimates(edges, sweeps=k)
        assert done == k and np.array_equal(np.array(est, np.int64), want), k
    assert D.hindex_estimates(edges)[1] == len(got) - 1
