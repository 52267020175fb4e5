"""The certificate checks (oracle/certificate.py) used for full-size parity: pinned against
the oracle, the definition and closed forms, and shown to reject wrong answers."""
import itertools
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import certificate as C
from oracle import definition as D


def graphs():
    yield "K6", gg.from_edges(6, itertools.combinations(range(6), 2))
    yield "rmat11", gg.rmat(11, 16, seed=3)
    yield "er600", gg.er(600, mean_degree=12.0, seed=2)
    yield "chunglu", gg.chunglu(1 << 11, 2.1, 1.2e4, draws=11_000, ncliques=3, cmin=8, cmax=20, seed=5)
    yield "rgg", gg.rgg(800, 12.0, seed=4)


@pytest.mark.parametrize("name,g", list(graphs()))
def test_oracle_answer_and_order_pass(name, g):
    tau, rank = oracle.truss(g, with_rank=True)
    res = C.verify(g, tau, rank)
    assert res["ok"], (name, res["monotone"], res["lower_bound_fails"][:5], res["upper_bound_fails"][:5])


def test_brute_force_answers_pass():
    rng = random.Random(7)
    for _ in range(60):
        n = rng.randint(4, 12)
        p = rng.uniform(0.3, 0.9)
        E = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
        g = gg.from_edges(n, E)
        bf = D.truss_by_definition(D.edges_from_csr(g))
        tau = np.array([bf[e] for e in D.edges_from_csr(g)], np.int32)
        _, rank = oracle.truss(g, with_rank=True)
        assert C.verify(g, tau, rank)["ok"]


def test_closed_forms():
    for n in range(3, 9):  # K_n: n everywhere, in any removal order
        g = gg.from_edges(n, itertools.combinations(range(n), 2))
        rank = np.random.default_rng(n).permutation(g.m)
        assert C.verify(g, np.full(g.m, n, np.int32), rank)["ok"]
    # a tree (path): 2 everywhere
    g = gg.from_edges(8, [(i, i + 1) for i in range(7)])
    assert C.verify(g, np.full(g.m, 2, np.int32), np.arange(g.m))["ok"]


@pytest.mark.parametrize("name,g", list(graphs())[1:])
def test_wrong_answers_fail(name, g):
    tau, rank = oracle.truss(g, with_rank=True)
    rng = np.random.default_rng(11)
    for e in rng.choice(g.m, size=12, replace=False):
        for d in (+1, -1):
            bad = tau.copy()
            bad[e] += d
            if bad[e] < 2:
                continue
            assert not C.verify(g, bad, rank)["ok"], (name, int(e), d)


def test_reversed_order_fails():
    g = gg.rmat(11, 16, seed=3)
    tau, rank = oracle.truss(g, with_rank=True)
    assert not C.monotone_order(tau, g.m - 1 - rank)
    res = C.Certificate(g).check(tau, g.m - 1 - rank, np.arange(g.m))
    assert res["upper_bound_fails"]  # removing the dense core first leaves too many triangles


def test_sampling_covers_every_value():
    tau = np.array([2] * 50 + [3] * 5 + [7], np.int32)
    s = C.sample_edges(tau, n_uniform=3, per_value=2)
    assert set(tau[s]) == {2, 3, 7}
