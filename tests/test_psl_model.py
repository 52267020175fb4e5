"""The concurrency rules of the level-synchronous peeling, checked on the CPU model.

* Fig. 3 worked example (PKT section): two frontier edges at support 2 share a
  triangle whose third edge has support 4; that edge ends at 3 whichever frontier
  edge owns the triangle.
* Per sub-level closed form: S_end[x] = max(l, S_start[x] - D[x]) and x joins the next
  frontier iff S_start[x] > l >= S_start[x] - D[x], D[x] = destroyed triangles of x.
* The full level-synchronous run equals the serial oracle, for the paper's
  lower-id ownership and for its higher-id alternative, under random interleavings
  with stale plain reads.
* Switching off the ownership rule or the restore step gives wrong answers.
"""
import os
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import definition as D
from oracle import psl_model as PM

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fig3():
    vals = {}
    for line in open(os.path.join(GOLDEN, "fig3_sublevel.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = int(v)
    return vals


@pytest.mark.parametrize("owner", ["lower", "higher"])
@pytest.mark.parametrize("ids", [(0, 1, 2), (1, 0, 2), (2, 1, 0), (0, 2, 1)])
def test_fig3_triangle_decremented_once(owner, ids):
    f = _fig3()
    # triangle u=0, v=1, w=2; assign the roles e1, e2, e3 to edge ids per `ids`
    E = [(0, 1), (0, 2), (1, 2)]
    e1, e2, e3 = ids
    for seed in range(25):
        S = [0, 0, 0]
        S[e1], S[e2], S[e3] = f["support_e1"], f["support_e2"], f["support_e3_before"]
        state = [PM.ALIVE] * 3
        state[e1] = state[e2] = PM.CURR
        nxt = PM.process_sublevel(E, S, state, [e1, e2], f["level"], random.Random(seed), owner=owner)
        assert S[e3] == f["support_e3_after"]
        assert nxt == []


def test_fig3_without_ownership_double_decrements():
    f = _fig3()
    E = [(0, 1), (0, 2), (1, 2)]
    seen = set()
    for seed in range(25):
        S = [f["support_e1"], f["support_e2"], f["support_e3_before"]]
        state = [PM.CURR, PM.CURR, PM.ALIVE]
        PM.process_sublevel(E, S, state, [0, 1], f["level"], random.Random(seed), owner="none",
                            stale_reads=False)
        seen.add(S[2])
    assert seen == {f["support_e3_after"] - 1}


def _random_graphs(count, seed):
    rng = random.Random(seed)
    for _ in range(count):
        n = rng.randint(4, 16)
        p = rng.uniform(0.3, 0.95)
        yield D.canonical_edges([(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p])


def test_sublevel_closed_form():
    for i, E in enumerate(_random_graphs(40, 1)):
        trace = []
        PM.pkt(E, seed=i, trace=trace)
        for l, S0, st0, curr, S1, nxt in trace:
            S_end, nxt_want = PM.sublevel_closed_form(E, S0, st0, curr, l)
            assert S1 == S_end
            assert set(nxt) == nxt_want
            assert len(nxt) == len(set(nxt))  # each edge joins the frontier once


@pytest.mark.parametrize("owner", ["lower", "higher"])
def test_model_matches_oracle(owner):
    for i, E in enumerate(_random_graphs(60, 2)):
        n = 1 + max((v for _, v in E), default=0)
        want = oracle.truss(gg.from_edges(n, E)).tolist()
        assert PM.pkt(E, seed=100 + i, owner=owner) == want


def test_model_on_dense_adversarial_graphs():
    # cliques minus matchings: many triangles with two frontier edges
    for n in (8, 10, 12):
        E = [(a, b) for a in range(n) for b in range(a + 1, n) if not (b == a + 1 and a % 2 == 0)]
        want = oracle.truss(gg.from_edges(n, E)).tolist()
        for seed in range(5):
            assert PM.pkt(E, seed=seed) == want


def test_rules_matter():
    wrong_owner = wrong_restore = 0
    for i, E in enumerate(_random_graphs(60, 3)):
        n = 1 + max((v for _, v in E), default=0)
        want = oracle.truss(gg.from_edges(n, E)).tolist()
        wrong_owner += PM.pkt(E, seed=i, owner="none") != want
        wrong_restore += PM.pkt(E, seed=i, restore=False) != want
    assert wrong_owner > 0 and wrong_restore > 0
