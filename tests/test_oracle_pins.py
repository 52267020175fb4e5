"""Pins for the CPU oracle: it is checked against things other than itself.

* the k-truss definition, written out by brute force, on every graph with 5
  vertices and on random small graphs;
* closed forms (cliques, cliques minus an edge, trees, cycles, wheels, windmills,
  bipartite graphs, grids, disjoint unions, planted cliques);
* the worked examples of the paper (Fig. 2 graph; Fig. 3 sub-level, in
  test_psl_model.py);
* invariants (tau >= 2, tau <= support + 2, every edge of H_k in >= k-2 triangles of
  H_k, t_max <= c_max + 1, sum of supports = 3 x triangles counted by a sparse matrix
  product);
* a second, independent algorithm (local h-index iteration) on medium graphs.
"""
import itertools
import os
import random

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg
import oracle
from oracle import definition as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tau_by_definition(g):
    E = D.edges_from_csr(g)
    bf = D.truss_by_definition(E)
    return np.array([bf[e] for e in E], dtype=np.int32)


def test_every_graph_on_five_vertices():
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        E = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        g = gg.from_edges(5, E)
        assert np.array_equal(oracle.truss(g), tau_by_definition(g)), E


def test_random_six_and_seven_vertex_graphs():
    rng = random.Random(11)
    for n in (6, 7):
        pairs = list(itertools.combinations(range(n), 2))
        for _ in range(400):
            E = [e for e in pairs if rng.random() < rng.choice((0.3, 0.5, 0.7, 0.9))]
            g = gg.from_edges(n, E)
            assert np.array_equal(oracle.truss(g), tau_by_definition(g)), E


def test_random_graphs_up_to_40_vertices():
    rng = random.Random(3)
    for _ in range(250):
        n = rng.randint(2, 40)
        p = rng.random() ** 1.5
        E = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
        g = gg.from_edges(n, E)
        assert np.array_equal(oracle.truss(g), tau_by_definition(g)), (n, E)


# ------------------------------------------------------------------ closed forms

def clique(nodes):
    return [(a, b) for a, b in itertools.combinations(nodes, 2)]


@pytest.mark.parametrize("n", range(2, 14))
def test_complete_graph(n):
    g = gg.from_edges(n, clique(range(n)))
    assert np.all(oracle.truss(g) == n)


@pytest.mark.parametrize("n", range(3, 12))
def test_complete_graph_minus_one_edge(n):
    E = [e for e in clique(range(n)) if e != (0, 1)]
    g = gg.from_edges(n, E)
    assert np.all(oracle.truss(g) == n - 1)


def test_trees_paths_stars_give_two():
    rng = random.Random(5)
    for _ in range(50):
        n = rng.randint(2, 60)
        E = [(rng.randrange(v), v) for v in range(1, n)]  # random recursive tree
        assert np.all(oracle.truss(gg.from_edges(n, E)) == 2)
    assert np.all(oracle.truss(gg.from_edges(30, [(i, i + 1) for i in range(29)])) == 2)
    assert np.all(oracle.truss(gg.from_edges(30, [(0, i) for i in range(1, 30)])) == 2)


def test_cycles():
    assert np.all(oracle.truss(gg.from_edges(3, [(0, 1), (1, 2), (0, 2)])) == 3)
    for n in range(4, 20):
        E = [(i, (i + 1) % n) for i in range(n)]
        assert np.all(oracle.truss(gg.from_edges(n, E)) == 2)


@pytest.mark.parametrize("rim", range(4, 15))
def test_wheel_gives_three(rim):
    E = [(0, i) for i in range(1, rim + 1)] + [(i, i % rim + 1) for i in range(1, rim + 1)]
    assert np.all(oracle.truss(gg.from_edges(rim + 1, E)) == 3)


def test_wheel_with_three_spokes_is_k4():
    E = [(0, 1), (0, 2), (0, 3), (1, 2), (2, 3), (1, 3)]
    assert np.all(oracle.truss(gg.from_edges(4, E)) == 4)


@pytest.mark.parametrize("blades", [1, 2, 5, 17])
def test_windmill_gives_three(blades):
    E = []
    for b in range(blades):
        x, y = 1 + 2 * b, 2 + 2 * b
        E += [(0, x), (0, y), (x, y)]
    assert np.all(oracle.truss(gg.from_edges(2 * blades + 1, E)) == 3)


def test_bipartite_and_grid_give_two():
    E = [(a, 6 + b) for a in range(6) for b in range(7)]
    assert np.all(oracle.truss(gg.from_edges(13, E)) == 2)
    w = 9
    E = [(r * w + c, r * w + c + 1) for r in range(w) for c in range(w - 1)]
    E += [(r * w + c, (r + 1) * w + c) for r in range(w - 1) for c in range(w)]
    assert np.all(oracle.truss(gg.from_edges(w * w, E)) == 2)


def test_disjoint_union_is_per_component():
    E = clique(range(6)) + [(6 + a, 6 + b) for a, b in clique(range(4))] + [(10, 11), (11, 12)]
    g = gg.from_edges(13, E)
    tau = oracle.truss(g)
    want = {e: (6 if e[1] < 6 else 4 if e[1] < 10 else 2) for e in D.canonical_edges(E)}
    assert np.array_equal(tau, np.array([want[e] for e in D.edges_from_csr(g)]))


def test_planted_clique_edges_reach_clique_size():
    base = gg.er(300, mean_degree=4.0, seed=9)
    members = list(range(0, 300, 13))[:20]
    E = D.edges_from_csr(base) + clique(members)
    g = gg.from_edges(300, E)
    tau = oracle.truss(g)
    idx = {e: i for i, e in enumerate(D.edges_from_csr(g))}
    assert all(tau[idx[e]] >= len(members) for e in clique(members))


def test_empty_and_edgeless_graphs():
    assert len(oracle.truss(gg.from_edges(0, []))) == 0
    assert len(oracle.truss(gg.from_edges(7, []))) == 0
    assert np.array_equal(oracle.truss(gg.from_edges(2, [(0, 1)])), [2])


def test_fig2_graph_golden():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "fig2_graph.txt")) if l.strip() and l[0] != "#"]
    n, m = map(int, lines[0])
    rows = [tuple(map(int, r)) for r in lines[1:]]
    assert len(rows) == m
    g = gg.from_edges(n, [(u, v) for u, v, _ in rows])
    idx = {e: i for i, e in enumerate(D.edges_from_csr(g))}
    tau = oracle.truss(g)
    for u, v, t in rows:
        assert tau[idx[(u, v)]] == t


# ------------------------------------------------------------------ invariants

def _triangles_scipy(g):
    A = sp.csr_matrix((np.ones(len(g.adj)), g.adj, g.offsets), shape=(g.n, g.n))
    return int(round((A @ A).multiply(A).sum() / 6))


@pytest.mark.parametrize("name,make", [
    ("er", lambda: gg.er(3000, mean_degree=20.0, seed=2)),
    ("rmat12", lambda: gg.rmat(12, 16, seed=4)),
    ("rgg", lambda: gg.rgg(4000, 24.0, seed=5)),
    ("chunglu", lambda: gg.chunglu(1 << 13, 2.1, 6.0e4, draws=55_000, ncliques=4, cmin=10, cmax=30, seed=6)),
])
def test_invariants(name, make):
    g = make()
    tau, S0 = oracle.truss(g, with_support=True)
    E = np.array(D.edges_from_csr(g), dtype=np.int64)
    # support by definition, and its sum against an independent triangle count
    assert int(S0.sum()) == 3 * _triangles_scipy(g)
    assert np.all(tau >= 2)
    assert np.all(tau <= S0 + 2)
    # validity: every edge of H_k = {tau >= k} lies in >= k-2 triangles inside H_k
    for k in sorted(set(tau.tolist())):
        keep = E[tau >= k]
        sub = gg.from_edges(g.n, keep)
        s_in = oracle.support(sub)
        assert np.all(s_in >= k - 2), (name, k)
    # maximality: no edge with tau = k survives in the definition's H_{k+1}
    # (checked through the h-index oracle below on these same graphs)
    core = D.kcore_numbers(g.n, E.tolist())
    assert tau.max() <= core.max() + 1


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(10, 16, seed=21),
    lambda: gg.er(1500, mean_degree=30.0, seed=22),
    lambda: gg.rgg(2000, 40.0, seed=23),
])
def test_hindex_second_oracle(make):
    g = make()
    E = D.edges_from_csr(g)
    assert np.array_equal(oracle.truss(g), D.hindex_truss(E))


def test_support_matches_definition():
    rng = random.Random(8)
    for _ in range(60):
        n = rng.randint(3, 50)
        p = rng.random()
        E = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
        g = gg.from_edges(n, E)
        sd = D.support_by_definition(D.edges_from_csr(g))
        assert np.array_equal(oracle.support(g), [sd[e] for e in D.edges_from_csr(g)])


def test_relabelling_permutes_output():
    g = gg.rmat(9, 12, seed=31)
    E = D.edges_from_csr(g)
    tau = oracle.truss(g)
    perm = np.random.default_rng(5).permutation(g.n)
    E2 = [(int(perm[u]), int(perm[v])) for u, v in E]
    g2 = gg.from_edges(g.n, E2)
    t2 = dict(zip(D.edges_from_csr(g2), oracle.truss(g2)))
    for (u, v), t in zip(E2, tau):
        assert t2[(min(u, v), max(u, v))] == t


def test_adding_edges_never_lowers_trussness():
    rng = random.Random(4)
    g = gg.er(200, mean_degree=10.0, seed=41)
    E = D.edges_from_csr(g)
    tau = dict(zip(E, oracle.truss(g)))
    extra = [(rng.randrange(200), rng.randrange(200)) for _ in range(150)]
    g2 = gg.from_edges(200, E + extra)
    t2 = dict(zip(D.edges_from_csr(g2), oracle.truss(g2)))
    assert all(t2[e] >= t for e, t in tau.items())


def test_malformed_csr_is_rejected():
    good = gg.from_edges(4, [(0, 1), (1, 2), (0, 2), (2, 3)])
    assert oracle.check_csr(good)
    bad_rows = [
        ([0, 2, 4, 7, 8], [1, 2, 0, 2, 1, 0, 3, 2]),  # row 2 unsorted? (1,0,3)
        ([0, 2, 4, 7, 8], [1, 1, 0, 2, 0, 1, 3, 2]),  # duplicate in row 0
        ([0, 2, 4, 7, 8], [0, 2, 0, 2, 0, 1, 3, 2]),  # self-loop
        ([0, 2, 4, 7, 8], [1, 3, 0, 2, 0, 1, 3, 2]),  # asymmetric (0,3) without (3,0)
        ([0, 2, 4, 7, 8], [1, 2, 0, 9, 0, 1, 3, 2]),  # id out of range
        ([0, 2, 1, 7, 8], [1, 2, 0, 2, 0, 1, 3, 2]),  # offsets decrease
        ([0, 2, 4, 7, 7], [1, 2, 0, 2, 0, 1, 3]),  # odd slot count
    ]
    for off, adj in bad_rows:
        g = gg.Graph(4, np.array(off, np.int64), np.array(adj, np.int32))
        assert not oracle.check_csr(g), (off, adj)
        with pytest.raises(oracle.OracleInputError):
            oracle.truss(g)


# ---- the stored full-size oracle records (tests/golden/*.json, *.txt) are self-consistent

def _full_size_records():
    import json

    for f in sorted(os.listdir(GOLDEN)):
        if f.endswith(".json"):
            rec = json.load(open(os.path.join(GOLDEN, f)))
            if "trussness_sha256" in rec:
                yield f, rec


@pytest.mark.parametrize("name,rec", list(_full_size_records()), ids=lambda x: x if isinstance(x, str) else "")
def test_stored_records_are_consistent(name, rec):
    """Every stored run: the trussness histogram covers all m edges, has no mass below 2 (every
    edge is in the 2-truss), ends at t_max, and a graph with triangles has t_max >= 3 (and none
    means t_max = 2); the digests are sha256 hex strings."""
    h = rec["histogram"]
    assert sum(h) == rec["m"] and len(h) == rec["t_max"] + 1 and h[-1] > 0
    assert h[0] == 0 and h[1] == 0
    assert (rec["triangles"] > 0) == (rec["t_max"] >= 3)
    for k in ("csr_sha256", "trussness_sha256", "support_sha256"):
        assert len(rec[k]) == 64 and int(rec[k], 16) >= 0


def test_stored_batch_records_are_consistent():
    """The per-graph batch records: one line per graph, in order, each with a sha256 digest and
    t_max >= 2 for a graph with edges."""
    for f in ("batch64.txt", "batch4096.txt"):
        path = os.path.join(GOLDEN, f)
        if not os.path.exists(path):
            continue
        rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
        assert [int(r[0]) for r in rows] == list(range(len(rows)))
        for g, n, m, t, h in rows:
            assert int(n) > 0 and int(m) >= 0 and len(h) == 64
            assert (int(m) == 0) or int(t) >= 2
