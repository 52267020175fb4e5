"""Seeded input generators: determinism, simplicity of the output, expected sizes."""
import numpy as np
import pytest

import graphgen as gg


def assert_simple_csr(g):
    off, adj, n = g.offsets, g.adj, g.n
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(adj)
    assert len(adj) % 2 == 0
    rows = np.repeat(np.arange(n), np.diff(off))
    assert np.all((adj >= 0) & (adj < n)) and np.all(adj != rows)
    same = rows[1:] == rows[:-1]
    assert np.all(np.diff(adj.astype(np.int64))[same] > 0)
    k1 = rows.astype(np.int64) * n + adj
    k2 = adj.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(k1), np.sort(k2))


@pytest.mark.parametrize("make", [
    lambda s: gg.er(4096, mean_degree=16.0, seed=s),
    lambda s: gg.rmat(14, 16, seed=s),
    lambda s: gg.rgg(5000, 20.0, seed=s),
    lambda s: gg.chunglu(1 << 14, 2.1, 1.2e5, draws=110_000, ncliques=3, cmin=20, cmax=40, seed=s),
])
def test_deterministic_and_simple(make):
    a, b, c = make(7), make(7), make(8)
    assert a.sha256() == b.sha256()
    assert a.sha256() != c.sha256()
    assert_simple_csr(a)


def test_er_mean_degree():
    g = gg.er(4096, mean_degree=16.0, seed=1)
    assert abs(2 * g.m / g.n - 16.0) < 0.5


def test_rmat_skew_and_size():
    g = gg.rmat(16, 16, seed=1)
    d = g.degrees()
    assert 0.75 * 16 * 65536 * 0.5 < g.m < 16 * 65536  # dedup removes a share
    assert d.max() > 50 * d[d > 0].mean()  # heavy tail
    assert (d == 0).mean() > 0.2  # R-MAT leaves many vertices isolated


def test_planted_cliques_present():
    g = gg.chunglu(1 << 12, 2.1, 2.0e4, draws=18_000, ncliques=2, cmin=30, cmax=30, seed=3)
    assert g.degrees().max() >= 29


def test_batch_layout():
    b = gg.batch(32, 64, 1024, seed=5)
    assert b.num_graphs == 32
    assert set(b.family.tolist()) <= {0, 1, 2}
    for i in range(b.num_graphs):
        g = b.graph(i)
        assert 64 <= g.n <= 1024
        assert_simple_csr(g)
    again = gg.batch(32, 64, 1024, seed=5)
    assert np.array_equal(again.adj, b.adj) and np.array_equal(again.offsets, b.offsets)


def test_from_edges_and_pack():
    g = gg.from_edges(5, [(0, 1), (1, 0), (2, 2), (3, 4), (1, 2)])
    assert g.m == 3
    assert_simple_csr(g)
    b = gg.pack([g, gg.from_edges(3, [(0, 2)])])
    assert b.num_graphs == 2 and b.total_m == 4
    assert np.array_equal(b.graph(1).adj, [2, 0])


def test_same_graph_at_any_thread_count():
    # a recipe and seed name one graph whatever OMP_NUM_THREADS is (the Chung-Lu weight
    # bisection once summed with a parallel reduction, whose rounding followed the
    # thread count)
    import os
    import subprocess
    import sys

    code = ("import graphgen as gg\n"
            "for name in ('chunglu18', 'rmat14', 'er4096'):\n"
            "    print(name, gg.workload(name, seed=1).sha256())\n"
            "print('batch16', gg.workload('batch16', seed=1).union().sha256())\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True,
                                   check=True, timeout=300).stdout)
    assert outs[0] == outs[1] == outs[2]
