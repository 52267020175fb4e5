"""Core numbers on the GPU (truss_kcore) against the oracle's bucket order, bit for
bit: small graphs and closed forms, random graphs, medium and full-size synthetic
graphs, the relation to the trussness (t_max <= c_max + 1), and the boundary's
edge cases."""
import itertools
import random

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def gpu_cores(g):
    import torch

    import paper_1707_02000_amd as pkt

    core, cmax = pkt.kcore(torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda())
    c = core.cpu().numpy()
    assert cmax == (int(c.max()) if len(c) else 0)
    return c


def closed_forms():
    yield "isolated", gg.from_edges(5, []), 0
    yield "path", gg.from_edges(6, [(i, i + 1) for i in range(5)]), 1
    yield "star", gg.from_edges(9, [(0, i) for i in range(1, 9)]), 1
    yield "cycle", gg.from_edges(11, [(i, (i + 1) % 11) for i in range(11)]), 2
    for n in (2, 3, 8, 40):
        yield f"K{n}", gg.from_edges(n, list(itertools.combinations(range(n), 2))), n - 1


@pytest.mark.parametrize("name,g,want", list(closed_forms()))
def test_closed_forms(gpu_lib, name, g, want):
    assert set(gpu_cores(g).tolist()) == {want}


@pytest.mark.parametrize("seed", range(12))
def test_random_graphs(gpu_lib, seed):
    rng = random.Random(seed)
    n = rng.randint(1, 300)
    p = rng.uniform(0.0, 0.1)
    edges = {(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p}
    for _ in range(rng.randint(0, 3)):
        vs = sorted(rng.sample(range(n), min(n, rng.randint(3, 30))))
        edges |= set(itertools.combinations(vs, 2))
    g = gg.from_edges(n, sorted(edges))
    assert np.array_equal(gpu_cores(g), oracle.kcore(g))


@pytest.mark.parametrize("name", ["er4096", "rmat16", "chunglu18", "rmat20"])
def test_synthetic_workloads(gpu_lib, name):
    g = gg.workload(name, seed=1)
    c = gpu_cores(g)
    assert np.array_equal(c, oracle.kcore(g))


def test_truss_within_core_bound(gpu_lib):
    import torch

    import paper_1707_02000_amd as pkt

    g = gg.workload("rmat16", seed=3)
    c = gpu_cores(g)
    tau = pkt.truss_decompose(torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda())
    assert int(tau.max().item()) <= int(c.max()) + 1


def test_edge_cases(gpu_lib):
    import torch

    import paper_1707_02000_amd as pkt

    core, cmax = pkt.kcore(np.zeros(1, np.int64), np.zeros(0, np.int32))  # no vertices
    assert core.numel() == 0 and cmax == 0
    # a neighbour id outside [0, n) is rejected
    with pytest.raises(pkt.TrussError) as ei:
        pkt.kcore(np.array([0, 1, 2], np.int64), np.array([1, 7], np.int32))
    assert ei.value.name == "TRUSS_E_RANGE"
    # offsets out of order are rejected
    with pytest.raises(pkt.TrussError) as ei:
        pkt.kcore(np.array([0, 2, 1, 2], np.int64), np.array([1, 2], np.int32))
    assert ei.value.name == "TRUSS_E_RANGE"
    torch.cuda.synchronize()
