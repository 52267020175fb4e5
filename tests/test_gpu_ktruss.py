"""The maximal k-trusses on the GPU (truss_ktruss) against the oracle's, bit for bit:
every label is the smallest edge id of its k-truss, so the labelling is unique.
Small graphs at every k, medium and full-size synthetic graphs at several k, and the
boundary's edge cases."""
import itertools

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import ktruss as KT

pytestmark = pytest.mark.gpu


def clique(vs):
    return list(itertools.combinations(vs, 2))


def small_graphs():
    yield "K2", gg.from_edges(2, [(0, 1)])
    yield "K7", gg.from_edges(7, clique(range(7)))
    yield "bridge", gg.from_edges(10, clique(range(5)) + clique(range(5, 10)) + [(4, 5)])
    yield "shared_vertex", gg.from_edges(7, clique(range(4)) + clique(range(3, 7)))
    edges = []
    for b in range(6):
        edges += clique(range(10 * b, 10 * b + 3 + b))
    yield "cliques", gg.from_edges(60, edges)
    yield "er", gg.er(300, mean_degree=8.0, seed=3)


def check(g, ks):
    import torch

    import paper_1707_02000_amd as pkt

    off = torch.from_numpy(g.offsets).cuda()
    adj = torch.from_numpy(g.adj).cuda()
    tau = pkt.truss_decompose(off, adj)
    el = pkt.edge_list(off, adj)
    tau_h, el_h = tau.cpu().numpy(), el.cpu().numpy()
    assert np.array_equal(el_h, oracle.edge_list(g))
    for k in ks:
        lab, cnt = pkt.ktruss(g.n, el, tau, k)
        want, wcnt = KT.labels(g.n, el_h, tau_h, k)
        assert np.array_equal(lab.cpu().numpy(), want), (k, cnt, wcnt)
        assert cnt == wcnt, k


@pytest.mark.parametrize("name,g", list(small_graphs()))
def test_small_graphs_every_k(gpu_lib, name, g):
    t = oracle.truss(g)
    check(g, range(2, int(t.max()) + 3))


@pytest.mark.parametrize("make", [
    lambda: gg.workload("rmat16", seed=2),
    lambda: gg.workload("chunglu18", seed=3),
    lambda: gg.rmat(12, 8, seed=5),
])
def test_medium_graphs(gpu_lib, make):
    g = make()
    t = oracle.truss(g)
    tmax = int(t.max())
    check(g, sorted({2, 3, 4, tmax // 2, tmax - 1, tmax, tmax + 1} - {0, 1}))


def test_full_size_rmat20(gpu_lib):
    g = gg.workload("rmat20", seed=1)
    check(g, [3, 50, 150, 304])


def test_edge_cases(gpu_lib):
    import torch

    import paper_1707_02000_amd as pkt

    # no edges
    lab, cnt = pkt.ktruss(4, np.zeros((0, 2), np.int32), np.zeros(0, np.int32), 3)
    assert lab.numel() == 0 and cnt == 0
    # k below 2
    with pytest.raises(pkt.TrussError) as ei:
        pkt.ktruss(3, np.array([[0, 1]], np.int32), np.array([2], np.int32), 1)
    assert ei.value.name == "TRUSS_E_ARG"
    # an endpoint outside [0, n) on an edge that counts is rejected ...
    el = np.array([[0, 1], [1, 5]], np.int32)
    with pytest.raises(pkt.TrussError) as ei:
        pkt.ktruss(3, el, np.array([3, 3], np.int32), 3)
    assert ei.value.name == "TRUSS_E_RANGE"
    # ... and ignored on an edge below k
    lab, cnt = pkt.ktruss(3, el, np.array([3, 2], np.int32), 3)
    assert lab.cpu().tolist() == [0, -1] and cnt == 1
    # k above every trussness
    lab, cnt = pkt.ktruss(3, np.array([[0, 1], [1, 2]], np.int32), np.array([2, 2], np.int32), 3)
    assert lab.cpu().tolist() == [-1, -1] and cnt == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("order", ["reversed_endpoints", "shuffled", "shuffled_and_reversed"])
def test_any_edge_order(gpu_lib, order):
    """The edge list may come in any order and orientation: labels still name the
    smallest edge id (in the given list) of every k-truss."""
    import paper_1707_02000_amd as pkt

    g = gg.workload("rmat16", seed=4)
    tau = oracle.truss(g)
    el = oracle.edge_list(g)
    rng = np.random.default_rng(5)
    perm = np.arange(g.m) if order == "reversed_endpoints" else rng.permutation(g.m)
    el2 = el[perm].copy()
    tau2 = tau[perm].copy()
    if order != "shuffled":
        flip = rng.random(g.m) < (1.0 if order == "reversed_endpoints" else 0.5)
        el2[flip] = el2[flip][:, ::-1]
    tmax = int(tau.max())
    for k in (2, 3, tmax // 2, tmax):
        lab, cnt = pkt.ktruss(g.n, el2, tau2, k)
        want, wcnt = KT.labels(g.n, el2, tau2, k)
        assert np.array_equal(lab.cpu().numpy(), want), (order, k)
        assert cnt == wcnt
    # the smallest case: one edge given as (1, 0)
    lab, cnt = pkt.ktruss(2, np.array([[1, 0]], np.int32), np.array([2], np.int32), 2)
    assert lab.cpu().tolist() == [0] and cnt == 1
