"""KCO reordering on the GPU (truss_kco_order, truss_kco_relabel, truss_kco_map) against
the oracle, bit for bit: the order on core vectors that span one, several and many
radix tiles and one to four radix passes, the relabelled CSR on small and full-size
graphs, and the whole chain (core numbers, order, relabelled CSR, decomposition of the
relabelled graph, trussness mapped back) against the oracle's trussness of the input,
plus the boundary's edge cases."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import kco as K

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("n,hi", [(1, 0), (1023, 3), (1024, 255), (1025, 256), (5000, 0), (5000, 1),
                                  (70_001, 70_000), (300_000, 2**31 - 1), (1 << 20, 609)])
def test_order(gpu_lib, n, hi):
    rng = np.random.default_rng(n + hi)
    core = rng.integers(0, hi + 1, n, dtype=np.int64).astype(np.int32)
    new_id, order = gpu_lib.kco_order(core)
    want_id, want_order = K.order(core)
    assert np.array_equal(order.cpu().numpy(), want_order)
    assert np.array_equal(new_id.cpu().numpy(), want_id)


def small_graphs():
    rng = np.random.default_rng(11)
    yield gg.from_edges(3, [])
    yield gg.from_edges(6, [(i, i + 1) for i in range(5)])
    yield gg.er(300, mean_degree=8.0, seed=3)
    yield gg.rmat(12, 8, seed=5)
    for s in range(3):
        n = int(rng.integers(2, 400))
        yield gg.er(n, mean_degree=float(rng.uniform(1, 12)), seed=20 + s)


def relabel_case(gpu_lib, g, new_id):
    import torch

    order = np.empty(g.n, np.int32)
    order[new_id] = np.arange(g.n, dtype=np.int32)
    off2, adj2 = gpu_lib.kco_relabel(g.offsets, g.adj, torch.from_numpy(new_id).cuda(),
                                     torch.from_numpy(order).cuda())
    w_off, w_adj = K.relabel(g.offsets, g.adj, new_id)
    assert np.array_equal(off2.cpu().numpy(), w_off)
    assert np.array_equal(adj2.cpu().numpy(), w_adj)


@pytest.mark.parametrize("g", list(small_graphs()), ids=lambda g: g.name or f"n{g.n}")
def test_relabel_small(gpu_lib, g):
    rng = np.random.default_rng(g.n)
    relabel_case(gpu_lib, g, rng.permutation(g.n).astype(np.int32))
    relabel_case(gpu_lib, g, K.order(oracle.kcore(g))[0])


def chain(gpu_lib, g):
    """Trussness of g through KCO on the GPU, and the relabelled graph."""
    import torch

    off = torch.from_numpy(g.offsets).cuda()
    adj = torch.from_numpy(g.adj).cuda()
    core, _ = gpu_lib.kcore(off, adj)
    new_id, order = gpu_lib.kco_order(core)
    off2, adj2 = gpu_lib.kco_relabel(off, adj, new_id, order)
    tau2 = gpu_lib.truss_decompose(off2, adj2)
    el = gpu_lib.edge_list(off, adj)
    tau = gpu_lib.kco_map(g.n, el, new_id, off2, adj2, tau2)
    return tau.cpu().numpy(), core.cpu().numpy(), new_id.cpu().numpy(), off2, adj2


@pytest.mark.parametrize("g", list(small_graphs()), ids=lambda g: g.name or f"n{g.n}")
def test_chain_small(gpu_lib, g):
    tau, core, new_id, _, _ = chain(gpu_lib, g)
    assert np.array_equal(core, oracle.kcore(g))
    assert np.array_equal(new_id, K.order(core)[0])
    assert np.array_equal(tau, oracle.truss(g))


@pytest.mark.parametrize("name", ["rmat16", "rmat20"])
def test_chain_full_size(gpu_lib, name):
    rec = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
    g = gg.workload(name, seed=rec["seed"])
    assert g.sha256() == rec["csr_sha256"]
    say("case", name, "m", g.m)
    tau, core, new_id, off2, adj2 = chain(gpu_lib, g)
    assert np.array_equal(core, oracle.kcore(g))
    assert np.array_equal(new_id, K.order(core)[0])
    w_off, w_adj = K.relabel(g.offsets, g.adj, new_id)
    assert np.array_equal(off2.cpu().numpy(), w_off)
    assert np.array_equal(adj2.cpu().numpy(), w_adj)
    import hashlib

    assert hashlib.sha256(np.ascontiguousarray(tau, np.int32).tobytes()).hexdigest() == rec["trussness_sha256"]


def test_edge_cases(gpu_lib):
    import torch

    pkt = gpu_lib
    new_id, order = pkt.kco_order(np.zeros(0, np.int32))  # no vertices
    assert new_id.numel() == 0 and order.numel() == 0
    with pytest.raises(pkt.TrussError) as ei:  # a negative core number
        pkt.kco_order(np.array([0, -1, 2], np.int32))
    assert ei.value.name == "TRUSS_E_RANGE"
    g = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    ident = np.arange(4, dtype=np.int32)
    with pytest.raises(pkt.TrussError) as ei:  # new_id not a permutation
        pkt.kco_relabel(g.offsets, g.adj, np.array([0, 0, 2, 3], np.int32), ident)
    assert ei.value.name == "TRUSS_E_RANGE"
    with pytest.raises(pkt.TrussError) as ei:  # order not the inverse of new_id
        pkt.kco_relabel(g.offsets, g.adj, np.array([1, 0, 2, 3], np.int32), ident)
    assert ei.value.name == "TRUSS_E_RANGE"
    with pytest.raises(pkt.TrussError) as ei:  # a neighbour out of range
        pkt.kco_relabel(np.array([0, 1, 2], np.int64), np.array([1, 9], np.int32), ident[:2], ident[:2])
    assert ei.value.name == "TRUSS_E_RANGE"
    with pytest.raises(pkt.TrussError) as ei:  # not symmetric
        pkt.kco_relabel(np.array([0, 1, 1], np.int64), np.array([1], np.int32), ident[:2], ident[:2])
    assert ei.value.name == "TRUSS_E_NOT_SYMMETRIC"
    with pytest.raises(pkt.TrussError) as ei:  # a directed 3-cycle: in- and out-degrees agree everywhere
        pkt.kco_relabel(np.array([0, 1, 2, 3], np.int64), np.array([1, 2, 0], np.int32), ident[:3], ident[:3])
    assert ei.value.name == "TRUSS_E_NOT_SYMMETRIC"
    with pytest.raises(pkt.TrussError) as ei:  # the same under a non-trivial relabelling
        pkt.kco_relabel(np.array([0, 1, 2, 3], np.int64), np.array([1, 2, 0], np.int32),
                        np.array([2, 0, 1], np.int32), np.array([1, 2, 0], np.int32))
    assert ei.value.name == "TRUSS_E_NOT_SYMMETRIC"
    off2, adj2 = pkt.kco_relabel(np.zeros(4, np.int64), np.zeros(0, np.int32), ident[:3], ident[:3])  # no edges
    assert off2.cpu().tolist() == [0, 0, 0, 0] and adj2.numel() == 0
    # mapping: an edge with no image, and a relabelled graph of another size
    tau2 = np.full(3, 2, np.int32)
    with pytest.raises(pkt.TrussError) as ei:
        pkt.kco_map(4, np.array([[0, 1], [1, 2], [0, 3]], np.int32), ident, g.offsets, g.adj, tau2)
    assert ei.value.name == "TRUSS_E_RANGE"
    with pytest.raises(pkt.TrussError) as ei:
        pkt.kco_map(4, np.array([[0, 1], [1, 2]], np.int32), ident, g.offsets, g.adj, tau2[:2])
    assert ei.value.name == "TRUSS_E_ARG"
    tau = pkt.kco_map(4, np.array([[2, 3], [0, 1], [1, 2]], np.int32), ident, g.offsets, g.adj,
                      np.array([5, 6, 7], np.int32))
    assert tau.cpu().tolist() == [7, 5, 6]
    torch.cuda.synchronize()
