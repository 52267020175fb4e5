"""The local h-index iteration on the GPU (truss_hindex) against the oracle, bit for bit:
the estimates after every sweep (the sweeps are synchronous, so each one is unique),
the number of sweeps, and the converged trussness on small and medium graphs and
R-MAT s16 (stored oracle record), plus the boundary's edge cases."""
import hashlib
import itertools
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import definition as D

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def graphs():
    yield gg.from_edges(5, list(itertools.combinations(range(5), 2)))
    yield gg.from_edges(4, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3)])  # two triangles on (0, 1)
    yield gg.from_edges(6, [(i, i + 1) for i in range(5)])  # no triangle
    for s in range(4):
        yield gg.er(60 + 40 * s, mean_degree=6.0 + 3 * s, seed=30 + s)
    yield gg.rmat(10, 8, seed=2)


@pytest.mark.parametrize("g", list(graphs()), ids=lambda g: g.name or f"n{g.n}")
def test_every_sweep(gpu_lib, g):
    E = D.edges_from_csr(g)
    want_est, want_sweeps = D.hindex_estimates(E)
    tau, sweeps, conv = gpu_lib.hindex(g.offsets, g.adj)
    assert conv and sweeps == want_sweeps
    assert np.array_equal(tau.cpu().numpy(), oracle.truss(g))
    assert np.array_equal(tau.cpu().numpy(), want_est + 2)
    for k in range(0, want_sweeps + 2):
        est_k, done = D.hindex_estimates(E, sweeps=k)
        t, s, c = gpu_lib.hindex(g.offsets, g.adj, max_sweeps=k)
        assert np.array_equal(t.cpu().numpy(), est_k + 2), k
        assert s == done, k


@pytest.mark.parametrize("make", [lambda: gg.rmat(12, 16, seed=7), lambda: gg.workload("er4096", seed=1)])
def test_medium_graphs(gpu_lib, make):
    g = make()
    tau, sweeps, conv = gpu_lib.hindex(g.offsets, g.adj)
    assert conv
    assert np.array_equal(tau.cpu().numpy(), oracle.truss(g))
    t1, s1, _ = gpu_lib.hindex(g.offsets, g.adj, max_sweeps=1)
    est1, _ = D.hindex_estimates(D.edges_from_csr(g), sweeps=1)
    assert np.array_equal(t1.cpu().numpy(), est1 + 2)


def test_rmat16_against_stored_oracle(gpu_lib):
    rec = json.load(open(os.path.join(GOLDEN, "rmat16.json")))
    g = gg.workload("rmat16", seed=rec["seed"])
    assert g.sha256() == rec["csr_sha256"]
    tau, sweeps, conv = gpu_lib.hindex(g.offsets, g.adj)
    print("rmat16 sweeps", sweeps, flush=True)
    assert conv
    t = np.ascontiguousarray(tau.cpu().numpy(), np.int32)
    assert hashlib.sha256(t.tobytes()).hexdigest() == rec["trussness_sha256"]


def test_edge_cases(gpu_lib):
    import torch

    pkt = gpu_lib
    tau, sweeps, conv = pkt.hindex(np.zeros(4, np.int64), np.zeros(0, np.int32))  # no edges
    assert tau.numel() == 0 and sweeps == 0 and conv
    cases = [
        ([0, 2, 3, 4], [2, 1, 0, 0], "TRUSS_E_NOT_SIMPLE"),  # a row not increasing
        ([0, 2, 4], [0, 1, 0, 1], "TRUSS_E_NOT_SIMPLE"),  # self loops
        ([0, 1, 1, 2], [1, 0], "TRUSS_E_NOT_SYMMETRIC"),  # (2, 0) without (0, 2)
        ([0, 1, 2, 3], [1, 0, 0], "TRUSS_E_NOT_SYMMETRIC"),  # odd slot count
        ([0, 1, 2], [1, 5], "TRUSS_E_RANGE"),  # a neighbour out of range
        ([0, 2, 1, 2], [1, 0], "TRUSS_E_RANGE"),  # offsets out of order
    ]
    for off, adj, want in cases:
        with pytest.raises(pkt.TrussError) as ei:
            pkt.hindex(np.array(off, np.int64), np.array(adj, np.int32))
        assert ei.value.name == want, (off, adj)
    torch.cuda.synchronize()
