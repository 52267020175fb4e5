"""GPU parity: libpkt (through its C ABI) against the CPU oracle, bit for bit.

All outputs are integers (edge ids, supports, trussness), so every comparison is
exact.  Small cases run the oracle in-process; full-size workloads compare against
stored expectations written by tests/golden/make_golden.py (oracle only).
"""
import hashlib
import itertools
import json
import os
import random

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import certificate
from oracle import definition as D

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)


def gpu_tau(pkt, g, **kw):
    return pkt.truss_decompose(g.offsets, g.adj, **kw).cpu().numpy()


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, np.int32).tobytes()).hexdigest()


def test_native_library_loaded(gpu_lib):
    assert gpu_lib.load()._name == gpu_lib.LIB_PATH


def small_graphs():
    yield "K2", gg.from_edges(2, [(0, 1)])
    for n in (3, 5, 9, 17, 40):
        yield f"K{n}", gg.from_edges(n, itertools.combinations(range(n), 2))
    yield "K12-e", gg.from_edges(12, [e for e in itertools.combinations(range(12), 2) if e != (0, 1)])
    yield "wheel", gg.from_edges(9, [(0, i) for i in range(1, 9)] + [(i, i % 8 + 1) for i in range(1, 9)])
    yield "windmill", gg.from_edges(11, sum(([(0, 2 * b + 1), (0, 2 * b + 2), (2 * b + 1, 2 * b + 2)]
                                             for b in range(5)), []))
    yield "path", gg.from_edges(50, [(i, i + 1) for i in range(49)])
    yield "isolated", gg.from_edges(30, [(3, 7), (7, 9), (3, 9), (20, 21)])
    rng = random.Random(1)
    for i in range(40):
        n = rng.randint(2, 40)
        p = rng.random() ** 1.3
        yield f"rand{i}", gg.from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p])


@pytest.mark.parametrize("name,g", list(small_graphs()))
def test_small_graphs(gpu_lib, name, g):
    say("case", name, "n", g.n, "m", g.m)
    want = oracle.truss(g)
    assert np.array_equal(gpu_tau(gpu_lib, g), want)
    assert np.array_equal(gpu_tau(gpu_lib, g, force_choice="wave"), want)
    assert np.array_equal(gpu_tau(gpu_lib, g, force_choice="hash"), want)
    assert np.array_equal(gpu_tau(gpu_lib, g, relabel=True), want)


@pytest.mark.parametrize("make", [
    lambda: gg.er(4096, mean_degree=16.0, seed=1),
    lambda: gg.rmat(12, 16, seed=3),
    lambda: gg.rgg(3000, 30.0, seed=4),
    lambda: gg.chunglu(1 << 13, 2.1, 6.0e4, draws=55_000, ncliques=4, cmin=10, cmax=40, seed=5),
])
def test_support_and_edge_list(gpu_lib, make):
    g = make()
    say("case", g.name)
    el = gpu_lib.edge_list(g.offsets, g.adj).cpu().numpy()
    assert np.array_equal(el, oracle.edge_list(g))
    S = gpu_lib.truss_support(g.offsets, g.adj).cpu().numpy()
    assert np.array_equal(S, oracle.support(g))


@pytest.mark.parametrize("make", [
    lambda: gg.er(4096, mean_degree=16.0, seed=1),
    lambda: gg.rmat(12, 16, seed=3),
    lambda: gg.rmat(14, 16, seed=7),
    lambda: gg.rgg(3000, 30.0, seed=4),
    lambda: gg.chunglu(1 << 13, 2.1, 6.0e4, draws=55_000, ncliques=4, cmin=10, cmax=40, seed=5),
])
@pytest.mark.parametrize("opts", [
    dict(),
    dict(owner_rule=1),
    dict(compact=False),
    dict(variant="bsearch"),
    dict(variant="merge"),
    dict(force_choice="fused_narrow"),
    dict(force_choice="wide"),
    dict(force_choice="wide_narrow"),
    dict(force_choice="wide_gallop"),
    dict(single_round=True),
    dict(device_loop="host"),
    dict(device_loop="graph"),
    dict(device_loop="device", steps_per_sync=1),
    dict(device_loop="graph", steps_per_sync=3),
    dict(device_loop="device", profile=True),
    dict(device_loop="host", force_choice="wide_narrow"),
    dict(device_loop="graph", force_choice="fused_narrow"),
    dict(device_loop="pipelined"),
    dict(device_loop="pipelined", force_choice="wide_narrow"),
    dict(device_loop="pipelined", force_choice="fused_narrow"),
    dict(device_loop="pipelined", variant="merge", profile=True),
    dict(device_loop="pipelined", compact=False),
    dict(force_choice="wave"),
    dict(force_choice="wave", owner_rule=1),
    dict(device_loop="host", force_choice="wave"),
    dict(device_loop="graph", force_choice="wave"),
    dict(device_loop="device", force_choice="wave", steps_per_sync=2),
    dict(device_loop="pipelined", force_choice="wave", compact=False),
    dict(multi_round=True),
    dict(device_loop="host", multi_round=True),
    dict(force_choice="hash"),
    dict(force_choice="hash", owner_rule=1, compact=False),
    dict(device_loop="host", force_choice="hash"),
    dict(device_loop="graph", force_choice="hash"),
    dict(multi_round=True, variant="merge"),
    dict(relabel=True),
    dict(relabel=True, device_loop="host"),
    dict(relabel=True, force_choice="wave", owner_rule=1),
    dict(relabel=True, device_loop="graph", compact=False),
    dict(relabel=False),
    dict(relabel=False, device_loop="host"),
    dict(relabel=False, force_choice="wave"),
    dict(relabel=False, device_loop="graph", compact=False),
])
def test_medium_graphs(gpu_lib, make, opts):
    g = make()
    say("case", g.name, opts)
    assert np.array_equal(gpu_tau(gpu_lib, g, **opts), oracle.truss(g))


@pytest.mark.parametrize("relabel", [True, False, "auto"])
def test_int32_offsets(gpu_lib, relabel):
    g = gg.rmat(11, 16, seed=2)
    tau = gpu_lib.truss_decompose(g.offsets.astype(np.int32), g.adj, relabel=relabel).cpu().numpy()
    assert np.array_equal(tau, oracle.truss(g))


def test_relabel_workspace_and_phase_times(gpu_lib):
    """The relabelling needs its larger workspace (refused below it) and reports its
    time inside the build phase; without it the smaller workspace is enough."""
    import torch

    g = gg.rmat(12, 16, seed=4)
    n, two_m = g.n, len(g.adj)
    small = gpu_lib.workspace_bytes(n, two_m, gpu_lib.make_options(relabel=False))
    big = gpu_lib.workspace_bytes(n, two_m)
    assert big > small
    off, adj = torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda()
    buf, ptr = gpu_lib.alloc_workspace(small)
    ws = gpu_lib.Workspace(n, two_m, buf, ptr, small)
    with pytest.raises(gpu_lib.TrussError) as ei:
        gpu_lib.truss_decompose(off, adj, workspace=ws)
    assert ei.value.name == "TRUSS_E_WORKSPACE"
    want = oracle.truss(g)
    assert np.array_equal(gpu_lib.truss_decompose(off, adj, workspace=ws, relabel=False).cpu().numpy(), want)
    tau, st = gpu_lib.truss_decompose(off, adj, return_stats=True, relabel=True)
    assert np.array_equal(tau.cpu().numpy(), want)
    assert st["ms_build"] > 0 and st["ms_total"] >= st["ms_build"] + st["ms_peel"]


@pytest.mark.parametrize("make", [
    lambda: gg.rgg(200_000, 30.0, seed=4),      # above the size limit, degrees not skewed: as given
    lambda: gg.rmat(17, 16, seed=11),           # above it and skewed: relabelled
    lambda: gg.er(90_000, mean_degree=24.0, seed=2),
])
def test_relabel_policies_agree(gpu_lib, make):
    """The automatic policy on graphs above its size limit, on both sides of its skew test,
    and the int32 entry point: every policy gives the trussness of the graph as given."""
    import torch

    g = make()
    say("case", g.name, "m", g.m)
    off, adj = torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda()
    base = gpu_lib.truss_decompose(off, adj, relabel=False).cpu().numpy()
    for mode in ("auto", "always"):
        for o in (off, off.to(torch.int32)):
            tau, rounds = gpu_lib.truss_decompose(o, adj, relabel=mode, return_rounds=True)
            assert np.array_equal(tau.cpu().numpy(), base), mode
            assert int(rounds.min()) >= 0


def test_repeatable(gpu_lib):
    g = gg.rmat(13, 16, seed=9)
    ref = gpu_tau(gpu_lib, g)
    for _ in range(5):
        assert np.array_equal(gpu_tau(gpu_lib, g), ref)


@pytest.mark.parametrize("n", [1100, 2100])
def test_large_cliques_closed_form(gpu_lib, n):
    # out-rows longer than the support kernel's LDS hash (1024): staged in LDS up to
    # 2048 entries, searched in memory beyond; K_n has trussness n and support n - 2
    g = gg.from_edges(n, itertools.combinations(range(n), 2))
    say("case K", n)
    assert np.all(gpu_lib.truss_support(g.offsets, g.adj).cpu().numpy() == n - 2)
    assert np.all(gpu_tau(gpu_lib, g) == n)


def test_empty_and_degenerate(gpu_lib):
    for g in (gg.from_edges(0, []), gg.from_edges(5, []), gg.from_edges(1, [])):
        assert gpu_tau(gpu_lib, g).shape == (0,)
    assert np.array_equal(gpu_tau(gpu_lib, gg.from_edges(2, [(0, 1)])), [2])


def test_malformed_inputs_rejected(gpu_lib):
    cases = {
        "TRUSS_E_NOT_SIMPLE": ([0, 2, 4, 7, 8], [1, 2, 0, 2, 1, 0, 3, 2]),
        "TRUSS_E_RANGE": ([0, 2, 4, 7, 8], [1, 2, 0, 9, 0, 1, 3, 2]),
        "TRUSS_E_NOT_SYMMETRIC": ([0, 2, 4, 7, 8], [1, 3, 0, 2, 0, 1, 3, 2]),
    }
    for want, (off, adj) in cases.items():
        with pytest.raises(gpu_lib.TrussError) as ei:
            gpu_lib.truss_decompose(np.array(off, np.int64), np.array(adj, np.int32))
        assert ei.value.name == want
    with pytest.raises(gpu_lib.TrussError) as ei:  # self-loops on both vertices of an edge
        gpu_lib.truss_decompose(np.array([0, 2, 4], np.int64), np.array([0, 1, 0, 1], np.int32))
    assert ei.value.name == "TRUSS_E_NOT_SIMPLE"
    with pytest.raises(gpu_lib.TrussError) as ei:  # odd slot count
        gpu_lib.truss_decompose(np.array([0, 2, 3], np.int64), np.array([1, 2, 0], np.int32))
    assert ei.value.name in ("TRUSS_E_ARG", "TRUSS_E_RANGE")


@pytest.mark.parametrize("mode", ["union", "sequential", "persistent"])
def test_batched_matches_oracle(gpu_lib, mode):
    b = gg.batch(24, 64, 700, seed=11)
    say("case batch24", b.total_m, "mode", mode)
    tau = gpu_lib.truss_decompose_batched(b.vtx_off, b.adj_off, b.offsets, b.adj, mode=mode).cpu().numpy()
    for i in range(b.num_graphs):
        g = b.graph(i)
        s = int(b.adj_off[i]) // 2
        assert np.array_equal(tau[s:s + g.m], oracle.truss(g)), i


@pytest.mark.parametrize("mode", ["union", "sequential", "persistent"])
def test_batched_edge_cases(gpu_lib, mode):
    graphs = [gg.from_edges(0, []), gg.from_edges(5, []), gg.from_edges(3, [(0, 1), (1, 2), (0, 2)]),
              gg.from_edges(1, []), gg.rmat(9, 8, seed=2), gg.from_edges(4, itertools.combinations(range(4), 2)),
              gg.from_edges(120, itertools.combinations(range(120), 2)),  # K_120: above the LDS support limit
              gg.from_edges(2, [(0, 1)])]
    b = gg.pack(graphs)
    tau = gpu_lib.truss_decompose_batched(b.vtx_off, b.adj_off, b.offsets, b.adj, mode=mode).cpu().numpy()
    want = np.concatenate([oracle.truss(g) for g in graphs])
    assert np.array_equal(tau, want)
    bad = gg.pack([gg.from_edges(3, [(0, 1)]), gg.from_edges(2, [(0, 1)])])
    bad.adj[0] = 5  # local id beyond its graph
    with pytest.raises(gpu_lib.TrussError) as ei:
        gpu_lib.truss_decompose_batched(bad.vtx_off, bad.adj_off, bad.offsets, bad.adj, mode=mode)
    assert ei.value.name in ("TRUSS_E_RANGE", "TRUSS_E_NOT_SYMMETRIC", "TRUSS_E_NOT_SIMPLE")
    # a row out of order, a self-loop, a missing mirror: each rejected
    for edit, want_name in ((lambda a: a.__setitem__(slice(0, 2), a[0:2][::-1].copy()), "TRUSS_E_NOT_SIMPLE"),
                            (lambda a: a.__setitem__(0, 0), "TRUSS_E_NOT_SIMPLE"),
                            (lambda a: a.__setitem__(1, 3), "TRUSS_E_NOT_SYMMETRIC")):
        t = gg.pack([gg.from_edges(4, [(0, 1), (0, 2), (1, 2), (2, 3)])])
        edit(t.adj)
        with pytest.raises(gpu_lib.TrussError) as ei:
            gpu_lib.truss_decompose_batched(t.vtx_off, t.adj_off, t.offsets, t.adj, mode=mode)
        assert ei.value.name in (want_name, "TRUSS_E_NOT_SIMPLE", "TRUSS_E_NOT_SYMMETRIC"), (mode, want_name)
    # a graph with no offsets entry at all (it would shift the next graph onto this one's
    # vertices), and graph offsets not starting at 0: rejected in every mode
    ok = gg.pack([gg.from_edges(3, [(0, 1), (1, 2), (0, 2)]), gg.from_edges(3, [(0, 1), (1, 2), (0, 2)])])
    for vo, ao in ((np.array([0, 4, 4, 8], np.int64), np.array([0, 6, 6, 12], np.int64)),
                   (np.array([1, 5, 8], np.int64), ok.adj_off)):
        offs = np.concatenate([ok.offsets, np.zeros(int(vo[-1]) - len(ok.offsets), np.int32)])
        for mode in ("union", "sequential", "persistent"):
            with pytest.raises(gpu_lib.TrussError) as ei:
                gpu_lib.truss_decompose_batched(vo, ao, offs, ok.adj, validate=False, mode=mode)
            assert ei.value.name == "TRUSS_E_RANGE"


def test_batched_full_config_sample(gpu_lib):
    # the 4096-graph recipe at its full size range, every 64th graph checked against the oracle
    b = gg.batch(256, 64, 16384, seed=1)
    say("case batch256", b.total_m)
    tau = gpu_lib.truss_decompose_batched(b.vtx_off, b.adj_off, b.offsets, b.adj, validate=False).cpu().numpy()
    for i in range(0, b.num_graphs, 64):
        g = b.graph(i)
        s = int(b.adj_off[i]) // 2
        assert np.array_equal(tau[s:s + g.m], oracle.truss(g)), i


@pytest.mark.parametrize("mode", ["host", "device", "graph", "pipelined"])
def test_loop_modes_full_size(gpu_lib, mode):
    rec = _golden("rmat18")
    g = gg.workload("rmat18", seed=rec["seed"])
    say("case rmat18 loop", mode)
    tau, st = gpu_lib.truss_decompose(g.offsets, g.adj, validate=False, device_loop=mode, return_stats=True)
    assert sha(tau.cpu().numpy()) == rec["trussness_sha256"]
    assert st["sublevels"] > 0 and sum(st["choice_count"]) > 0


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored expectation for {name}")
    return json.load(open(path))


@pytest.mark.parametrize("name", ["er4096", "rmat16", "rmat18", "rmat20", "chunglu23", "rmat24"])
def test_full_size_against_stored_oracle(gpu_lib, name):
    """Every edge of the full-size workloads, bit for bit, against the stored oracle run."""
    import torch

    rec = _golden(name)
    g = gg.workload(name, seed=rec["seed"])
    assert g.sha256() == rec["csr_sha256"]
    say("case", name, "m", g.m)
    off, adj = torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda()
    tau, st = gpu_lib.truss_decompose(off, adj, validate=False, return_stats=True)
    tau = tau.cpu().numpy()
    assert int(tau.max()) == rec["t_max"]
    assert np.bincount(tau).tolist() == rec["histogram"]
    assert sha(tau) == rec["trussness_sha256"]
    assert st["triangles"] == rec["triangles"]
    S = gpu_lib.truss_support(off, adj).cpu().numpy()
    assert sha(S) == rec["support_sha256"]


@pytest.mark.parametrize("opts", [
    dict(device_loop="host"),
    dict(device_loop="graph"),
    dict(variant="merge"),
    dict(force_choice="wide_narrow"),
    dict(compact=False),
    dict(owner_rule=1),
    dict(force_choice="wave"),
    dict(force_choice="hash"),
    dict(multi_round=True),
    dict(relabel=False),
])
def test_full_size_variants_rmat20(gpu_lib, opts):
    """Launch variants and loop drivers at the full R-MAT scale-20 size: every one gives
    the oracle's trussness."""
    import torch

    rec = _golden("rmat20")
    g = gg.workload("rmat20", seed=rec["seed"])
    say("case rmat20", opts)
    off, adj = torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda()
    tau = gpu_lib.truss_decompose(off, adj, validate=False, **opts).cpu().numpy()
    assert sha(tau) == rec["trussness_sha256"]


def _batch_golden(name):
    path = os.path.join(GOLDEN, f"{name}.txt")
    if not os.path.exists(path):
        pytest.skip(f"no stored expectation for {name}")
    rows = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        g, n, m, t, h = line.split()
        rows.append((int(g), int(n), int(m), int(t), h))
    return rows


@pytest.mark.parametrize("name,mode,variant", [
    ("batch64", "union", "auto"), ("batch64", "sequential", "auto"), ("batch64", "persistent", "auto"),
    ("batch64", "union", "wave"), ("batch4096", "union", "auto"), ("batch4096", "persistent", "auto"),
    ("batch4096", "union", "learned"),
])
def test_batch_every_graph_against_stored_oracle(gpu_lib, name, mode, variant):
    """Every graph of the packed batch workloads against the oracle run on that graph alone."""
    import torch

    rows = _batch_golden(name)
    b = gg.workload(name, seed=1)
    assert b.num_graphs == len(rows)
    say("case", name, mode, variant, "graphs", b.num_graphs, "total m", b.total_m)
    dev = [torch.from_numpy(x).cuda() for x in (b.vtx_off, b.adj_off, b.offsets, b.adj)]
    kw = {}
    if variant == "wave":
        kw["force_choice"] = "wave"
    elif variant == "learned":
        from paper_1707_02000_amd import tuner

        kw.update(variant="learned", mlp_weights=tuner.load_weights())
    tau = gpu_lib.truss_decompose_batched(*dev, validate=False, mode=mode, **kw).cpu().numpy()
    bad = []
    for g, n, m, t, h in rows:
        s = int(b.adj_off[g]) // 2
        assert int(b.adj_off[g + 1] - b.adj_off[g]) == 2 * m
        part = tau[s:s + m]
        if sha(part) != h:
            bad.append(g)
    assert not bad, f"{len(bad)} graphs differ, first {bad[:10]}"


# ---- peeling-order certificates (oracle/certificate.py): exact at any size

@pytest.mark.parametrize("make", [
    lambda: gg.rmat(13, 16, seed=5),
    lambda: gg.chunglu(1 << 12, 2.1, 3.0e4, draws=27_000, ncliques=4, cmin=10, cmax=40, seed=6),
])
@pytest.mark.parametrize("mode,relabel", [("pipelined", True), ("host", True), ("pipelined", False)])
def test_rounds_are_a_peeling_certificate(gpu_lib, make, mode, relabel):
    g = make()
    say("case", g.name, mode, "relabel", relabel)
    tau, rounds = gpu_lib.truss_decompose(g.offsets, g.adj, device_loop=mode, return_rounds=True,
                                          relabel=relabel)
    tau, rounds = tau.cpu().numpy(), rounds.cpu().numpy()
    assert np.array_equal(tau, oracle.truss(g))
    res = certificate.verify(g, tau, rounds)
    assert res["ok"], (res["monotone"], res["lower_bound_fails"][:5], res["upper_bound_fails"][:5])


def _sampled_support_ok(g, S, edges):
    cert = certificate.Certificate(g)
    return all(len(cert.partners(int(e))[0]) == int(S[e]) for e in edges)


@pytest.mark.parametrize("name", ["rmat24", "chunglu23"])
def test_full_size_certificate(gpu_lib, name):
    """Full-size inputs the serial oracle cannot finish in a test: the trussness is checked
    against the definition through the peeling-order certificate on a stratified sample
    (every trussness value), the support on a sample, and two loop drivers agree."""
    import time

    import torch

    t0 = time.time()
    g = gg.workload(name, seed=1)
    say("case", name, "n", g.n, "m", g.m, "generated in", round(time.time() - t0, 1), "s")
    off, adj = torch.from_numpy(g.offsets).cuda(), torch.from_numpy(g.adj).cuda()
    t0 = time.time()
    tau, rounds, st = gpu_lib.truss_decompose(off, adj, validate=True, return_rounds=True, return_stats=True)
    tau, rounds = tau.cpu().numpy(), rounds.cpu().numpy()
    say("decomposed in", round(time.time() - t0, 2), "s; t_max", st["t_max"], "levels", st["levels"],
        "rounds", st["sublevels"])
    assert int(tau.min()) >= 2 and int(tau.max()) == st["t_max"]
    assert int(rounds.min()) >= 0 and st["sublevels"] == int(rounds.max()) + 1
    assert certificate.monotone_order(tau, rounds)
    edges = certificate.sample_edges(tau, n_uniform=20_000, per_value=20)
    res = certificate.Certificate(g).check(tau, rounds, edges)
    say("certificate on", len(edges), "edges:", len(res["lower_bound_fails"]), len(res["upper_bound_fails"]), "fails")
    assert not res["lower_bound_fails"] and not res["upper_bound_fails"]
    S = gpu_lib.truss_support(off, adj).cpu().numpy()
    assert int(S.sum()) == 3 * st["triangles"]
    assert _sampled_support_ok(g, S, edges[:5000])
    tau2 = gpu_lib.truss_decompose(off, adj, validate=False, device_loop="host").cpu().numpy()
    assert np.array_equal(tau, tau2)
