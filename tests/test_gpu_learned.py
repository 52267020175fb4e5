"""The learned launch dispatcher on the GPU: cost-model kernels against the CPU fp64
reference, training, the in-loop decision routine, bit-identical trussness under the
learned policy, and what the trained model gains over the heuristic on held-out
traces."""
import ctypes
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import mlp as ref

pytestmark = pytest.mark.gpu
K = 6  # launch choices the model scores (TRUSS_MODEL_CHOICES)


def say(*a):
    print(*a, flush=True)


def problem(seed, n=256):
    rng = np.random.default_rng(seed)
    _, total = ref.layout(K)
    w = rng.normal(0, 0.25, total).astype(np.float32)
    lay, _ = ref.layout(K)
    a, b = lay["mu"]
    w[a:b] = rng.normal(0, 1, b - a)
    a, b = lay["sig"]
    w[a:b] = rng.uniform(0.5, 2.0, b - a)
    X = rng.normal(0, 2, (n, 6)).astype(np.float32)
    T = rng.normal(0, 1, (n, K)).astype(np.float32)
    M = (rng.random((n, K)) < 0.7).astype(np.float32)
    return w, X, T, M


def test_parameter_count(gpu_lib):
    assert gpu_lib.load().truss_mlp_num_params() == ref.layout(K)[1]


def test_forward_matches_cpu(gpu_lib):
    from paper_1707_02000_amd import tuner
    import torch

    w, X, _, _ = problem(1)
    Y = tuner.predict(torch.from_numpy(w).cuda(), X)
    Yr, _ = ref.forward(w.astype(np.float64), X.astype(np.float64), K)
    assert np.allclose(Y, Yr, rtol=1e-4, atol=1e-4)


def test_gradient_matches_cpu(gpu_lib):
    import torch

    lib = gpu_lib.load()
    w, X, T, M = problem(2)
    n = X.shape[0]
    d = {k: torch.from_numpy(v).cuda() for k, v in dict(w=w, X=X, T=T, M=M).items()}
    g = torch.zeros_like(d["w"])
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    nb = lib.truss_mlp_workspace_bytes(n)
    _buf, wptr = gpu_lib.alloc_workspace(nb)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    code = lib.truss_mlp_gradient(p(d["X"]), p(d["T"]), p(d["M"]), n, p(d["w"]), p(g), p(loss),
                                  ctypes.c_void_p(wptr), nb, None)
    assert code == 0
    g_ref = ref.gradient(w.astype(np.float64), X.astype(np.float64), T.astype(np.float64), M, K)
    g_gpu = g.cpu().numpy().astype(np.float64)
    # element by element: fp32 accumulation over 256 rows against fp64
    tol = 1e-4 * np.abs(g_ref) + 1e-5 * np.abs(g_ref).max()
    bad = np.flatnonzero(np.abs(g_gpu - g_ref) > tol)
    assert bad.size == 0, (bad[:10], g_gpu[bad[:10]], g_ref[bad[:10]])
    assert np.isclose(loss.item(), ref.loss(w.astype(np.float64), X, T, M, K), rtol=1e-4)


def test_forward_on_hand_built_network(gpu_lib):
    # the hand-built network of test_mlp_reference.py, whose outputs are known in closed form
    from paper_1707_02000_amd import tuner
    import torch

    from test_mlp_reference import hand_network, hand_outputs

    X = np.random.default_rng(9).normal(0, 6, (300, 6)).astype(np.float32)
    w = hand_network(K).astype(np.float32)
    Y = tuner.predict(torch.from_numpy(w).cuda(), X)
    assert np.allclose(Y, hand_outputs(X.astype(np.float64), K), rtol=1e-5, atol=1e-4)


def test_choose_matches_cpu_decision(gpu_lib):
    from paper_1707_02000_amd import tuner
    import torch

    w, X, _, _ = problem(3, n=500)
    ncurr = np.where(np.arange(500) % 3 == 0, 100000, 500).astype(np.int32)
    c, Y = tuner.choose_batch(torch.from_numpy(w).cuda(), X, ncurr)
    c_ref, Y_ref = ref.choose(w.astype(np.float64), X.astype(np.float64), ncurr, K)
    srt = np.sort(Y_ref, axis=1)
    rows = np.arange(500)
    h = np.where(ncurr <= 2048, 0, 2)
    gap = Y_ref[rows, h] - srt[:, 0] - ref.MARGIN
    clear = ((srt[:, 1] - srt[:, 0]) > 1e-3) & (np.abs(gap) > 1e-3)  # decisions not decided by rounding
    assert np.array_equal(c[clear], c_ref[clear])
    assert np.all(np.isin(c[ncurr > 2048], [2, 3, 4, 5]))


def test_training_fits_a_known_function(gpu_lib):
    from paper_1707_02000_amd import tuner

    rng = np.random.default_rng(4)
    X = rng.uniform(0, 10, (2000, 6)).astype(np.float32)
    T = np.stack([X[:, 0] * 0.5 + np.sin(X[:, 1]), X[:, 2] - X[:, 3], np.abs(X[:, 4] - 5), X[:, 5] ** 0.5,
                  X[:, 0] * 0.1, np.maximum(X[:, 1], X[:, 2]) * 0.3], axis=1).astype(np.float32)
    assert T.shape[1] == K
    M = (rng.random(T.shape) < 0.8).astype(np.float32)
    W, hist = tuner.train(X, T, M, steps=1500, lr=3e-3)
    assert hist[-1] < 0.05 * hist[0]
    w = W.cpu().numpy().astype(np.float64)
    assert ref.loss(w, X, T, M, K) < 0.05 * hist[0]


def test_learned_policy_keeps_output_bit_identical(gpu_lib):
    import torch

    g = gg.rmat(14, 16, seed=7)
    want = oracle.truss(g)
    w, _, _, _ = problem(5)
    # random weights: arbitrary launch choices, same trussness
    tau, st = gpu_lib.truss_decompose(g.offsets, g.adj, variant="learned", mlp_weights=torch.from_numpy(w).cuda(),
                                      return_stats=True)
    assert np.array_equal(tau.cpu().numpy(), want)
    say("choices under random weights", st["choice_count"])
    # NaN weights: every prediction fails and the heuristic takes over
    wn = np.full_like(w, np.nan)
    tau = gpu_lib.truss_decompose(g.offsets, g.adj, variant="learned", mlp_weights=torch.from_numpy(wn).cuda())
    assert np.array_equal(tau.cpu().numpy(), want)


def test_trained_model_gain_on_held_out_traces(gpu_lib):
    from paper_1707_02000_amd import tuner

    if not os.path.exists(tuner.DEFAULT_WEIGHTS):
        pytest.skip("no trained cost model shipped")
    W = tuner.load_weights()
    # workloads the model was not trained on: R-MAT scale 21 (another seed) and the
    # 64-graph batch recipe as one union graph
    rounds = []
    for g in (gg.rmat(21, 16, seed=2), gg.workload("batch64", seed=3).union()):
        rounds += tuner.collect_rounds(g.offsets, g.adj, repeats=2)
    choice = tuner.learned_choices(W, rounds)  # the model above the size the loop consults it at
    learned = tuner.evaluate(rounds, lambda r, it=iter(choice): int(next(it)))
    heur = tuner.evaluate(rounds, lambda r: tuner.heuristic_choice(r["frontier"]))
    departs = sum(int(c) != tuner.heuristic_choice(r["frontier"]) for c, r in zip(choice, rounds))
    say("held-out: learned", learned, "heuristic", heur, "rounds", len(rounds), "departures", departs)
    # the model's choices cost less than the heuristic's, and than picking at random
    assert departs > 0
    assert learned["total_us"] < heur["total_us"]
    rng = np.random.default_rng(0)
    rand = tuner.evaluate(rounds, lambda r: int(rng.choice(tuner.valid_choices(r["frontier"]))))
    assert learned["total_us"] < rand["total_us"]
