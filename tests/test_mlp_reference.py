"""The CPU fp64 reference of the cost model, pinned by central finite differences
(and by the definition of the masked loss); the GPU kernels are checked against it
in test_gpu_learned.py."""
import numpy as np

from oracle import mlp

K = 5


def random_problem(seed, n=40):
    rng = np.random.default_rng(seed)
    _, total = mlp.layout(K)
    w = rng.normal(0, 0.3, total)
    lay, _ = mlp.layout(K)
    a, b = lay["sig"]
    w[a:b] = rng.uniform(0.5, 2.0, b - a)
    X = rng.normal(0, 2, (n, mlp.IN))
    T = rng.normal(0, 1, (n, K))
    M = (rng.random((n, K)) < 0.7).astype(float)
    return w, X, T, M


def test_gradient_matches_central_differences():
    w, X, T, M = random_problem(1)
    g = mlp.gradient(w, X, T, M, K)
    lay, _ = mlp.layout(K)
    rng = np.random.default_rng(2)
    idx = rng.choice(np.arange(lay["W1"][0], len(w)), 200, replace=False)
    h = 1e-6
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss(wp, X, T, M, K) - mlp.loss(wm, X, T, M, K)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])
    a, b = lay["sig"]
    assert np.all(g[: b] == 0)  # normalisation is not trained


def test_loss_definition_and_mask():
    w, X, T, M = random_problem(3, n=10)
    y, _ = mlp.forward(w, X, K)
    want = sum((y[i, k] - T[i, k]) ** 2 for i in range(10) for k in range(K) if M[i, k]) / M.sum()
    assert np.isclose(mlp.loss(w, X, T, M, K), want)
    # entries outside the mask do not affect loss or gradient
    T2 = T.copy()
    T2[M == 0] += 100.0
    assert np.isclose(mlp.loss(w, X, T2, M, K), mlp.loss(w, X, T, M, K))
    assert np.allclose(mlp.gradient(w, X, T2, M, K), mlp.gradient(w, X, T, M, K))


def test_choose_respects_validity():
    w, X, T, M = random_problem(4, n=50)
    ncurr = np.where(np.arange(50) % 2 == 0, 100, 100000)
    c, y = mlp.choose(w, X, ncurr, K)
    assert np.all(np.isin(c[ncurr > 2048], [2, 3, 4]))
    rows = np.arange(50)
    h = np.where(ncurr <= 2048, 0, 2)
    best = np.argmin(y, axis=1)
    departs = y[rows, best] + mlp.MARGIN < y[rows, h]
    assert np.all(c[departs] == best[departs]) and np.all(c[~departs] == h[~departs])
    # with no margin the rule is the plain argmin over valid choices
    c0, y0 = mlp.choose(w, X, ncurr, K, margin=0.0)
    assert np.all(c0 == np.argmin(y0, axis=1))
    # a non-finite output keeps the heuristic's launch
    w_bad = w.copy()
    w_bad[-1] = np.nan
    cb, _ = mlp.choose(w_bad, X, ncurr, K)
    assert np.all(cb == h)
