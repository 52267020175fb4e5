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


def hand_network(k=K):
    """A network whose outputs are known in closed form (every layer, bias, ReLU and the
    input normalisation take part; weight matrices are read as [out][in]):
      xn = (X - mu) / sig, with mu = 1, sig = 2
      h1[i] = relu(xn_i), h1[6 + i] = relu(-xn_i)            (i < 6; other units get bias -1)
      h2[i] = relu(h1[i] + h1[6 + i]) = |xn_i|, h2[7] = relu(0.5)
      h3[0] = sum_i |xn_i|, h3[1] = 2 * h2[7] = 1, h3[2] = relu(|xn_0| - 3)
      y0 = h3[0] + 0.25, y1 = 3 h3[1], y2 = h3[2], y3 = -h3[0], y4 = h3[0] - h3[2] + 1
    """
    lay, total = mlp.layout(k)
    w = np.zeros(total)

    def put(name, arr):
        a, b = lay[name]
        w[a:b] = np.asarray(arr, dtype=np.float64).ravel()

    H, IN = mlp.H, mlp.IN
    put("mu", np.ones(IN))
    put("sig", np.full(IN, 2.0))
    W1 = np.zeros((H, IN))
    b1 = np.full(H, -1.0)
    for i in range(IN):
        W1[i, i] = 1.0
        W1[IN + i, i] = -1.0
        b1[i] = b1[IN + i] = 0.0
    W2 = np.zeros((H, H))
    b2 = np.zeros(H)
    for i in range(IN):
        W2[i, i] = W2[i, IN + i] = 1.0
    b2[7] = 0.5
    W3 = np.zeros((H, H))
    b3 = np.zeros(H)
    W3[0, :IN] = 1.0
    W3[1, 7] = 2.0
    W3[2, 0] = 1.0
    b3[2] = -3.0
    W4 = np.zeros((k, H))
    b4 = np.zeros(k)
    W4[0, 0] = 1.0
    b4[0] = 0.25
    W4[1, 1] = 3.0
    W4[2, 2] = 1.0
    W4[3, 0] = -1.0
    W4[4, 0], W4[4, 2], b4[4] = 1.0, -1.0, 1.0
    for name, arr in (("W1", W1), ("b1", b1), ("W2", W2), ("b2", b2), ("W3", W3), ("b3", b3),
                      ("W4", W4), ("b4", b4)):
        put(name, arr)
    return w


def hand_outputs(X, k=K):
    xn = (np.asarray(X, np.float64) - 1.0) / 2.0
    s = np.abs(xn).sum(axis=1)
    r = np.maximum(np.abs(xn[:, 0]) - 3.0, 0.0)
    y = np.zeros((len(xn), k))
    y[:, 0] = s + 0.25
    y[:, 1] = 3.0
    y[:, 2] = r
    y[:, 3] = -s
    y[:, 4] = s - r + 1.0
    return y


def test_forward_on_a_hand_built_network():
    # parity pin of the forward pass independent of its own gradient
    rng = np.random.default_rng(7)
    X = rng.normal(0, 6, (64, mlp.IN))
    X[0] = [1, 1, 1, 1, 1, 1]  # xn = 0: every unit at its bias
    X[1] = [20, -3, 5, 1, 0, 9]
    y, _ = mlp.forward(hand_network(), X, K)
    assert np.allclose(y, hand_outputs(X), rtol=0, atol=1e-12)
    assert np.allclose(y[0], [0.25, 3.0, 0.0, 0.0, 1.0])
    # |xn| = 9.5, 2, 2, 0, 0.5, 4 -> sum 18, relu(9.5 - 3) = 6.5
    assert np.allclose(y[1], [18.25, 3.0, 6.5, -18.0, 12.5])


def test_forward_hand_network_detects_layout_mistakes():
    # a transposed hidden matrix or a dropped bias changes the hand network's outputs
    X = np.random.default_rng(8).normal(0, 6, (32, mlp.IN))
    w = hand_network()
    lay, _ = mlp.layout(K)
    a, b = lay["W2"]
    wt = w.copy()
    wt[a:b] = w[a:b].reshape(mlp.H, mlp.H).T.ravel()
    assert not np.allclose(mlp.forward(wt, X, K)[0], hand_outputs(X))
    a, b = lay["b3"]
    wb = w.copy()
    wb[a:b] = 0.0
    assert not np.allclose(mlp.forward(wb, X, K)[0], hand_outputs(X))
