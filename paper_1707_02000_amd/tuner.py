"""Launch tuning of the peeling loop: timing traces, the autotuned heuristic, and the
learned cost model (an fp32 MLP trained on the GPU by libpkt's own kernels).

Every frontier round can be launched several ways (``CHOICES``); all give the same
trussness.  The frontier *sets* of a decomposition do not depend on how rounds are
launched, so runs that force each choice in turn, one round per launch sequence,
produce timings that line up round by round: for each round, the device time of
every valid choice, plus the frontier's features.  From those:

* ``autotune_threshold`` picks the frontier size up to which the fused launch is
  used (the built-in heuristic's rule) by least total time over the traces;
* ``train`` fits the cost model (features -> log2 microseconds per choice);
* ``evaluate`` scores a policy on traces: total time of its choices, and its
  regret against the best choice of every round.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

from . import CHOICES, MODEL_CHOICES, NUM_FEATURES, _check, _stream, _torch, alloc_workspace, load, truss_decompose

FUSED_LIMIT = 2048  # frontier edges the fused launch accepts
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
DEFAULT_WEIGHTS = os.path.join(DATA_DIR, "cost_model.json")


def valid_choices(frontier: int):
    return [c for c in range(MODEL_CHOICES) if c >= 2 or frontier <= FUSED_LIMIT]


def collect_rounds(offsets, adj, *, repeats: int = 1, capacity: int = 1 << 20):
    """Per-round timings of every launch choice on one graph (device tensors or arrays).

    Returns a list of rounds: {"round", "level", "frontier", "features", "us": {choice: us}}.
    """
    torch = _torch()
    off = offsets if hasattr(offsets, "is_cuda") else torch.from_numpy(np.asarray(offsets)).cuda()
    adj_t = adj if hasattr(adj, "is_cuda") else torch.from_numpy(np.asarray(adj)).cuda()
    per_choice = {}
    for c in range(MODEL_CHOICES):
        best = None
        for _ in range(max(1, repeats)):
            _, st = truss_decompose(off, adj_t, validate=False, force_choice=c, single_round=True,
                                    return_stats=True, trace_capacity=capacity)
            recs = {r["round_index"]: r for r in st["trace"] if r["kind"] != 0}
            if best is None:
                best = recs
            else:  # keep the fastest of the repeats, round by round
                for k, r in recs.items():
                    if k in best and r["ms"] < best[k]["ms"]:
                        best[k] = r
        per_choice[c] = best
    ref = per_choice[2]  # WIDE is valid for every round: take features from its run
    rounds = []
    for k in sorted(ref):
        r0 = ref[k]
        us = {}
        for c in range(MODEL_CHOICES):
            r = per_choice[c].get(k)
            if r is not None and r["choice"] == c:  # a forced choice that was invalid fell back
                us[c] = r["ms"] * 1e3
        rounds.append({"round": k, "level": r0["level"], "frontier": r0["frontier"],
                       "features": [float(x) for x in r0["features"][:NUM_FEATURES]], "us": us})
    return rounds


def dataset(rounds):
    """X (n, 6) features, T (n, K) log2 microseconds, M (n, K) measured mask, ncurr (n,)."""
    n, k = len(rounds), MODEL_CHOICES
    X = np.zeros((n, NUM_FEATURES), np.float32)
    T = np.zeros((n, k), np.float32)
    M = np.zeros((n, k), np.float32)
    nc = np.zeros(n, np.int32)
    for i, r in enumerate(rounds):
        X[i] = r["features"]
        nc[i] = r["frontier"]
        for c, us in r["us"].items():
            T[i, int(c)] = math.log2(max(us, 1e-3))
            M[i, int(c)] = 1.0
    return X, T, M, nc


HEURISTIC_THRESHOLD = 2048  # the library's built-in rule (see autotune_threshold)


def heuristic_choice(frontier: int, threshold: int = HEURISTIC_THRESHOLD) -> int:
    return 0 if frontier <= threshold else 2


def evaluate(rounds, choose):
    """Total microseconds of a policy's choices, and its regret against the best per round.

    ``choose(round) -> choice``; a choice with no measurement for a round falls back to WIDE.
    """
    total = best = 0.0
    for r in rounds:
        us = {int(c): v for c, v in r["us"].items()}
        c = choose(r)
        total += us.get(c, us.get(2, 0.0))
        best += min(us.values()) if us else 0.0
    return {"total_us": total, "best_us": best, "regret_us": total - best}


def autotune_threshold(rounds, candidates=(0, 64, 128, 256, 512, 1024, 2048)):
    """Fused-vs-wide frontier threshold with the least total time over the traces."""
    scores = {t: evaluate(rounds, lambda r, t=t: heuristic_choice(r["frontier"], t))["total_us"] for t in candidates}
    return min(scores, key=scores.get), scores


def _dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def train(X, T, M, *, steps: int = 3000, lr: float = 3e-3, seed: int = 1):
    """Fits the cost model on the GPU (libpkt's forward / backward / Adam kernels)."""
    torch = _torch()
    lib = load()
    n = int(X.shape[0])
    Xd, Td, Md = _dev(X, torch), _dev(T, torch), _dev(M, torch)
    W = torch.zeros(lib.truss_mlp_num_params(), dtype=torch.float32, device="cuda")
    s = _stream(torch, None)
    _check(lib.truss_mlp_init(ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Td.data_ptr()),
                              ctypes.c_void_p(Md.data_ptr()), n, seed, ctypes.c_void_p(W.data_ptr()), s))
    nb = lib.truss_mlp_workspace_bytes(n)
    _buf, wptr = alloc_workspace(nb)
    hist = torch.zeros(max(steps, 1), dtype=torch.float32, device="cuda")
    _check(lib.truss_mlp_train(ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Td.data_ptr()),
                               ctypes.c_void_p(Md.data_ptr()), n, ctypes.c_void_p(W.data_ptr()), steps, lr,
                               ctypes.c_void_p(hist.data_ptr()), ctypes.c_void_p(wptr), nb, s))
    return W, hist[:steps].cpu().numpy()


def predict(W, X):
    """Model outputs (n, K) through libpkt's batched forward."""
    torch = _torch()
    lib = load()
    n = int(X.shape[0])
    Xd = _dev(np.asarray(X, np.float32), torch)
    Y = torch.empty((n, MODEL_CHOICES), dtype=torch.float32, device="cuda")
    nb = lib.truss_mlp_workspace_bytes(n)
    _buf, wptr = alloc_workspace(nb)
    _check(lib.truss_mlp_forward(ctypes.c_void_p(Xd.data_ptr()), n, ctypes.c_void_p(W.data_ptr()),
                                 ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(wptr), nb, _stream(torch, None)))
    return Y.cpu().numpy()


def choose_batch(W, X, ncurr):
    """The peeling loop's own decision routine on many feature rows."""
    torch = _torch()
    lib = load()
    n = int(X.shape[0])
    Xd = _dev(np.asarray(X, np.float32), torch)
    Nd = _dev(np.asarray(ncurr, np.int32), torch)
    C = torch.empty(n, dtype=torch.int32, device="cuda")
    Y = torch.empty((n, MODEL_CHOICES), dtype=torch.float32, device="cuda")
    _check(lib.truss_mlp_choose(ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(Nd.data_ptr()), n,
                                ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                                ctypes.c_void_p(Y.data_ptr()), _stream(torch, None)))
    return C.cpu().numpy(), Y.cpu().numpy()


LEARNED_MIN_FRONTIER = 32768  # the library consults the model above this frontier size


def learned_choices(W, rounds):
    """The learned policy's choice for every traced round, as the peeling loop makes it:
    the model above LEARNED_MIN_FRONTIER frontier edges, the heuristic below."""
    X, _, _, nc = dataset(rounds)
    c, _ = choose_batch(W, X, nc)
    return [int(ci) if r["frontier"] > LEARNED_MIN_FRONTIER else heuristic_choice(r["frontier"])
            for ci, r in zip(c, rounds)]


def save_weights(W, path=DEFAULT_WEIGHTS, meta=None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    w = W.cpu().numpy() if hasattr(W, "cpu") else np.asarray(W)
    with open(path, "w") as f:
        json.dump({"weights": [float(x) for x in w], "meta": meta or {}}, f)


def load_weights(path=DEFAULT_WEIGHTS):
    """Cost-model weights as a CUDA float32 tensor (raises if the file is missing)."""
    torch = _torch()
    d = json.load(open(path))
    w = np.asarray(d["weights"], np.float32)
    if len(w) != load().truss_mlp_num_params():
        raise ValueError(f"{path}: {len(w)} weights, the model has {load().truss_mlp_num_params()}")
    return torch.from_numpy(w).cuda()


def _graph_for(name):
    import graphgen as gg

    if name.startswith("batch"):
        return gg.workload(name, seed=1).union()
    return gg.workload(name, seed=1)


def evaluate_weights(path, train, held_out, repeats=2, report_path=None):
    """The learned policy of the weights at path against the heuristic, on fresh traces of
    every named graph (the training graphs and the held-out ones), as the loop makes it."""
    import time

    W = load_weights(path)
    report = {"weights": os.path.basename(path), "learned_min_frontier": LEARNED_MIN_FRONTIER,
              "meta": json.load(open(path)).get("meta", {}), "train": {}, "held_out": {}}
    for part, names in (("train", train), ("held_out", held_out)):
        for name in names:
            g = _graph_for(name)
            t0 = time.time()
            r = collect_rounds(g.offsets, g.adj, repeats=repeats)
            it = iter(learned_choices(W, r))
            report[part][name] = {"rounds": len(r), "learned": evaluate(r, lambda q: int(next(it))),
                                  "heuristic": evaluate(r, lambda q: heuristic_choice(q["frontier"]))}
            print(part, name, f"{time.time() - t0:.1f}s", report[part][name], flush=True)
    if report_path:
        with open(report_path, "w") as f:
            json.dump(report, f, indent=1)
    return report


def main(argv=None):
    """python -m paper_1707_02000_amd.tuner --train er4096 rmat20 chunglu20 batch256 --held-out rmat24"""
    import argparse
    import time

    ap = argparse.ArgumentParser()
    ap.add_argument("--train", nargs="+", default=["er4096", "rmat20", "chunglu20", "batch256"])
    ap.add_argument("--held-out", nargs="*", default=["rmat22"])
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--evaluate", default=None,
                    help="score these weights on fresh traces of the --train and --held-out graphs "
                         "instead of training")
    args = ap.parse_args(argv)
    if args.evaluate:
        return evaluate_weights(args.evaluate, args.train, args.held_out, args.repeats, args.report)
    train_rounds, report = [], {"train": {}, "held_out": {}}
    for name in args.train:
        g = _graph_for(name)
        t0 = time.time()
        r = collect_rounds(g.offsets, g.adj, repeats=args.repeats)
        train_rounds += r
        print(f"traces {name}: {len(r)} rounds in {time.time() - t0:.1f}s", flush=True)
    thr, scores = autotune_threshold(train_rounds)
    X, T, M, nc = dataset(train_rounds)
    W, hist = train(X, T, M, steps=args.steps, lr=args.lr)
    it = iter(learned_choices(W, train_rounds))
    report["autotuned_threshold"] = thr
    report["threshold_scores_us"] = {str(k): v for k, v in scores.items()}
    report["train"] = {"rounds": len(train_rounds), "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
                       "learned": evaluate(train_rounds, lambda r: int(next(it))),
                       "heuristic": evaluate(train_rounds, lambda r: heuristic_choice(r["frontier"], thr))}
    print("train", report["train"], "threshold", thr, flush=True)
    for name in args.held_out:
        g = _graph_for(name)
        r = collect_rounds(g.offsets, g.adj, repeats=args.repeats)
        it = iter(learned_choices(W, r))
        report["held_out"][name] = {"rounds": len(r), "learned": evaluate(r, lambda q: int(next(it))),
                                    "heuristic": evaluate(r, lambda q: heuristic_choice(q["frontier"], thr))}
        print("held out", name, report["held_out"][name], flush=True)
    save_weights(W, args.out, meta={"train": args.train, "steps": args.steps, "lr": args.lr,
                                    "autotuned_threshold": thr})
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    main()
