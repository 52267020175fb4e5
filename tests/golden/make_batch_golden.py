"""Writes the stored per-graph expectations for a packed batch workload.

For every graph of the named batch (graphgen.workload, seed 1) this runs the CPU
oracle (oracle.truss, the serial bucket peel) on that graph alone and records one
line: graph index, n, m, t_max and the sha256 of its int32 trussness array in output
edge order.  The graphs are independent, so they are spread over worker processes;
each oracle call stays serial.  Only graphgen (inputs) and oracle/ are used.

    python tests/golden/make_batch_golden.py batch4096 [workers]
"""
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

_BATCH = None


def _one(g_idx):
    g = _BATCH.graph(g_idx)
    t0 = time.time()
    tau = oracle.truss(g)
    dt = time.time() - t0
    h = hashlib.sha256(np.ascontiguousarray(tau, np.int32).tobytes()).hexdigest()
    return g_idx, g.n, g.m, int(tau.max()) if len(tau) else 0, h, dt


def main(name, workers):
    global _BATCH
    _BATCH = gg.workload(name, seed=1)
    G = _BATCH.num_graphs
    t0 = time.time()
    rows = [None] * G
    secs = 0.0
    # largest graphs first so the pool's tail is short
    order = sorted(range(G), key=lambda i: -int(_BATCH.adj_off[i + 1] - _BATCH.adj_off[i]))
    with mp.get_context("fork").Pool(workers) as pool:
        for k, r in enumerate(pool.imap_unordered(_one, order, chunksize=4)):
            rows[r[0]] = r
            secs += r[5]
            if (k + 1) % 256 == 0:
                print(f"{name}: {k + 1}/{G} graphs, {time.time() - t0:.0f}s", flush=True)
    h = hashlib.sha256()
    for r in rows:
        h.update(bytes.fromhex(r[4]))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.txt")
    with open(path, "w") as f:
        f.write(f"# {name} seed 1: {G} graphs, total m {int(_BATCH.total_m)}, "
                f"oracle {secs:.1f} s summed over graphs\n")
        f.write(f"# sha256 over the per-graph digests in graph order: {h.hexdigest()}\n")
        f.write("# graph n m t_max trussness_sha256\n")
        for r in rows:
            f.write(f"{r[0]} {r[1]} {r[2]} {r[3]} {r[4]}\n")
    print(f"{name}: {G} graphs, oracle {secs:.1f} s summed -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "batch4096", int(sys.argv[2]) if len(sys.argv) > 2 else 4)
