"""Writes the stored expectations for the full-size parity tests.

For each named synthetic workload (graphgen recipes, seed 1) this runs the CPU
oracle (oracle.truss, the serial bucket peel) and records the input's sha256, m, the
sha256 of the int32 trussness array in output edge order, t_max, the trussness
histogram and the triangle count.  Only graphgen (inputs) and oracle/ are used.

    python tests/golden/make_golden.py rmat20 [more workloads ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def main(names):
    for name in names:
        g = gg.workload(name, seed=1)
        t0 = time.time()
        tau, S0 = oracle.truss(g, with_support=True)
        dt = time.time() - t0
        rec = {
            "workload": name,
            "seed": 1,
            "n": int(g.n),
            "m": int(g.m),
            "csr_sha256": g.sha256(),
            "trussness_sha256": hashlib.sha256(np.ascontiguousarray(tau, np.int32).tobytes()).hexdigest(),
            "support_sha256": hashlib.sha256(np.ascontiguousarray(S0, np.int32).tobytes()).hexdigest(),
            "t_max": int(tau.max()) if len(tau) else 0,
            "triangles": int(S0.sum()) // 3,
            "histogram": np.bincount(tau).tolist() if len(tau) else [],
            "oracle_seconds": round(dt, 2),
        }
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"{name}: m={g.m} t_max={rec['t_max']} oracle {dt:.1f}s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["er4096", "rmat16"])
