"""Benchmark: truss-decomposed edges/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat20]

A step is one whole truss decomposition (the degree-order relabelling, edge ids,
orientation, support, every level scan and sub-level, the map back to the input's
edge order) of one synthetic graph that is already resident
in device memory, through the library's C ABI with input validation off (the input
is validated once, outside the timed region, and the result is checked against the
stored oracle expectation when one exists).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "er4096": "Erdos-Renyi G(n=4096, mean degree 16), seed 1",
    "rmat20": "R-MAT scale 20, edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), symmetrized, dedup, "
              "self-loops removed, ids permuted, seed 1",
    "rmat24": "R-MAT scale 24, edge factor 16, same recipe, seed 1",
    "chunglu23": "Chung-Lu n=2^23, exponent 2.1, ~1e8 edges, 200 planted cliques of 50..500, seed 1",
}


METRIC = "truss-decomposed edges/s, R-MAT s20/s24; batched+learned vs plain, 1 MI355X"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Algorithmic bytes of the wide sub-level kernel (one item = one entry of the shorter
# working row searched in the longer row).  Model of the hot-path plan (4 B ids): the
# shorter-row entry (4 B) and the longer-row entry the search lands on (4 B) per item;
# per frontier edge: its id (4 B), endpoints (8 B) and four row offsets (32 B).
BYTES_PER_ITEM = 8
BYTES_PER_FRONTIER_EDGE = 44
# A fuller model also counts the entry's edge id and that edge's state byte (13 B per item).
BYTES_PER_ITEM_FULL = 13


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, np.int32).tobytes()).hexdigest()


def measured_traffic(workload):
    """HBM-side bytes per launch of the dominant kernel from the committed counter summary,
    or None if there is none for this workload or the kernel's sources changed since."""
    path = os.path.join(ROOT, "profiles", f"k_psl_bsearch_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = dict(l.split(" = ", 1) for l in open(path).read().splitlines() if " = " in l)
    csrc = os.path.join(ROOT, "paper_1707_02000_amd", "csrc")
    src = "".join(open(os.path.join(csrc, f)).read()
                  for f in ("common.h", "truss.h", "peel.h", "scan.h", "psl.h", "peel.hip", "relabel.hip", "kco.hip"))
    if hashlib.sha256(src.encode()).hexdigest()[:16] != fields.get("source_sha256_16", "").strip():
        return None
    return float(fields["traffic_bytes_per_launch"])


_CPU_CHILD = r"""
import json, os, sys, time
sys.path.insert(0, sys.argv[1])
cpu = sorted(os.sched_getaffinity(0))[-1]
os.sched_setaffinity(0, {cpu})  # one host core
import graphgen as gg
import oracle
g = gg.workload(sys.argv[2], seed=1)
oracle.truss(gg.er(64, mean_degree=4.0, seed=1))  # library loaded before the clock starts
t0 = time.perf_counter()
oracle.truss(g)
print(json.dumps({"m": g.m, "s": time.perf_counter() - t0, "cpu": cpu}))
"""


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample_name="rmat17"):
    """The CPU oracle (serial bucket peel) on one pinned host core, in a child process, on a
    bounded sample of the same recipe (R-MAT scale 17: about 20 s of one core)."""
    import subprocess

    r = subprocess.run([sys.executable, "-c", _CPU_CHILD, ROOT, sample_name], capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline child failed: {r.stderr[-2000:]}")
    d = json.loads(r.stdout.strip().splitlines()[-1])
    out = {"value": d["m"] / d["s"], "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": f"{sample_name}: R-MAT scale {sample_name[4:]}, edge factor 16, same (a,b,c,d) recipe, seed 1 "
                     f"(m={d['m']}); one full serial decomposition on one pinned core, {d['s']:.1f} s",
           "host_nproc": os.cpu_count(), "host_affinity": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model()}
    for name in ("rmat20", "rmat24"):  # the stored full-size runs, as context (another host, same oracle)
        gold = os.path.join(ROOT, "tests", "golden", f"{name}.json")
        if os.path.exists(gold):
            rec = json.load(open(gold))
            out[f"context_{name}_oracle"] = {"seconds": rec["oracle_seconds"],
                                             "edges_per_s": rec["m"] / rec["oracle_seconds"]}
    return out


def graph_work(g):
    """Host-side work measures of a CSR: W+ = sum_v d+(v) d-(v) under the (degree, id)
    orientation (the support walk), W_min = sum over edges of the smaller degree."""
    deg = np.diff(g.offsets).astype(np.int64)
    u = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    v = g.adj.astype(np.int64)
    up = (deg[u] < deg[v]) | ((deg[u] == deg[v]) & (u < v))  # slot u -> v points up in rank
    dplus = np.bincount(u[up], minlength=g.n).astype(np.int64)
    wplus = int((dplus * (deg - dplus)).sum())
    half = u < v
    wmin = int(np.minimum(deg[u[half]], deg[v[half]]).sum())
    return wplus, wmin


def model_bytes(g, stats, wplus, wmin):
    """Algorithmic bytes of one decomposition under the hot-path plan's per-phase models."""
    m, n, T = g.m, g.n, stats["triangles"]
    build = 32 * m + 8 * n
    support = 4 * (m + wplus) + 36 * T
    scan = 5 * m
    peel = 4 * wmin + 44 * m
    return {"build": build, "support": support, "scan": scan, "peel": peel, "total": build + support + scan + peel}


def _timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def extras(pkt, torch, gg, off20, adj20, m20, ms20, steps):
    """The other parts of the metric: the level loop's drivers, the k-truss listing, core
    numbers, KCO reordering, the local h-index iteration, learned dispatch vs the plain heuristic (R-MAT s20 and s24), R-MAT s24 itself,
    and batched (one union level loop) vs one graph after another.  Inputs resident, as
    for the main line."""
    from paper_1707_02000_amd import tuner

    out = {}
    # the main line without the library's degree-order relabelling (same output)
    t = _timed(lambda: pkt.truss_decompose(off20, adj20, validate=False, relabel=False), steps, 1, torch)
    out["no_relabel_rmat20"] = {"ms_per_step": round(t * 1e3, 2), "value": m20 / t, "relabel_gain": t * 1e3 / ms20}
    print(f"bench: rmat20 without relabelling {t * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # the level loop's drivers on the same graph (pipelined is the main line's)
    drivers = {}
    for mode in ("host", "device", "graph", "pipelined"):
        t = _timed(lambda: pkt.truss_decompose(off20, adj20, validate=False, device_loop=mode), 2, 1, torch)
        drivers[mode] = round(t * 1e3, 2)
    out["loop_drivers_rmat20_ms"] = drivers
    print(f"bench: loop drivers rmat20 {drivers}", file=sys.stderr, flush=True)
    # the maximal k-trusses from the trussness (three passes over the edges, two over
    # the vertices: 32 B per edge and 16 B per vertex algorithmic)
    tau20 = pkt.truss_decompose(off20, adj20, validate=False)
    el20 = pkt.edge_list(off20, adj20)
    n20 = int(off20.numel()) - 1
    tmax = int(tau20.max().item())
    kt = {}
    for k in (3, tmax // 2, tmax):
        t = _timed(lambda: pkt.ktruss(n20, el20, tau20, k), 3, 1, torch)
        _, cnt = pkt.ktruss(n20, el20, tau20, k)
        gbs = (32 * m20 + 16 * n20) / t / 1e9
        kt[str(k)] = {"ms": round(t * 1e3, 3), "trusses": cnt, "edges_per_s": m20 / t, "GB/s": gbs,
                      "frac_of_hbm": gbs / HBM_PEAK_GBS}
    out["ktruss_rmat20"] = kt
    print(f"bench: k-truss listing rmat20 { {k: v['ms'] for k, v in kt.items()} } ms", file=sys.stderr, flush=True)
    # core numbers (level-synchronous vertex peeling; the host reads counters each round)
    tk = _timed(lambda: pkt.kcore(off20, adj20), 3, 1, torch)
    _, cmax = pkt.kcore(off20, adj20)
    out["kcore_rmat20"] = {"ms": round(tk * 1e3, 3), "max_core": cmax, "edges_per_s": m20 / tk}
    # KCO reordering (Table 2's increasing core order) and the decomposition of the relabelled graph
    core20, _ = pkt.kcore(off20, adj20)
    to = _timed(lambda: pkt.kco_order(core20), 3, 1, torch)
    nid, order = pkt.kco_order(core20)
    tr = _timed(lambda: pkt.kco_relabel(off20, adj20, nid, order), 3, 1, torch)
    off2, adj2 = pkt.kco_relabel(off20, adj20, nid, order)
    td = _timed(lambda: pkt.truss_decompose(off2, adj2, validate=False, relabel=False), 2, 1, torch)
    tau2 = pkt.truss_decompose(off2, adj2, validate=False, relabel=False)
    tm = _timed(lambda: pkt.kco_map(n20, el20, nid, off2, adj2, tau2), 3, 1, torch)
    same = bool(torch.equal(pkt.kco_map(n20, el20, nid, off2, adj2, tau2), tau20))
    out["kco_rmat20"] = {"order_ms": round(to * 1e3, 3), "relabel_ms": round(tr * 1e3, 3),
                         "decompose_relabelled_ms": round(td * 1e3, 3), "map_ms": round(tm * 1e3, 3),
                         "trussness_unchanged": same}
    print(f"bench: kcore + KCO rmat20 {out['kcore_rmat20']['ms']} ms, {out['kco_rmat20']}", file=sys.stderr, flush=True)
    # the local h-index iteration on the same graph (one run: it takes seconds)
    t0 = time.perf_counter()
    tau_h, hs, hc = pkt.hindex(off20, adj20)
    torch.cuda.synchronize()
    th = time.perf_counter() - t0
    out["hindex_rmat20"] = {"ms": round(th * 1e3, 1), "sweeps": hs, "converged": hc,
                            "same_as_pkt": bool(torch.equal(tau_h, tau20)), "vs_pkt_time": th / (ms20 / 1e3)}
    print(f"bench: h-index rmat20 {out['hindex_rmat20']}", file=sys.stderr, flush=True)
    del tau_h
    del core20, nid, order, off2, adj2, tau2, tau20, el20
    print(f"bench: k-core rmat20 {tk * 1e3:.2f} ms, max core {cmax}", file=sys.stderr, flush=True)
    W = tuner.load_weights()
    t = _timed(lambda: pkt.truss_decompose(off20, adj20, validate=False, variant="learned", mlp_weights=W),
               steps, 1, torch)
    out["learned_rmat20"] = {"value": m20 / t, "ms_per_step": t * 1e3, "vs_plain": ms20 / (t * 1e3)}
    print(f"bench: learned rmat20 {t * 1e3:.1f} ms", file=sys.stderr, flush=True)

    for name in ("rmat24", "chunglu23", "er4096"):
        g = gg.workload(name, seed=1)
        off = torch.from_numpy(g.offsets).cuda()
        adj = torch.from_numpy(g.adj).cuda()
        ws = pkt.Workspace.for_graph(g.n, len(g.adj))
        o = torch.empty(max(g.m, 1), dtype=torch.int32, device="cuda")
        ref, st = pkt.truss_decompose(off, adj, validate=True, workspace=ws, out=o, return_stats=True)
        ref = ref.clone()
        reps = 2 if g.m > 5e7 else 5
        tp = _timed(lambda: pkt.truss_decompose(off, adj, validate=False, workspace=ws, out=o), reps, 1, torch)
        tl = _timed(lambda: pkt.truss_decompose(off, adj, validate=False, workspace=ws, out=o, variant="learned",
                                                mlp_weights=W), reps, 1, torch)
        tn = _timed(lambda: pkt.truss_decompose(off, adj, validate=False, workspace=ws, out=o, relabel=False),
                    reps, 1, torch)
        same = bool(torch.equal(o[:g.m], ref[:g.m]))
        gold = os.path.join(ROOT, "tests", "golden", f"{name}.json")
        parity = None
        if os.path.exists(gold):
            rec = json.load(open(gold))
            parity = rec["csr_sha256"] == g.sha256() and rec["trussness_sha256"] == sha(ref[:g.m].cpu().numpy())
        out[name] = {"m": g.m, "value": g.m / tp, "ms_per_step": tp * 1e3, "t_max": st["t_max"],
                     "levels": st["levels"], "sublevels": st["sublevels"], "parity_vs_oracle": parity,
                     "learned_value": g.m / tl, "learned_vs_plain": tp / tl, "learned_bit_identical": same,
                     "no_relabel_ms_per_step": tn * 1e3, "relabel_gain": tn / tp}
        print(f"bench: {name} plain {tp * 1e3:.1f} ms learned {tl * 1e3:.1f} ms no relabel {tn * 1e3:.1f} ms "
              f"parity {parity}", file=sys.stderr,
              flush=True)
        del off, adj, ws, o, ref
        torch.cuda.empty_cache()

    b = gg.workload("batch4096", seed=1)
    args_b = [torch.from_numpy(x).cuda() for x in (b.vtx_off, b.adj_off, b.offsets, b.adj)]
    tb = _timed(lambda: pkt.truss_decompose_batched(*args_b, validate=False), 2, 1, torch)
    tbl = _timed(lambda: pkt.truss_decompose_batched(*args_b, validate=False, variant="learned", mlp_weights=W),
                 2, 1, torch)
    tbp = _timed(lambda: pkt.truss_decompose_batched(*args_b, validate=False, mode="persistent"), 2, 1, torch)
    G = 256  # the sequential comparison on the first graphs (one after another is slow)
    sub = [torch.from_numpy(x).cuda() for x in
           (b.vtx_off[:G + 1], b.adj_off[:G + 1], b.offsets[:int(b.vtx_off[G])], b.adj[:int(b.adj_off[G])])]
    m_sub = int(b.adj_off[G]) // 2
    tu = _timed(lambda: pkt.truss_decompose_batched(*sub, validate=False), 2, 1, torch)
    tsq = _timed(lambda: pkt.truss_decompose_batched(*sub, validate=False, sequential=True), 1, 1, torch)
    out["batch4096"] = {"graphs": b.num_graphs, "m": b.total_m, "value": b.total_m / tb, "ms_per_step": tb * 1e3,
                        "learned_value": b.total_m / tbl, "learned_vs_plain": tb / tbl,
                        "persistent_value": b.total_m / tbp, "persistent_vs_union": tb / tbp,
                        "first_256": {"m": m_sub, "union_value": m_sub / tu, "sequential_value": m_sub / tsq,
                                      "union_vs_sequential": tsq / tu}}
    print(f"bench: batch4096 union {tb * 1e3:.0f} ms, learned {tbl * 1e3:.0f} ms, persistent {tbp * 1e3:.0f} ms; "
          f"first 256 union {tu * 1e3:.1f} ms sequential {tsq * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--loop", default="pipelined", choices=["host", "device", "graph", "pipelined"],
                    help="level-loop driver: host reads state per launch sequence; device/graph run gated steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the learned / R-MAT s24 / batched comparison fields")
    ap.add_argument("--profile-batch", action="store_true",
                    help="only decompose the 4096-graph batch once as one union and once with the persistent "
                         "launch (validation off), for a kernel-time profile of the batched modes")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (5 times), to scale "
                         "the FETCH_SIZE / WRITE_SIZE hardware counters")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch

        src = torch.ones(args.calibrate_copy_mib * (1 << 20) // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 5}))
        return
    if args.profile_batch:
        import torch

        import graphgen as gg
        import paper_1707_02000_amd as pkt

        b = gg.workload("batch4096", seed=1)
        dev = [torch.from_numpy(x).cuda() for x in (b.vtx_off, b.adj_off, b.offsets, b.adj)]
        out = {}
        for mode in ("union", "persistent"):
            t0 = time.perf_counter()
            pkt.truss_decompose_batched(*dev, validate=False, mode=mode)
            torch.cuda.synchronize()
            out[mode + "_s"] = time.perf_counter() - t0
        print(json.dumps({"graphs": b.num_graphs, "m": b.total_m, **out}))
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs one decomposition on one GPU (got --gpus {args.gpus}); "
              "sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen as gg
    import paper_1707_02000_amd as pkt

    pkt.load()
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = gg.workload(args.workload, seed=1)
    gen_s = time.perf_counter() - t0
    print(f"bench: {args.workload} n={g.n} m={g.m} generated in {gen_s:.1f}s", file=sys.stderr, flush=True)
    off = torch.from_numpy(g.offsets).cuda()
    adj = torch.from_numpy(g.adj).cuda()
    ws = pkt.Workspace.for_graph(g.n, len(g.adj))
    out = torch.empty(max(g.m, 1), dtype=torch.int32, device="cuda")

    # untimed: validation + parity against the stored oracle result
    tau, st0 = pkt.truss_decompose(off, adj, validate=True, variant=args.variant, workspace=ws, out=out,
                                   return_stats=True, device_loop=args.loop)
    tau_h = tau.cpu().numpy()
    parity = None
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    if os.path.exists(gold):
        rec = json.load(open(gold))
        parity = rec["csr_sha256"] == g.sha256() and rec["trussness_sha256"] == sha(tau_h)
    print(f"bench: first run stats {st0} parity={parity}", file=sys.stderr, flush=True)

    def step():
        return pkt.truss_decompose(off, adj, validate=False, variant=args.variant, workspace=ws, out=out,
                                   return_stats=True, profile=True, device_loop=args.loop)[1]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1000.0 / args.steps
    value = g.m / (ms / 1000.0)
    phases = {k: round(float(np.mean([s[k] for s in stats])), 3)
              for k in ("ms_build", "ms_support", "ms_peel", "ms_total")}
    deg = g.degrees()
    # dominant kernel: the wide sub-level intersection kernel; its launches are timed
    # with HIP events on the library's stream inside the timed steps
    launches = sum(s["wide_timed"] for s in stats)
    dom_ms = sum(s["wide_ms"] for s in stats)
    items = sum(s["wide_items"] for s in stats)
    frontier = sum(s["wide_frontier"] for s in stats)
    alg_bytes = BYTES_PER_ITEM * items + BYTES_PER_FRONTIER_EDGE * frontier
    roofline = None
    if launches and dom_ms > 0:
        achieved = alg_bytes / launches / (dom_ms / launches / 1e3) / 1e9
        full = (BYTES_PER_ITEM_FULL * items + BYTES_PER_FRONTIER_EDGE * frontier) / (dom_ms / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload),
                    "kernel": "k_psl_bsearch", "launches_per_step": launches / args.steps,
                    "avg_launch_us": dom_ms / launches * 1e3,
                    "alg_bytes_per_launch": alg_bytes / launches,
                    "model": f"{BYTES_PER_ITEM} B per shorter-row entry searched (the entry and the longer-row "
                             f"entry its search lands on) + {BYTES_PER_FRONTIER_EDGE} B per frontier edge",
                    "frac_full_model": full / HBM_PEAK_GBS,
                    "full_model": f"{BYTES_PER_ITEM_FULL} B per entry (also its edge id and state byte)"}
    # the whole step and the support kernel against the same roofline, by the per-phase models
    wplus, wmin = graph_work(g)
    mb = model_bytes(g, st0, wplus, wmin)
    step_frac = mb["total"] / (ms / 1e3) / 1e9 / HBM_PEAK_GBS
    sup_ms = phases["ms_support"]
    support_roofline = {"kernel": "k_support", "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                        "alg_bytes": mb["support"], "ms": sup_ms,
                        "achieved": mb["support"] / (sup_ms / 1e3) / 1e9 if sup_ms > 0 else None,
                        "frac": mb["support"] / (sup_ms / 1e3) / 1e9 / HBM_PEAK_GBS if sup_ms > 0 else None,
                        "model": "4 (m + W+) B of rows + 36 B per triangle", "W_plus": wplus}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "n": g.n, "m": g.m,
                   "variant": args.variant, "loop": args.loop, "relabel": "auto (degree order)"},
        "parity_vs_oracle": parity,
        "wedges_per_s": pkt.wedges(deg) / (ms / 1000.0),
        "t_max": st0["t_max"],
        "levels": st0["levels"],
        "sublevels": st0["sublevels"],
        "phases_ms": phases,
        "roofline": roofline,
        "whole_step": {"alg_bytes": mb, "frac": step_frac, "W_min": wmin,
                       "model": "build 32m + 8n; support 4(m + W+) + 36 B/triangle; scan 5 B/edge; "
                                "peel 4 W_min + 44 B per frontier edge"},
        "support_roofline": support_roofline,
        "cpu_baseline": None,
    }
    if not args.no_extras and args.workload == "rmat20":
        line["extras"] = extras(pkt, torch, gg, off, adj, g.m, ms, args.steps)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
