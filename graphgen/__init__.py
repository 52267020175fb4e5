"""Seeded synthetic graph inputs (ER, R-MAT, Chung-Lu + planted cliques, 2-D RGG, packed batches).

Inputs only: this module holds none of the truss-decomposition arithmetic.  The
tests, the benchmark and the smoke check use it to make one CSR that is fed both to
the GPU library and to the CPU oracle.

Every graph is simple and undirected, returned as a symmetric CSR with strictly
ascending rows: ``offsets`` (int64, n+1) and ``adj`` (int32, 2m).  The sampling runs
in C (``graphgen.c``) with a counter-based generator, so a (recipe, seed) pair names
one graph regardless of the thread count.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "_graphgen.so")
_lib = None


def build() -> str:
    """Compile the generator library in-tree (host code, gcc + OpenMP)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("PKT_GRAPHGEN_LIB")  # another build of the same source (the sanitizer test's)
    if not path:
        path = _LIB
        if not os.path.exists(_LIB):
            build()
    lib = ctypes.CDLL(path)
    P64 = ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))
    P32 = ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.gg_er.argtypes = [i32, dbl, u64, P64, P32]
    lib.gg_rmat.argtypes = [i32, i32, i64, dbl, dbl, dbl, i32, u64, P64, P32]
    lib.gg_chunglu.argtypes = [i32, dbl, dbl, i64, i32, i32, i32, i32, u64, P64, P32]
    lib.gg_rgg.argtypes = [i32, dbl, u64, P64, P32]
    lib.gg_batch.argtypes = [i32, i32, i32, dbl, dbl, i32, i32, u64, P64, P64, P32, P32, P32]
    for f in (lib.gg_er, lib.gg_rmat, lib.gg_chunglu, lib.gg_rgg, lib.gg_batch):
        f.restype = ctypes.c_int
    lib.gg_free.argtypes = [ctypes.c_void_p]
    lib.gg_free.restype = None
    _lib = lib
    return lib


@dataclass
class Graph:
    """A simple undirected graph as symmetric CSR (rows strictly ascending)."""

    n: int
    offsets: np.ndarray  # int64 [n+1]
    adj: np.ndarray  # int32 [2m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.offsets[-1]) // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.offsets, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.adj, dtype=np.int32).tobytes())
        return h.hexdigest()


@dataclass
class Batch:
    """Packed independent graphs: local int32 CSRs back to back."""

    vtx_off: np.ndarray  # int64 [G+1]; offsets of graph g start here, n_g+1 entries
    adj_off: np.ndarray  # int64 [G+1]; adjacency of graph g starts here, 2 m_g entries
    offsets: np.ndarray  # int32 packed local offsets
    adj: np.ndarray  # int32 packed local ids
    family: np.ndarray  # int32 [G]: 0 ER, 1 R-MAT, 2 RGG

    @property
    def num_graphs(self) -> int:
        return len(self.vtx_off) - 1

    @property
    def total_m(self) -> int:
        return int(self.adj_off[-1]) // 2

    def union(self) -> Graph:
        """The disjoint union as one graph (vertex ids shifted by each graph's vertex base)."""
        G = self.num_graphs
        n_g = np.diff(self.vtx_off) - 1
        vbase = np.concatenate([[0], np.cumsum(n_g)]).astype(np.int64)
        off = np.empty(int(vbase[-1]) + 1, np.int64)
        for g in range(G):
            a = int(self.vtx_off[g])
            off[vbase[g]:vbase[g + 1]] = self.offsets[a:a + n_g[g]].astype(np.int64) + self.adj_off[g]
        off[-1] = self.adj_off[-1]
        shift = np.repeat(vbase[:-1], np.diff(self.adj_off))
        return Graph(int(vbase[-1]), off, (self.adj.astype(np.int64) + shift).astype(np.int32), name="batch-union")

    def graph(self, g: int) -> Graph:
        a, b = int(self.vtx_off[g]), int(self.vtx_off[g + 1])
        s, t = int(self.adj_off[g]), int(self.adj_off[g + 1])
        off = self.offsets[a:b].astype(np.int64)
        return Graph(b - a - 1, off, self.adj[s:t].copy(), name=f"batch[{g}]")


def _take(lib, p, count, dtype):
    if count == 0:
        lib.gg_free(p)
        return np.zeros(0, dtype=dtype)
    arr = np.ctypeslib.as_array(p, shape=(count,)).copy().astype(dtype, copy=False)
    lib.gg_free(p)
    return arr


def _finish(lib, rc, n, po, pa, name):
    if rc != 0:
        raise RuntimeError(f"graph generator failed with code {rc} ({name})")
    off = _take(lib, po, n + 1, np.int64)
    adj = _take(lib, pa, int(off[-1]), np.int32)
    return Graph(n, off, adj, name=name)


def er(n: int, mean_degree: float | None = None, p: float | None = None, seed: int = 1) -> Graph:
    """Erdos-Renyi G(n, p); give p directly or a mean degree k (p = k/(n-1))."""
    lib = _load()
    if p is None:
        p = 0.0 if n <= 1 else min(1.0, float(mean_degree) / (n - 1))
    po, pa = ctypes.POINTER(ctypes.c_int64)(), ctypes.POINTER(ctypes.c_int32)()
    rc = lib.gg_er(n, float(p), seed, ctypes.byref(po), ctypes.byref(pa))
    return _finish(lib, rc, n, po, pa, f"er(n={n},p={p:.6g},seed={seed})")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         n: int | None = None, permute: bool = True, seed: int = 1) -> Graph:
    """R-MAT with edge_factor * n generated pairs, symmetrized, deduplicated, ids permuted."""
    lib = _load()
    if n is None:
        n = 1 << scale
    po, pa = ctypes.POINTER(ctypes.c_int64)(), ctypes.POINTER(ctypes.c_int32)()
    rc = lib.gg_rmat(scale, n, int(edge_factor) * n, a, b, c, int(permute), seed,
                     ctypes.byref(po), ctypes.byref(pa))
    return _finish(lib, rc, n, po, pa, f"rmat(s={scale},ef={edge_factor},seed={seed})")


def chunglu(n: int, beta: float = 2.1, target_m: float = 1.0e8, draws: int | None = None,
            ncliques: int = 200, cmin: int = 50, cmax: int = 500, permute: bool = True,
            seed: int = 1) -> Graph:
    """Chung-Lu power-law graph (exponent beta) plus planted cliques, ids permuted."""
    lib = _load()
    if draws is None:
        draws = int(target_m)
    po, pa = ctypes.POINTER(ctypes.c_int64)(), ctypes.POINTER(ctypes.c_int32)()
    rc = lib.gg_chunglu(n, beta, float(target_m), int(draws), ncliques, cmin, cmax, int(permute),
                        seed, ctypes.byref(po), ctypes.byref(pa))
    return _finish(lib, rc, n, po, pa,
                   f"chunglu(n={n},beta={beta},draws={draws},cliques={ncliques}x[{cmin},{cmax}],seed={seed})")


def rgg(n: int, mean_degree: float, seed: int = 1) -> Graph:
    """2-D random geometric graph, radius sqrt(k / (pi (n-1)))."""
    lib = _load()
    po, pa = ctypes.POINTER(ctypes.c_int64)(), ctypes.POINTER(ctypes.c_int32)()
    rc = lib.gg_rgg(n, float(mean_degree), seed, ctypes.byref(po), ctypes.byref(pa))
    return _finish(lib, rc, n, po, pa, f"rgg(n={n},k={mean_degree},seed={seed})")


def batch(num_graphs: int = 4096, nmin: int = 64, nmax: int = 16384, kmin: float = 8.0,
          kmax: float = 64.0, efmin: int = 8, efmax: int = 32, seed: int = 1) -> Batch:
    """Packed batch of mixed ER / R-MAT / RGG graphs with n uniform in [nmin, nmax]."""
    lib = _load()
    pv, pe = ctypes.POINTER(ctypes.c_int64)(), ctypes.POINTER(ctypes.c_int64)()
    po, pa, pf = (ctypes.POINTER(ctypes.c_int32)(), ctypes.POINTER(ctypes.c_int32)(),
                  ctypes.POINTER(ctypes.c_int32)())
    rc = lib.gg_batch(num_graphs, nmin, nmax, kmin, kmax, efmin, efmax, seed, ctypes.byref(pv),
                      ctypes.byref(pe), ctypes.byref(po), ctypes.byref(pa), ctypes.byref(pf))
    if rc != 0:
        raise RuntimeError(f"batch generator failed with code {rc}")
    vtx_off = _take(lib, pv, num_graphs + 1, np.int64)
    adj_off = _take(lib, pe, num_graphs + 1, np.int64)
    offsets = _take(lib, po, int(vtx_off[-1]), np.int32)
    adj = _take(lib, pa, int(adj_off[-1]), np.int32)
    fam = _take(lib, pf, num_graphs, np.int32)
    return Batch(vtx_off, adj_off, offsets, adj, fam)


def from_edges(n: int, edges) -> Graph:
    """Simple symmetric CSR from an iterable of (u, v) pairs (self-loops dropped, deduplicated)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if len(e):
        e = e[e[:, 0] != e[:, 1]]
    both = np.concatenate([e, e[:, ::-1]]) if len(e) else np.zeros((0, 2), np.int64)
    if len(both):
        key = np.unique(both[:, 0] * max(n, 1) + both[:, 1])
        rows, cols = key // max(n, 1), key % max(n, 1)
    else:
        rows = cols = np.zeros(0, np.int64)
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, rows + 1, 1)
    off = np.cumsum(off)
    return Graph(n, off, cols.astype(np.int32), name=f"edges(n={n},m={len(cols)//2})")


def pack(graphs) -> Batch:
    """Pack a list of Graph objects into one Batch (int32 local CSRs)."""
    vtx = [0]
    adj_off = [0]
    offs, adjs = [], []
    for g in graphs:
        offs.append(g.offsets.astype(np.int32))
        adjs.append(g.adj.astype(np.int32))
        vtx.append(vtx[-1] + g.n + 1)
        adj_off.append(adj_off[-1] + len(g.adj))
    return Batch(np.array(vtx, np.int64), np.array(adj_off, np.int64),
                 np.concatenate(offs) if offs else np.zeros(0, np.int32),
                 np.concatenate(adjs) if adjs else np.zeros(0, np.int32),
                 np.full(len(vtx) - 1, -1, np.int32))


# ---------------------------------------------------------------- named workloads

def workload(name: str, seed: int = 1):
    """The named synthetic workloads the benchmark and parity tests use.

    er4096        Erdos-Renyi, n = 4096, mean degree 16.
    rmat20        R-MAT scale 20, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), permuted.
    chunglu23     Chung-Lu, n = 2^23, exponent 2.1, about 1e8 edges, 200 cliques of 50..500.
    batch4096     4096 graphs, n in [64, 16384], ER / R-MAT / RGG mix.
    rmat24        R-MAT scale 24, same parameters as rmat20.
    Smaller variants (rmat16, rmat18, chunglu18, batch64) keep the same recipes at a
    size the CPU oracle finishes in seconds.
    """
    if name == "er4096":
        return er(4096, mean_degree=16.0, seed=seed)
    if name.startswith("rmat"):
        return rmat(int(name[4:]), 16, seed=seed)
    if name == "chunglu23":
        return chunglu(1 << 23, 2.1, 1.0e8, draws=92_000_000, seed=seed)
    if name.startswith("chunglu"):
        s = int(name[7:])
        scale = (1 << s) / float(1 << 23)
        tm = 1.0e8 * scale
        return chunglu(1 << s, 2.1, tm, draws=int(0.92 * tm), ncliques=max(1, int(200 * scale)),
                       cmin=50, cmax=min(500, max(60, int(500 * math.sqrt(scale)))), seed=seed)
    if name.startswith("batch"):
        g = int(name[5:])
        nmax = 16384 if g >= 1024 else 2048
        return batch(g, 64, nmax, seed=seed)
    raise KeyError(name)
