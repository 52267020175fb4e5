"""CPU ORACLE -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg
may import this package.  It shares no code with the GPU library
(``paper_1707_02000_amd``) and the GPU library never imports it.

Contents
  * ``truss`` / ``support`` / ``edge_list`` -- the serial Wang-Cheng style bucket peel
    (Background section, Algorithm 1) and the support definition, in plain C
    (``wc_truss.c``), called through ctypes.
  * ``definition`` -- the k-truss definition written out in pure Python for tiny
    graphs (repeated deletion of edges in fewer than k-2 triangles), support by set
    intersection, k-core numbers, and the local h-index iteration.
  * ``certificate`` -- checks of a trussness array against the definition that hold at
    any size, given a peeling order: every edge of trussness k lies in >= k-2
    triangles of the edges of trussness >= k, and no edge had more than k-2 triangles
    left when the order removed it; run on sampled edges at full scale.
  * ``kcore`` -- core numbers of the vertices (Batagelj-Zaversnik bucket order, in C),
    pinned against the k-core definition in ``definition``.
  * ``ktruss`` -- the maximal k-trusses given the trussness (Background section): the
    connected components of the edges of trussness >= k, each named by its smallest
    edge id.
  * ``kco`` -- vertex reordering by increasing core number before support (Table 2's
    KCO), the relabelled CSR, the trussness mapped back, and the work estimate
    sum_v d+(v)^2.
  * ``psl_model`` -- a step-by-step model of the level-synchronous peeling
    (Algorithms 4 and 5 of the PKT section) whose threads interleave at random, to
    check the concurrency rules (lower-edge-id ownership, clamp and restore).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wc_truss.c")
_LIB = os.path.join(_HERE, "_wc_truss.so")
_lib = None


class OracleInputError(ValueError):
    pass


def build() -> str:
    """Compile the C oracle in-tree (serial, -O2)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("PKT_ORACLE_LIB")  # another build of the same source (the sanitizer test's)
    if not path:
        path = _LIB
        if not os.path.exists(_LIB):
            build()
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    lib.oracle_check_csr.argtypes = [ctypes.c_int32, vp, vp]
    lib.oracle_check_csr.restype = ctypes.c_int
    lib.oracle_edge_ids.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
    lib.oracle_edge_ids.restype = ctypes.c_int64
    lib.oracle_support.argtypes = [ctypes.c_int32, vp, vp, vp]
    lib.oracle_support.restype = ctypes.c_int64
    lib.oracle_truss.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
    lib.oracle_truss.restype = ctypes.c_int64
    lib.oracle_kcore.argtypes = [ctypes.c_int32, vp, vp, vp]
    lib.oracle_kcore.restype = ctypes.c_int64
    _lib = lib
    return lib


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    adj = np.ascontiguousarray(g.adj, dtype=np.int32)
    if len(adj) == 0:
        adj = np.zeros(1, np.int32)  # a valid pointer for an empty graph
    return g.n, off, adj


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def check_csr(g) -> bool:
    n, off, adj = _csr(g)
    return _load().oracle_check_csr(n, _ptr(off), _ptr(adj)) == 0


def edge_list(g) -> np.ndarray:
    """(m, 2) int32 endpoints (u < v) in canonical order: row-major upper triangle."""
    n, off, adj = _csr(g)
    m = int(off[-1]) // 2
    eu = np.zeros(max(m, 1), np.int32)
    ev = np.zeros(max(m, 1), np.int32)
    eid = np.zeros(max(int(off[-1]), 1), np.int32)
    r = _load().oracle_edge_ids(n, _ptr(off), _ptr(adj), _ptr(eu), _ptr(ev), _ptr(eid))
    if r < 0:
        raise OracleInputError(f"oracle_edge_ids failed ({r})")
    return np.stack([eu[:m], ev[:m]], axis=1)


def support(g) -> np.ndarray:
    """Support |N(u) ∩ N(v)| of every edge, canonical order (int32)."""
    n, off, adj = _csr(g)
    m = int(off[-1]) // 2
    S = np.zeros(max(m, 1), np.int32)
    r = _load().oracle_support(n, _ptr(off), _ptr(adj), _ptr(S))
    if r < 0:
        raise OracleInputError(f"oracle_support failed ({r})")
    return S[:m]


def truss(g, with_support: bool = False, with_rank: bool = False):
    """Trussness of every edge, canonical order (int32, >= 2).

    with_support adds the initial support; with_rank adds the removal step of every
    edge in the bucket peel (int64, a peeling order for ``certificate``).
    """
    n, off, adj = _csr(g)
    m = int(off[-1]) // 2
    tau = np.zeros(max(m, 1), np.int32)
    S0 = np.zeros(max(m, 1), np.int32)
    rank = np.zeros(max(m, 1), np.int64) if with_rank else None
    r = _load().oracle_truss(n, _ptr(off), _ptr(adj), _ptr(tau), _ptr(S0), _ptr(rank) if with_rank else None)
    if r < 0:
        raise OracleInputError(f"oracle_truss failed ({r})")
    out = (tau[:m],)
    if with_support:
        out += (S0[:m],)
    if with_rank:
        out += (rank[:m],)
    return out if len(out) > 1 else out[0]


def edge_ids(g):
    """(endpoints (m, 2) int32, edge id of every adjacency slot int32[2m]) in canonical order."""
    n, off, adj = _csr(g)
    two_m = int(off[-1])
    m = two_m // 2
    eu = np.zeros(max(m, 1), np.int32)
    ev = np.zeros(max(m, 1), np.int32)
    eid = np.zeros(max(two_m, 1), np.int32)
    r = _load().oracle_edge_ids(n, _ptr(off), _ptr(adj), _ptr(eu), _ptr(ev), _ptr(eid))
    if r < 0:
        raise OracleInputError(f"oracle_edge_ids failed ({r})")
    return np.stack([eu[:m], ev[:m]], axis=1), eid[:two_m]


def kcore(g) -> np.ndarray:
    """Core number of every vertex (int32), by the bucket order in C."""
    n, off, adj = _csr(g)
    core = np.zeros(max(n, 1), np.int32)
    r = _load().oracle_kcore(n, _ptr(off), _ptr(adj), _ptr(core))
    if r < 0:
        raise OracleInputError(f"oracle_kcore failed ({r})")
    return core[:n]

