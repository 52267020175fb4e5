"""Python binding of libpkt, a gfx950 (MI355X) truss decomposition library.

Argument marshalling only: every step of the computation runs in the HIP kernels of
``libpkt.so`` (``csrc/``), reached through its C ABI (``include/pkt.h``).  PyTorch
provides device memory and the stream.  There is no CPU fallback: if the library
is missing or no GPU is visible, calls raise.

    import paper_1707_02000_amd as pkt
    tau = pkt.truss_decompose(offsets, adj)      # int32 trussness per edge, on the GPU

Edge order of every per-edge output: the pairs (u, v), u < v, in row-major order
of the input CSR.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpkt.so")

VARIANTS = {"auto": 0, "bsearch": 1, "merge": 2, "fixed": 3, "learned": 4}
CHOICES = ["fused", "fused_narrow", "wide", "wide_narrow", "wide_gallop", "wave", "hash"]
MODEL_CHOICES = 6  # the first six: the ones the cost model scores (TRUSS_MODEL_CHOICES)
LOOP_MODES = {"host": 0, "device": 1, "graph": 2, "pipelined": 3}  # truss_options.device_loop


def loop_mode(x) -> int:
    """truss_options.device_loop from a name, a bool (True = device-driven) or an int."""
    if isinstance(x, str):
        return LOOP_MODES[x]
    if isinstance(x, bool) or x is None:
        return 1 if x else 0
    return int(x)
NUM_FEATURES = 6

STATUS = {
    0: "TRUSS_OK", 1: "TRUSS_E_ARG", 2: "TRUSS_E_NOT_SIMPLE", 3: "TRUSS_E_NOT_SYMMETRIC",
    4: "TRUSS_E_RANGE", 5: "TRUSS_E_WORKSPACE", 6: "TRUSS_E_DEVICE", 7: "TRUSS_E_INTERNAL",
}


class TrussError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class Options(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("device_loop", ctypes.c_int32),
        ("validate", ctypes.c_int32),
        ("owner_rule", ctypes.c_int32),
        ("compact", ctypes.c_int32),
        ("steps_per_sync", ctypes.c_int32),
        ("mlp_weights", ctypes.c_void_p),
        ("trace", ctypes.c_void_p),
        ("profile", ctypes.c_int32),
        ("batch_mode", ctypes.c_int32),
        ("force_choice", ctypes.c_int32),
        ("single_round", ctypes.c_int32),
        ("peel_round", ctypes.c_void_p),
        ("multi_round", ctypes.c_int32),
        ("relabel", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 6),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("levels", ctypes.c_int64),
        ("sublevels", ctypes.c_int64),
        ("triangles", ctypes.c_int64),
        ("t_max", ctypes.c_int32),
        ("compactions", ctypes.c_int32),
        ("ms_validate", ctypes.c_float),
        ("ms_build", ctypes.c_float),
        ("ms_support", ctypes.c_float),
        ("ms_peel", ctypes.c_float),
        ("ms_total", ctypes.c_float),
        ("choice_count", ctypes.c_int64 * 8),
        ("wide_launches", ctypes.c_int64),
        ("wide_items", ctypes.c_int64),
        ("wide_frontier", ctypes.c_int64),
        ("wide_ms", ctypes.c_float),
        ("wide_timed", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("choice_count",)}
        d["choice_count"] = list(self.choice_count)[:len(CHOICES)]
        return d


class TraceRecord(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int32),
        ("kind", ctypes.c_int32),
        ("choice", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("frontier", ctypes.c_int64),
        ("items", ctypes.c_int64),
        ("ms", ctypes.c_float),
        ("features", ctypes.c_float * 8),
        ("round_index", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "features"}
        d["features"] = list(self.features)
        return d


class Trace(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("count", ctypes.c_int64),
                ("records", ctypes.POINTER(TraceRecord))]


_lib = None

# exported C functions and their signatures
_SIGS = {
    "truss_default_options": (None, [ctypes.c_void_p]),
    "truss_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "truss_decompose": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 4 + [ctypes.c_size_t]
                        + [ctypes.c_void_p] * 3),
    "truss_decompose32": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 4 + [ctypes.c_size_t]
                          + [ctypes.c_void_p] * 3),
    "truss_decompose32_static": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 6),
    "truss_support": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 4 + [ctypes.c_size_t]
                      + [ctypes.c_void_p] * 2),
    "truss_edge_list": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 5 + [ctypes.c_size_t]
                        + [ctypes.c_void_p]),
    "truss_ktruss_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p]),
    "truss_kcore_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p]),
    "truss_hindex_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p]),
    "truss_hindex": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 3 + [ctypes.c_int32]
                     + [ctypes.c_void_p] * 3 + [ctypes.c_size_t, ctypes.c_void_p]),
    "truss_kco_order_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p]),
    "truss_kco_order": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 4 + [ctypes.c_size_t, ctypes.c_void_p]),
    "truss_kco_relabel_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p]),
    "truss_kco_relabel": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 7
                          + [ctypes.c_size_t, ctypes.c_void_p]),
    "truss_kco_map_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p]),
    "truss_kco_map": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64] + [ctypes.c_void_p] * 8
                      + [ctypes.c_size_t, ctypes.c_void_p]),
    "truss_kcore": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 5 + [ctypes.c_size_t, ctypes.c_void_p]),
    "truss_ktruss": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64] + [ctypes.c_void_p] * 3 + [ctypes.c_int32]
                     + [ctypes.c_void_p] * 3 + [ctypes.c_size_t, ctypes.c_void_p]),
    "truss_batched_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                                     ctypes.c_void_p, ctypes.c_void_p]),
    "truss_decompose_batched": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 5
                                + [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t]
                                + [ctypes.c_void_p] * 3),
    "truss_mlp_num_params": (ctypes.c_int32, []),
    "truss_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "truss_mlp_init": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p,
                                                              ctypes.c_void_p]),
    "truss_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "truss_mlp_gradient": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32] + [ctypes.c_void_p] * 4
                           + [ctypes.c_size_t, ctypes.c_void_p]),
    "truss_mlp_train": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                                              ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                                              ctypes.c_size_t, ctypes.c_void_p]),
    "truss_mlp_choose": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 4),
    "truss_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "truss_last_error": (ctypes.c_char_p, []),
}


def load():
    """Load libpkt.so (built by ``paper_1707_02000_amd.build``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpkt.so not built at {LIB_PATH}; run __graft_entry__.build() "
                          "(python -m paper_1707_02000_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int):
    if code != 0:
        msg = load().truss_last_error().decode(errors="replace")
        raise TrussError(code, msg)


def default_options() -> Options:
    o = Options()
    load().truss_default_options(ctypes.byref(o))
    return o


def make_options(variant="auto", device_loop="pipelined", validate=True, owner_rule=0, compact=True,
                 steps_per_sync=0, mlp_weights=None, profile=False, force_choice=None,
                 single_round=False, multi_round=False, relabel="auto") -> Options:
    o = default_options()
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.device_loop = loop_mode(device_loop)
    o.validate = int(bool(validate))
    o.owner_rule = int(owner_rule)
    o.compact = int(bool(compact))
    o.steps_per_sync = int(steps_per_sync)
    o.mlp_weights = None if mlp_weights is None else ctypes.c_void_p(mlp_weights.data_ptr())
    o.profile = int(bool(profile))
    if force_choice is not None:
        o.variant = VARIANTS["fixed"]
        o.force_choice = CHOICES.index(force_choice) if isinstance(force_choice, str) else int(force_choice)
    o.single_round = int(bool(single_round))
    o.multi_round = int(bool(multi_round))
    o.relabel = relabel_mode(relabel)
    return o


RELABEL = {"off": 0, "auto": 1, "always": 2}


def relabel_mode(x) -> int:
    """truss_options.relabel from "off" / "auto" / "always", False (off) or True (always)."""
    if isinstance(x, str):
        return RELABEL[x]
    if isinstance(x, bool):
        return 2 if x else 0
    return int(x)


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: libpkt runs only on the GPU")
    return torch


def _dev(x, dtype, torch):
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    x = x.to(device="cuda", dtype=dtype)
    return x.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def alloc_workspace(nbytes: int):
    """Device workspace of nbytes, 256-byte aligned (over-allocates and offsets if needed)."""
    torch = _torch()
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
    shift = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + shift


def workspace_bytes(n: int, two_m: int, options: Options | None = None) -> int:
    nb = ctypes.c_size_t(0)
    _check(load().truss_workspace_bytes(int(n), int(two_m), ctypes.byref(options) if options else None,
                                        ctypes.byref(nb)))
    return nb.value


@dataclass
class Workspace:
    """A reusable device workspace for graphs up to (n, two_m)."""

    n: int
    two_m: int
    buf: object
    ptr: int
    nbytes: int

    @classmethod
    def for_graph(cls, n: int, two_m: int, batched: bool = False, num_graphs: int = 0):
        lib = load()
        nb = ctypes.c_size_t(0)
        if batched:
            _check(lib.truss_batched_workspace_bytes(int(num_graphs), int(n), int(two_m), None, ctypes.byref(nb)))
        else:
            _check(lib.truss_workspace_bytes(int(n), int(two_m), None, ctypes.byref(nb)))
        buf, ptr = alloc_workspace(nb.value)
        return cls(n, two_m, buf, ptr, nb.value)


def truss_decompose(offsets, adj, *, variant="auto", device_loop="pipelined", validate=True, owner_rule=0,
                    compact=True, steps_per_sync=0, mlp_weights=None, stream=None, workspace=None,
                    out=None, return_stats=False, trace_capacity=0, profile=False, force_choice=None,
                    single_round=False, return_rounds=False, multi_round=False, relabel="auto"):
    """Trussness (int32, >= 2) of every edge of a simple undirected CSR graph, on the GPU.

    offsets: int64 (or int32) [n+1]; adj: int32 [2m]; numpy arrays (copied to the GPU) or
    CUDA tensors.  Returns a CUDA int32 tensor [m] (and a stats dict if return_stats; with
    trace_capacity > 0 the stats dict also holds the per-sequence trace of the peeling loop).
    With return_rounds, also the frontier round that processed every edge (int32 [m], a
    peeling order), right after the trussness.  relabel: "auto" (default) decomposes large
    graphs with skewed degrees relabelled by increasing degree and maps the result back (same
    output, faster there); True / "always" does so for every graph, False / "off" never.
    """
    torch = _torch()
    lib = load()
    off32 = (isinstance(offsets, np.ndarray) and offsets.dtype == np.int32) or \
            (hasattr(offsets, "dtype") and str(offsets.dtype) == "torch.int32")
    off_t = _dev(offsets, torch.int32 if off32 else torch.int64, torch)
    adj_t = _dev(adj, torch.int32, torch)
    n = off_t.numel() - 1
    two_m = adj_t.numel()
    m = two_m // 2
    opt = make_options(variant, device_loop, validate, owner_rule, compact, steps_per_sync, mlp_weights, profile,
                       force_choice, single_round, multi_round, relabel)
    if workspace is None:
        nb = workspace_bytes(n, two_m, opt) + (8 * (n + 1) + 256 if off32 else 0)
        _buf, wptr = alloc_workspace(nb)
    else:
        _buf, wptr, nb = workspace.buf, workspace.ptr, workspace.nbytes
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    rounds = None
    if return_rounds:
        rounds = torch.full((max(m, 1),), -1, dtype=torch.int32, device="cuda")
        opt.peel_round = ctypes.c_void_p(rounds.data_ptr())
    st = Stats()
    trace = None
    if trace_capacity > 0:
        recs = (TraceRecord * int(trace_capacity))()
        trace = Trace(int(trace_capacity), 0, ctypes.cast(recs, ctypes.POINTER(TraceRecord)))
        opt.trace = ctypes.cast(ctypes.pointer(trace), ctypes.c_void_p)
    fn = lib.truss_decompose32 if off32 else lib.truss_decompose
    code = fn(n, _ptr(off_t), _ptr(adj_t), _ptr(out), ctypes.c_void_p(wptr), nb, ctypes.byref(opt),
              ctypes.byref(st), _stream(torch, stream))
    _check(code)
    res = out[:m]
    sd = st.as_dict()
    if trace is not None:
        sd["trace"] = [recs[i].as_dict() for i in range(trace.count)]
    ret = (res,) + ((rounds[:m],) if return_rounds else ()) + ((sd,) if return_stats else ())
    return ret if len(ret) > 1 else res


def truss_support(offsets, adj, *, stream=None):
    """Initial support (triangles per edge), int32 [m] CUDA tensor, computed on the GPU."""
    torch = _torch()
    lib = load()
    off_t = _dev(offsets, torch.int64, torch)
    adj_t = _dev(adj, torch.int32, torch)
    n, two_m = off_t.numel() - 1, adj_t.numel()
    nb = workspace_bytes(n, two_m)
    _buf, wptr = alloc_workspace(nb)
    out = torch.empty(max(two_m // 2, 1), dtype=torch.int32, device="cuda")
    _check(lib.truss_support(n, _ptr(off_t), _ptr(adj_t), _ptr(out), ctypes.c_void_p(wptr), nb, None,
                             _stream(torch, stream)))
    return out[: two_m // 2]


def edge_list(offsets, adj, *, stream=None):
    """Endpoints of every edge in output order, (m, 2) int32 CUDA tensor (u < v)."""
    torch = _torch()
    lib = load()
    off_t = _dev(offsets, torch.int64, torch)
    adj_t = _dev(adj, torch.int32, torch)
    n, two_m = off_t.numel() - 1, adj_t.numel()
    m = two_m // 2
    nb = workspace_bytes(n, two_m)
    _buf, wptr = alloc_workspace(nb)
    eu = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    ev = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    _check(lib.truss_edge_list(n, _ptr(off_t), _ptr(adj_t), _ptr(eu), _ptr(ev), ctypes.c_void_p(wptr), nb,
                               _stream(torch, stream)))
    return torch.stack([eu[:m], ev[:m]], dim=1)


def ktruss(n, edges, trussness, k, *, stream=None, out=None):
    """The maximal k-trusses: per edge the smallest edge id of its k-truss (-1 below k).

    edges: (m, 2) int32 endpoints (as from edge_list) or a pair of int32 [m] arrays;
    trussness: int32 [m].  Returns (labels int32 [m] CUDA tensor, number of k-trusses).
    """
    torch = _torch()
    lib = load()
    if isinstance(edges, (tuple, list)):
        eu, ev = (_dev(x, torch.int32, torch).contiguous() for x in edges)
    else:
        e = _dev(edges, torch.int32, torch).reshape(-1, 2)
        eu, ev = e[:, 0].contiguous(), e[:, 1].contiguous()
    tau = _dev(trussness, torch.int32, torch).contiguous()
    m = tau.numel()
    nb = ctypes.c_size_t(0)
    _check(lib.truss_ktruss_workspace_bytes(int(n), ctypes.byref(nb)))
    _buf, wptr = alloc_workspace(nb.value)
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    count = ctypes.c_int32(0)
    _check(lib.truss_ktruss(int(n), m, _ptr(eu), _ptr(ev), _ptr(tau), int(k), _ptr(out), ctypes.byref(count),
                            ctypes.c_void_p(wptr), nb.value, _stream(torch, stream)))
    return out[:m], int(count.value)


def kcore(offsets, adj, *, stream=None):
    """Core numbers of every vertex (int32 [n] CUDA tensor) and the largest one."""
    torch = _torch()
    lib = load()
    off_t = _dev(offsets, torch.int64, torch)
    adj_t = _dev(adj, torch.int32, torch)
    n = off_t.numel() - 1
    nb = ctypes.c_size_t(0)
    _check(lib.truss_kcore_workspace_bytes(int(n), ctypes.byref(nb)))
    _buf, wptr = alloc_workspace(nb.value)
    out = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    cmax = ctypes.c_int32(0)
    _check(lib.truss_kcore(int(n), _ptr(off_t), _ptr(adj_t), _ptr(out), ctypes.byref(cmax), ctypes.c_void_p(wptr),
                           nb.value, _stream(torch, stream)))
    return out[:n], int(cmax.value)


def hindex(offsets, adj, *, max_sweeps=-1, stream=None):
    """Trussness by the local h-index iteration: (int32 [m] CUDA tensor, sweeps that changed
    an estimate, converged).  With max_sweeps >= 0 the estimates + 2 after that many sweeps."""
    torch = _torch()
    lib = load()
    off_t = _dev(offsets, torch.int64, torch)
    adj_t = _dev(adj, torch.int32, torch)
    n = off_t.numel() - 1
    two_m = adj_t.numel()
    nb = ctypes.c_size_t(0)
    _check(lib.truss_hindex_workspace_bytes(int(n), int(two_m), ctypes.byref(nb)))
    _buf, wptr = alloc_workspace(nb.value)
    out = torch.empty(max(two_m // 2, 1), dtype=torch.int32, device="cuda")
    sw = ctypes.c_int32(0)
    conv = ctypes.c_int32(0)
    _check(lib.truss_hindex(int(n), _ptr(off_t), _ptr(adj_t), _ptr(out), int(max_sweeps), ctypes.byref(sw),
                            ctypes.byref(conv), ctypes.c_void_p(wptr), nb.value, _stream(torch, stream)))
    return out[:two_m // 2], int(sw.value), bool(conv.value)


def kco_order(core, *, stream=None):
    """KCO order: (new_id, order) int32 [n] CUDA tensors, vertices sorted by (core number, id)."""
    torch = _torch()
    lib = load()
    c = _dev(core, torch.int32, torch)
    n = c.numel()
    nb = ctypes.c_size_t(0)
    _check(lib.truss_kco_order_workspace_bytes(int(n), ctypes.byref(nb)))
    _buf, wptr = alloc_workspace(nb.value)
    new_id = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    order = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    _check(lib.truss_kco_order(int(n), _ptr(c), _ptr(new_id), _ptr(order), ctypes.c_void_p(wptr), nb.value,
                               _stream(torch, stream)))
    return new_id[:n], order[:n]


def kco_relabel(offsets, adj, new_id, order, *, stream=None):
    """The relabelled CSR (offsets2 int64 [n+1], adj2 int32 [2m] CUDA tensors), rows sorted."""
    torch = _torch()
    lib = load()
    off_t = _dev(offsets, torch.int64, torch)
    adj_t = _dev(adj, torch.int32, torch)
    nid = _dev(new_id, torch.int32, torch)
    ordr = _dev(order, torch.int32, torch)
    n = off_t.numel() - 1
    two_m = adj_t.numel()
    nb = ctypes.c_size_t(0)
    _check(lib.truss_kco_relabel_workspace_bytes(int(n), int(two_m), ctypes.byref(nb)))
    _buf, wptr = alloc_workspace(nb.value)
    off2 = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    adj2 = torch.empty(max(two_m, 1), dtype=torch.int32, device="cuda")
    _check(lib.truss_kco_relabel(int(n), _ptr(off_t), _ptr(adj_t), _ptr(nid), _ptr(ordr), _ptr(off2),
                                 _ptr(adj2) if two_m else ctypes.c_void_p(0), ctypes.c_void_p(wptr), nb.value,
                                 _stream(torch, stream)))
    return off2, adj2[:two_m]


def kco_map(n, edges, new_id, offsets2, adj2, trussness2, *, stream=None):
    """Trussness per input edge (int32 [m] CUDA tensor) from that of the relabelled graph.

    edges: (m, 2) int32 endpoints of the input (as from edge_list) or a pair of int32 [m] arrays.
    """
    torch = _torch()
    lib = load()
    if isinstance(edges, (tuple, list)):
        eu, ev = (_dev(x, torch.int32, torch).contiguous() for x in edges)
    else:
        e = _dev(edges, torch.int32, torch).reshape(-1, 2)
        eu, ev = e[:, 0].contiguous(), e[:, 1].contiguous()
    nid = _dev(new_id, torch.int32, torch)
    off2 = _dev(offsets2, torch.int64, torch)
    adj2 = _dev(adj2, torch.int32, torch)
    tau2 = _dev(trussness2, torch.int32, torch)
    m = eu.numel()
    nb = ctypes.c_size_t(0)
    _check(lib.truss_kco_map_workspace_bytes(int(n), ctypes.byref(nb)))
    _buf, wptr = alloc_workspace(nb.value)
    out = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    _check(lib.truss_kco_map(int(n), int(m), _ptr(eu), _ptr(ev), _ptr(nid), _ptr(off2), _ptr(adj2), _ptr(tau2),
                             _ptr(out), ctypes.c_void_p(wptr), nb.value, _stream(torch, stream)))
    return out[:m]


def truss_decompose32_static(offsets, adj, *, validate=True, device_loop="device", stream=None, out=None,
                             return_stats=False):
    """truss_decompose32_static: int32 offsets, the library's static scratch as workspace
    (no allocation inside the library); int32 [m] CUDA tensor.  ``out`` may be given
    so that the call allocates nothing on the Python side either."""
    torch = _torch()
    lib = load()
    off_t = _dev(offsets, torch.int32, torch)
    adj_t = _dev(adj, torch.int32, torch)
    n = off_t.numel() - 1
    m = adj_t.numel() // 2
    opt = make_options("auto", device_loop, validate)
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    st = Stats()
    _check(lib.truss_decompose32_static(int(n), _ptr(off_t), _ptr(adj_t), _ptr(out), ctypes.byref(opt),
                                        ctypes.byref(st), _stream(torch, stream)))
    res = out[:m]
    return (res, st.as_dict()) if return_stats else res


BATCH_MODES = {"union": 0, "sequential": 1, "persistent": 2}  # truss_options.batch_mode


def truss_decompose_batched(vtx_off, adj_off, offsets_packed, adj_packed, *, variant="auto", validate=True,
                            mode="union", sequential=False, stream=None, workspace=None, out=None,
                            return_stats=False, device_loop="pipelined", mlp_weights=None, force_choice=None):
    """Trussness of many packed graphs (layout of include/pkt.h); int32 [sum m_g] CUDA tensor.

    mode: "union" (one level loop over the disjoint union, the default), "persistent" (one
    launch, a workgroup per graph) or "sequential" (one graph after another);
    sequential=True is the same as mode="sequential"."""
    torch = _torch()
    lib = load()
    vo = _dev(vtx_off, torch.int64, torch)
    ao = _dev(adj_off, torch.int64, torch)
    op = _dev(offsets_packed, torch.int32, torch)
    ap = _dev(adj_packed, torch.int32, torch)
    G = vo.numel() - 1
    total_vtx, total_adj = int(op.numel()), int(ap.numel())
    opt = make_options(variant, device_loop, validate, mlp_weights=mlp_weights, force_choice=force_choice)
    opt.batch_mode = BATCH_MODES["sequential" if sequential else mode]
    if workspace is None:
        nb = ctypes.c_size_t(0)
        _check(lib.truss_batched_workspace_bytes(G, total_vtx, total_adj, ctypes.byref(opt), ctypes.byref(nb)))
        nb = nb.value
        _buf, wptr = alloc_workspace(nb)
    else:
        _buf, wptr, nb = workspace.buf, workspace.ptr, workspace.nbytes
    if out is None:
        out = torch.empty(max(total_adj // 2, 1), dtype=torch.int32, device="cuda")
    st = Stats()
    _check(lib.truss_decompose_batched(G, _ptr(vo), _ptr(ao), _ptr(op), _ptr(ap), _ptr(out), total_vtx, total_adj,
                                       ctypes.c_void_p(wptr), nb, ctypes.byref(opt), ctypes.byref(st),
                                       _stream(torch, stream)))
    res = out[: total_adj // 2]
    return (res, st.as_dict()) if return_stats else res


def wedges(degrees: np.ndarray) -> int:
    """Wedge count (sum of d(d-1)/2), the paper's work measure for its GWeps rate."""
    d = np.asarray(degrees, dtype=np.int64)
    return int((d * (d - 1) // 2).sum())
