"""truss_decompose32_static (no allocation: the library's static scratch as workspace)
against truss_decompose32 with a caller workspace, both called through the C ABI, bit
for bit: two calls in a row on one GPU, the second on a smaller graph (the scratch
keeps the first call's contents), and a graph too large for the scratch rejected."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _dev32(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else ctypes.c_void_p(0)


def _with_workspace(pkt, lib, torch, g):
    off, adj = _dev32(torch, g.offsets), _dev32(torch, g.adj)
    out = torch.full((max(g.m, 1),), -7, dtype=torch.int32, device="cuda")
    nb = ctypes.c_size_t(0)
    assert lib.truss_workspace_bytes(g.n, int(g.offsets[-1]), None, ctypes.byref(nb)) == 0
    need = nb.value + 8 * (g.n + 1) + 256
    _buf, wptr = pkt.alloc_workspace(need)
    code = lib.truss_decompose32(g.n, _p(off), _p(adj), _p(out), ctypes.c_void_p(wptr), need, None, None,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == 0, lib.truss_last_error()
    return out[:g.m].cpu().numpy()


def _static(lib, torch, g, out_fill=-7):
    off, adj = _dev32(torch, g.offsets), _dev32(torch, g.adj)
    out = torch.full((max(g.m, 1),), out_fill, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # inputs and output in place before the call
    code = lib.truss_decompose32_static(g.n, _p(off), _p(adj), _p(out), None, None,
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return code, out[:g.m].cpu().numpy()


def test_static_scratch_matches_caller_workspace(gpu_lib):
    import torch

    lib = gpu_lib.load()
    first = gg.rmat(15, 16, seed=21)          # larger first: the second call sees its leftovers
    second = gg.er(3000, mean_degree=20.0, seed=22)
    for g in (first, second):
        say("case static", g.name, "m", g.m)
        code, tau = _static(lib, torch, g)
        assert code == 0, lib.truss_last_error()
        ref = _with_workspace(gpu_lib, lib, torch, g)
        assert np.array_equal(tau, ref)
        assert np.array_equal(tau, oracle.truss(g))
    # an edgeless graph and a single triangle after them
    for g in (gg.from_edges(5, []), gg.from_edges(3, [(0, 1), (1, 2), (0, 2)])):
        code, tau = _static(lib, torch, g)
        assert code == 0 and np.array_equal(tau, oracle.truss(g))


def test_static_scratch_rejects_large_graph(gpu_lib):
    import torch

    lib = gpu_lib.load()
    g = gg.rmat(18, 16, seed=3)  # about 2 million edges: far beyond 64 MiB of workspace
    say("case static too large", g.name, "m", g.m)
    code, _ = _static(lib, torch, g)
    assert code == 5  # TRUSS_E_WORKSPACE
    assert b"static scratch" in lib.truss_last_error()
    # and the scratch still works afterwards
    small = gg.rmat(10, 16, seed=4)
    code, tau = _static(lib, torch, small)
    assert code == 0 and np.array_equal(tau, oracle.truss(small))


def test_static_binding_and_options(gpu_lib):
    import torch

    g = gg.rmat(12, 16, seed=6)
    want = oracle.truss(g)
    for loop in ("host", "device", "pipelined", "graph"):  # the last two run as device steps
        tau = gpu_lib.truss_decompose32_static(g.offsets.astype(np.int32), g.adj, device_loop=loop)
        assert np.array_equal(tau.cpu().numpy(), want), loop
    torch.cuda.synchronize()
