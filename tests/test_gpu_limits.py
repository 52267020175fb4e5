"""Size limits of the boundary on the GPU: the 29-bit support field.

A star whose centre has degree 2^28 + 2 has more than 2^28 - 1 edges, so the library
must check degrees, and the centre's degree is above 2^28: the call must fail with
TRUSS_E_RANGE before any support is counted (a support of that size would not fit the
word that also holds the edge state).  One degree lower the same star is accepted and
every edge gets trussness 2 (no triangles).  About 36 GB of device memory each."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def star(leaves):
    n = leaves + 1
    adj = np.empty(2 * leaves, np.int32)
    adj[:leaves] = np.arange(1, leaves + 1, dtype=np.int32)
    adj[leaves:] = 0
    off = np.empty(n + 1, np.int64)
    off[0] = 0
    off[1] = leaves
    off[2:] = leaves + np.arange(1, leaves + 1, dtype=np.int64)
    return off, adj


def run(leaves):
    import torch

    import paper_1707_02000_amd as pkt

    off, adj = star(leaves)
    print(f"star with {leaves} leaves", flush=True)
    off_t = torch.from_numpy(off).cuda()
    adj_t = torch.from_numpy(adj).cuda()
    del off, adj
    try:
        return pkt.truss_decompose(off_t, adj_t, validate=False)
    finally:
        del off_t, adj_t
        torch.cuda.empty_cache()


def test_degree_past_support_field_is_rejected():
    import torch

    import paper_1707_02000_amd as pkt

    with pytest.raises(pkt.TrussError) as ei:
        run((1 << 28) + 2)
    torch.cuda.empty_cache()
    assert ei.value.name == "TRUSS_E_RANGE"
    assert "degree" in str(ei.value)


def test_largest_degree_that_fits_is_accepted():
    import torch

    tau = run(1 << 28)  # degree 2^28: supports up to 2^28 - 1 fit
    t = tau.cpu().numpy()
    del tau
    torch.cuda.empty_cache()
    assert len(t) == 1 << 28
    assert int(t.min()) == 2 and int(t.max()) == 2
