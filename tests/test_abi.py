"""The C ABI without a GPU: the library loads, exports every declared symbol,
host-only entry points behave, and the Python layer refuses to run without it."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pkt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(truss_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1707_02000_amd as pkt

    if not os.path.exists(pkt.LIB_PATH):
        pytest.fail("libpkt.so is not built (run __graft_entry__.build())")
    return pkt.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    import paper_1707_02000_amd as pkt

    out = subprocess.check_output(["nm", "-D", "--defined-only", pkt.LIB_PATH]).decode()
    exported = set(re.findall(r"\bT (truss_\w+)", out))
    assert set(names) == exported


def declared_param_counts():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(truss_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", text):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_signatures_match_header(lib):
    import paper_1707_02000_amd as pkt

    counts = declared_param_counts()
    assert set(counts) == set(pkt._SIGS)
    for name, (_, args) in pkt._SIGS.items():
        assert len(args) == counts[name], name


def test_default_options_and_struct_sizes(lib):
    import paper_1707_02000_amd as pkt

    o = pkt.default_options()
    assert (o.variant, o.device_loop, o.validate, o.owner_rule, o.compact) == (0, 3, 1, 0, 1)
    assert o.batch_mode == 0 and o.multi_round == 0 and o.relabel == 1 and list(o.reserved) == [0] * 6
    assert ctypes.sizeof(pkt.Options) == 96
    assert ctypes.sizeof(pkt.Stats) == 160
    assert ctypes.sizeof(pkt.TraceRecord) == 72


def test_workspace_bytes_host_only(lib):
    import paper_1707_02000_amd as pkt

    a = pkt.workspace_bytes(1000, 20000)
    b = pkt.workspace_bytes(1000, 40000)
    assert 0 < a < b
    assert a % 256 == 0
    with pytest.raises(pkt.TrussError) as ei:
        pkt.workspace_bytes(-1, 10)
    assert ei.value.name == "TRUSS_E_ARG"
    with pytest.raises(pkt.TrussError) as ei:
        pkt.workspace_bytes(10, 7)  # odd slot count
    assert ei.value.name == "TRUSS_E_ARG"
    with pytest.raises(pkt.TrussError) as ei:
        pkt.workspace_bytes(10, 2 * (2**31))  # m above 2^31 - 1
    assert ei.value.name == "TRUSS_E_RANGE"


def test_relabel_option_and_its_workspace(lib):
    # host only: relabel = 1 (auto, default) and 2 (always) need the relabelled CSR and the
    # permutation on top of the decomposition's own arrays (about 16 B per edge and 40 per
    # vertex); 0 does not; other values are rejected before any device work
    import paper_1707_02000_amd as pkt

    n, two_m = 100_000, 4_000_000
    plain = pkt.workspace_bytes(n, two_m, pkt.make_options(relabel="off"))
    auto = pkt.workspace_bytes(n, two_m)
    always = pkt.workspace_bytes(n, two_m, pkt.make_options(relabel="always"))
    assert auto == always == pkt.workspace_bytes(n, two_m, pkt.make_options(relabel=True))
    assert plain == pkt.workspace_bytes(n, two_m, pkt.make_options(relabel=False))
    assert auto - plain >= 16 * (two_m // 2) + 36 * n
    assert pkt.relabel_mode("auto") == 1 and pkt.relabel_mode(True) == 2 and pkt.relabel_mode(False) == 0
    o = pkt.default_options()
    o.relabel = 3
    assert lib.truss_decompose(4, None, None, None, None, 0, ctypes.byref(o), None, None) == 1
    assert b"relabel" in lib.truss_last_error()


def test_strerror_covers_every_status(lib):
    for code in range(8):
        assert lib.truss_strerror(code)
    assert b"unknown" in lib.truss_strerror(99)


def test_bad_arguments_rejected_before_device_work(lib):
    # n < 0 and bad option values are rejected before any HIP call
    import paper_1707_02000_amd as pkt

    code = lib.truss_decompose(-1, None, None, None, None, 0, None, None, None)
    assert code == 1
    o = pkt.default_options()
    o.variant = 42
    code = lib.truss_decompose(4, None, None, None, None, 0, ctypes.byref(o), None, None)
    assert code == 1
    o = pkt.default_options()
    o.device_loop = 7
    code = lib.truss_decompose(4, None, None, None, None, 0, ctypes.byref(o), None, None)
    assert code == 1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1707_02000_amd as pkt

    monkeypatch.setattr(pkt, "_lib", None)
    monkeypatch.setattr(pkt, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        pkt.load()


def test_product_code_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1707_02000_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
                assert "wc_truss" not in text, f


def _ws(lib, name, *args):
    nb = ctypes.c_size_t(0)
    code = getattr(lib, name)(*args, ctypes.byref(nb))
    return code, nb.value


def test_workspace_sizes_of_the_other_entry_points(lib):
    # host only: sizes grow with the input, stay 256-byte multiples, and cover the
    # per-slot and per-vertex arrays each call carves out
    for name in ("truss_ktruss_workspace_bytes", "truss_kcore_workspace_bytes",
                 "truss_kco_order_workspace_bytes", "truss_kco_map_workspace_bytes"):
        c1, a = _ws(lib, name, 1000)
        c2, b = _ws(lib, name, 100_000)
        assert c1 == 0 and c2 == 0 and 0 < a < b and a % 256 == 0 and b % 256 == 0, name
        assert _ws(lib, name, -1)[0] == 1, name
    c, a = _ws(lib, "truss_kcore_workspace_bytes", 1 << 20)
    assert a >= 5 * 4 * (1 << 20) + 8 * (1 << 20)  # degrees, two alive lists, two frontiers, prefix
    for name, per_slot in (("truss_kco_relabel_workspace_bytes", 16), ("truss_hindex_workspace_bytes", 9)):
        c1, a = _ws(lib, name, 1000, 20_000)
        c2, b = _ws(lib, name, 1000, 2_000_000)
        assert c1 == 0 and c2 == 0 and a < b and b >= per_slot * 2_000_000, name
        assert _ws(lib, name, -1, 10)[0] == 1 and _ws(lib, name, 10, -2)[0] == 1, name
    assert lib.truss_kco_order_workspace_bytes(10, None) == 1


def test_other_entry_points_reject_bad_arguments_before_device_work(lib):
    # every check here returns before the first HIP call, so it runs without a GPU
    vp = ctypes.c_void_p
    assert lib.truss_ktruss(3, -1, None, None, None, 3, None, None, None, 0, None) == 1  # m < 0
    assert lib.truss_ktruss(3, 1, None, None, None, 1, None, None, None, 0, None) == 1  # k < 2
    assert lib.truss_ktruss(3, 2, None, None, None, 3, None, None, None, 0, None) == 1  # NULL edges
    assert lib.truss_kcore(-1, None, None, None, None, None, 0, None) == 1
    assert lib.truss_kcore(4, None, None, None, None, None, 0, None) == 1  # NULL offsets
    host = (ctypes.c_int64 * 8)()
    # a workspace too small or misaligned is refused before the offsets are read
    assert lib.truss_kcore(4, host, host, host, None, None, 0, None) == 5
    assert lib.truss_kco_order(-1, None, None, None, None, 0, None) == 1
    assert lib.truss_kco_order(4, None, host, host, None, 0, None) == 1  # NULL core
    assert lib.truss_kco_order(4, host, host, host, vp(4096 + 8), 1 << 20, None) == 5  # misaligned
    assert lib.truss_kco_relabel(-1, None, None, None, None, host, None, None, 0, None) == 1
    assert lib.truss_kco_relabel(4, host, host, host, host, None, None, None, 0, None) == 1  # NULL offsets2
    assert lib.truss_kco_map(-1, 0, None, None, None, None, None, None, None, None, 0, None) == 1
    assert lib.truss_kco_map(0, 3, host, host, None, None, host, host, host, None, 0, None) == 1  # m > 0, n = 0
    sweeps, conv = ctypes.c_int32(7), ctypes.c_int32(7)
    assert lib.truss_hindex(-1, None, None, None, -1, ctypes.byref(sweeps), ctypes.byref(conv), None, 0,
                            None) == 1
    assert sweeps.value == 0 and conv.value == 0  # outputs cleared first
    assert lib.truss_hindex(4, None, None, None, -1, None, None, None, 0, None) == 1  # NULL offsets
    assert lib.truss_last_error()
