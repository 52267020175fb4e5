"""Plant plausible mistakes in a copy of the C oracle (on the CPU, in a temp dir)
and show that the pins used in test_oracle_pins.py catch every one of them."""
import ctypes
import itertools
import multiprocessing as mp
import os
import random
import subprocess

import numpy as np
import pytest

import graphgen as gg
from oracle import definition as D

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "wc_truss.c")

MUTANTS = {
    "decrement_when_equal": ("if (S[x] > k) {", "if (S[x] >= k) {"),
    "check_only_one_other_edge": ("if (gone[f[0]] || gone[f[1]]) continue;", "if (gone[f[1]]) continue;"),
    "no_bin_shrink": ("bin[s]++;\n          S[x]--;", "S[x]--;"),
    "mirror_slot_in_wrong_row": ("find_slot(adj, off[v], off[v + 1], u);\n        if (k < 0) return ORC_EINPUT;",
                                 "find_slot(adj, off[u], off[u + 1], v);\n        if (k < 0) return ORC_EINPUT;"),
    "merge_skips_equal": ("if (adj[i] < adj[j])\n        ++i;", "if (adj[i] <= adj[j])\n        ++i;"),
    "level_off_by_one": ("tau[e] = k + 2;", "tau[e] = k + 1;"),
    "no_delete": ("gone[e] = 1;", "gone[e] = 0;"),
}


def _pins_pass(lib):
    def run(g):
        m = g.m
        off = np.ascontiguousarray(g.offsets, np.int64)
        adj = np.ascontiguousarray(g.adj if len(g.adj) else np.zeros(1, np.int32), np.int32)
        tau = np.zeros(max(m, 1), np.int32)
        r = lib.oracle_truss(g.n, off.ctypes.data_as(ctypes.c_void_p), adj.ctypes.data_as(ctypes.c_void_p),
                             tau.ctypes.data_as(ctypes.c_void_p), None, None)
        return None if r < 0 else tau[:m]

    for n in range(3, 9):  # closed form: K_n -> n
        t = run(gg.from_edges(n, itertools.combinations(range(n), 2)))
        if t is None or not np.all(t == n):
            return False
    rng = random.Random(0)
    for _ in range(150):  # brute force from the definition
        n = rng.randint(3, 14)
        p = rng.uniform(0.2, 0.9)
        E = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
        g = gg.from_edges(n, E)
        bf = D.truss_by_definition(D.edges_from_csr(g))
        t = run(g)
        if t is None or not np.array_equal(t, [bf[e] for e in D.edges_from_csr(g)]):
            return False
    return True


def _compile(src_text, tmp_path, name):
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-w", "-o", str(so), str(c)])
    lib = ctypes.CDLL(str(so))
    lib.oracle_truss.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 5
    lib.oracle_truss.restype = ctypes.c_int64
    return lib


def test_unmutated_copy_passes(tmp_path):
    assert _pins_pass(_compile(open(SRC).read(), tmp_path, "orig"))


def _child(path, q):
    import faulthandler

    faulthandler.disable()  # a crashing mutant is an expected outcome here
    lib = ctypes.CDLL(path)
    lib.oracle_truss.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 5
    lib.oracle_truss.restype = ctypes.c_int64
    q.put(_pins_pass(lib))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert old in text, f"mutation site for {name} not found"
    _compile(text.replace(old, new, 1), tmp_path, name)
    # a mutant may also crash; run it in a child process so a crash counts as caught
    ctx = mp.get_context("fork")
    q = ctx.Queue()
    p = ctx.Process(target=_child, args=(str(tmp_path / f"{name}.so"), q))
    p.start()
    p.join(120)
    if p.is_alive():
        p.kill()
        p.join()
        return  # a hang is caught too
    passed = q.get() if p.exitcode == 0 else False
    assert not passed
