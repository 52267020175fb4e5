"""CPU model of the one-wave-per-edge intersection (wave_edge in csrc/psl.h): the
64-lane chunked merge path -- each lane's entry located among the other row's 64
register values by a six-step shuffle search, then the chunk pointers advanced by
ballot counts -- and the bracketed per-lane search for skewed rows, written lane by
lane.  Both must find exactly the common entries of two sorted rows, each once, at
their positions in both rows."""
import numpy as np
import pytest

W = 64
BIG = np.iinfo(np.int32).max


def wave_rank(lv, s):
    pos = np.zeros(W, np.int64)
    step = W // 2
    while step >= 1:
        v = lv[pos + step - 1]
        pos = np.where(v < s, pos + step, pos)
        step //= 2
    return pos


def merge_model(S, L):
    a, b = len(S), len(L)
    found = []
    i = j = 0
    steps = 0
    lane = np.arange(W)
    while i < a and j < b:
        steps += 1
        sv = i + lane < a
        s = np.where(sv, S[np.minimum(i + lane, a - 1)], BIG)
        lv = np.where(j + lane < b, L[np.minimum(j + lane, b - 1)], BIG)
        pos = wave_rank(lv, s)
        hit = sv & (lv[pos] == s)
        found += [(i + k, j + int(pos[k])) for k in np.flatnonzero(hit)]
        s_last, l_last = s[W - 1], lv[W - 1]
        if s_last <= l_last:
            j += int(np.count_nonzero(lv <= s_last))
            i += W
        else:
            i += int(np.count_nonzero(sv & (s <= l_last)))
            j += W
    return found, steps


def search_model(S, L):
    a = len(S)
    found = []
    for i in range(0, a, W):
        chunk = S[i:i + W]
        lo = int(np.searchsorted(L, chunk[0], side="left"))
        hi = int(np.searchsorted(L, chunk[-1], side="right"))
        for k, s in enumerate(chunk):
            p = lo + int(np.searchsorted(L[lo:hi], s, side="left"))
            if p < hi and L[p] == s:
                found.append((i + k, p))
    return found


def truth(S, L):
    pos = {int(x): j for j, x in enumerate(L)}
    return [(i, pos[int(x)]) for i, x in enumerate(S) if int(x) in pos]


def rows(rng, a, b, universe, overlap):
    common = rng.choice(universe, size=min(a, b, int(overlap * min(a, b))), replace=False)
    rest = np.setdiff1d(np.arange(universe), common)
    sa = rng.choice(rest, size=a - len(common), replace=False)
    rest2 = np.setdiff1d(rest, sa)
    sb = rng.choice(rest2, size=b - len(common), replace=False)
    return np.sort(np.concatenate([common, sa])).astype(np.int64), np.sort(np.concatenate([common, sb])).astype(np.int64)


@pytest.mark.parametrize("a,b", [(1, 1), (1, 64), (63, 64), (64, 64), (65, 64), (64, 65), (100, 700), (700, 100),
                                 (129, 130), (500, 520), (3, 400), (1000, 1000), (200, 1600), (5, 5000)])
@pytest.mark.parametrize("overlap", [0.0, 0.3, 1.0])
def test_merge_and_search_find_every_common_entry_once(a, b, overlap):
    rng = np.random.default_rng(a * 1000 + b + int(overlap * 7))
    S, L = rows(rng, a, b, max(4 * (a + b), 64), overlap)
    want = truth(S, L)
    got, steps = merge_model(S, L)
    assert sorted(got) == want and len(set(got)) == len(got)
    assert steps <= (a + W - 1) // W + (b + W - 1) // W
    assert sorted(search_model(S, L)) == want


def test_interleaved_and_disjoint_ranges():
    # rows whose values interleave finely, and rows in disjoint ranges (one chunk pointer races ahead)
    S = np.arange(0, 2000, 2, dtype=np.int64)
    L = np.arange(1, 2000, 3, dtype=np.int64)
    assert sorted(merge_model(S, L)[0]) == truth(S, L)
    S2, L2 = np.arange(0, 300, dtype=np.int64), np.arange(1000, 1300, dtype=np.int64)
    got, steps = merge_model(S2, L2)
    assert got == [] and steps <= 10
    got, _ = merge_model(L2, S2)
    assert got == []


SLOTS, CAP = 512, 256


def slot(w):
    return ((int(w) * 0x9E3779B1) & 0xFFFFFFFF) >> (32 - 9)


def hash_model(S, L):
    """The LDS-hash variant (wave_intersect_hash) lane by lane: the longer row into an
    open-addressing table of 512 slots (linear probing) with each key's position, then
    every shorter-row entry probed."""
    assert len(L) <= CAP
    keys = [-1] * SLOTS
    pos = [0] * SLOTS
    for j, w in enumerate(L):
        h = slot(w)
        while keys[h] != -1:
            h = (h + 1) & (SLOTS - 1)
        keys[h], pos[h] = int(w), j
    found = []
    for i, s in enumerate(S):
        h = slot(s)
        while keys[h] != -1:
            if keys[h] == s:
                found.append((i, pos[h]))
                break
            h = (h + 1) & (SLOTS - 1)
    return found


@pytest.mark.parametrize("a,b", [(1, 1), (5, 256), (256, 256), (40, 100), (300, 256), (3, 17)])
@pytest.mark.parametrize("overlap", [0.0, 0.5, 1.0])
def test_hash_finds_every_common_entry_once(a, b, overlap):
    rng = np.random.default_rng(7 * a + b)
    S, L = rows(rng, a, b, max(4 * (a + b), 64), overlap)
    assert sorted(hash_model(S, L)) == truth(S, L)


def test_hash_clusters_and_large_ids():
    # ids that share the hash's top bits cluster into long probe runs; ids near 2^31
    L = np.array(sorted({(k << 23) for k in range(200)} | {2**31 - 2 - k for k in range(56)}), np.int64)
    S = L[::3].copy()
    assert sorted(hash_model(S, L)) == truth(S, L)


# ---- the grouped search of a small round's item (group_item in csrc/peel.hip)

def group_search(adj, lb, le, w, G):
    """G lanes find the first entry of adj[lb:le] not below w: G evenly spaced entries
    of the open range per step, their count below w narrows it; then one last load of
    at most G entries.  Returns (position, steps)."""
    def gather(q, hi):
        out = np.full(G, BIG, np.int64)
        m = q < hi
        out[m] = adj[q[m]]
        return out

    lo, hi, steps = lb, le, 0
    while hi - lo > G:
        step = (hi - lo + G - 1) // G
        v = gather(lo + np.arange(G) * step, hi)
        below = int(np.count_nonzero(v < w))
        assert np.all(v[:below] < w) and np.all(v[below:] >= w)  # a prefix of the lanes
        nhi = min(lo + below * step, hi)
        if below > 0:
            lo += (below - 1) * step + 1
        hi = nhi
        steps += 1
    v = gather(lo + np.arange(G), hi)
    return lo + int(np.count_nonzero(v < w)), steps


@pytest.mark.parametrize("G", [8, 16, 32, 64])
def test_group_search_is_a_lower_bound(G):
    rng = np.random.default_rng(G)
    for t in range(1500):
        L = int(rng.integers(0, 3000)) if t % 3 else int(rng.integers(0, 2 * G + 3))
        row = np.sort(rng.choice(100_000, size=L, replace=False)).astype(np.int64)
        pad = int(rng.integers(0, 5))
        adj = np.concatenate([np.sort(rng.integers(0, 100_000, pad)), row,
                              np.sort(rng.integers(0, 100_000, pad))]).astype(np.int64)
        w = int(rng.choice(row)) if (L and t % 2) else int(rng.integers(0, 100_001))
        p, steps = group_search(adj, pad, pad + L, w, G)
        assert p == pad + int(np.searchsorted(row, w))
        bound = 0
        while G ** (bound + 1) < L:
            bound += 1
        assert steps <= bound + 1
