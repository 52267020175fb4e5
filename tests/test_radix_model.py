"""A step-by-step model of the reordering's LSD radix pass (count, prefix, scatter) on
the CPU: per tile of 2048 pairs, sub-steps of 256 lanes in four waves of 64, the
stable rank of every pair among the tile's pairs of its digit (earlier sub-steps,
then lower waves, then lower lanes), the digit-major count matrix and its prefix,
and the LDS staging in digit order.  Its output must equal a stable sort by digit,
and whole sorts (several passes) a stable sort by key."""
import numpy as np
import pytest

BINS, WAVE, BLOCK, ITEMS = 256, 64, 256, 8
TILE = BLOCK * ITEMS


def tile_counts(keys, shift, t):
    h = np.zeros(BINS, np.int64)
    for i in range(t * TILE, min((t + 1) * TILE, len(keys))):
        h[(keys[i] >> shift) & (BINS - 1)] += 1
    return h


def radix_pass(keys, vals, shift):
    cnt = len(keys)
    tiles = (cnt + TILE - 1) // TILE
    hist = np.zeros((BINS, tiles), np.int64)  # digit-major: index d * tiles + t
    for t in range(tiles):
        hist[:, t] = tile_counts(keys, shift, t)
    flat = hist.reshape(-1)
    start = np.concatenate([[0], np.cumsum(flat)])[:-1].reshape(BINS, tiles)  # exclusive prefix
    okeys = np.full(cnt, -1, np.int64)
    ovals = np.full(cnt, -1, np.int64)
    for t in range(tiles):
        lstart = np.concatenate([[0], np.cumsum(hist[:, t])])[:-1]
        run = np.zeros(BINS, np.int64)
        lk = np.zeros(TILE, np.int64)
        lv = np.zeros(TILE, np.int64)
        for sub in range(ITEMS):
            idx = t * TILE + sub * BLOCK + np.arange(BLOCK)
            valid = idx < cnt
            d = np.where(valid, (keys[np.minimum(idx, cnt - 1)] >> shift) & (BINS - 1), 0)
            wc = np.zeros((BLOCK // WAVE, BINS), np.int64)
            lower = np.zeros(BLOCK, np.int64)
            for w in range(BLOCK // WAVE):  # equal-digit lanes of a wave
                for lane in range(WAVE):
                    tid = w * WAVE + lane
                    if valid[tid]:
                        same = valid[w * WAVE:(w + 1) * WAVE] & (d[w * WAVE:(w + 1) * WAVE] == d[tid])
                        lower[tid] = same[:lane].sum()
                        if lower[tid] == 0:
                            wc[w, d[tid]] = same.sum()
            for tid in range(BLOCK):
                if valid[tid]:
                    w = tid // WAVE
                    r = lstart[d[tid]] + run[d[tid]] + lower[tid] + wc[:w, d[tid]].sum()
                    lk[r] = keys[idx[tid]]
                    lv[r] = vals[idx[tid]]
            run += wc.sum(axis=0)
        total = int(hist[:, t].sum())
        for p in range(total):  # the tile leaves LDS in digit order
            dd = (lk[p] >> shift) & (BINS - 1)
            pos = start[dd, t] + (p - lstart[dd])
            okeys[pos] = lk[p]
            ovals[pos] = lv[p]
    assert (okeys >= 0).all() and (ovals >= 0).all()  # every place written once
    return okeys, ovals


@pytest.mark.parametrize("cnt,top,seed", [(1, 5, 0), (255, 3, 1), (2048, 255, 2), (2049, 70000, 3),
                                          (5000, 1, 4), (6500, 2**20, 5), (4096, 0, 6)])
def test_pass_is_a_stable_sort_by_digit(cnt, top, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, top + 1, cnt)
    vals = np.arange(cnt)
    for shift in (0, 8):
        k2, v2 = radix_pass(keys, vals, shift)
        order = np.argsort((keys >> shift) & (BINS - 1), kind="stable")
        assert np.array_equal(v2, vals[order]) and np.array_equal(k2, keys[order])


@pytest.mark.parametrize("cnt,bits,seed", [(3000, 10, 7), (4200, 20, 8), (2100, 17, 9)])
def test_passes_sort_by_key_keeping_ties_in_order(cnt, bits, seed):
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << bits, cnt)
    keys[: cnt // 3] = keys[cnt // 3: 2 * (cnt // 3)]  # many equal keys
    vals = np.arange(cnt)
    k, v = keys, vals
    for shift in range(0, bits, 8):
        k, v = radix_pass(k, v, shift)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(v, order) and np.array_equal(k, keys[order])
