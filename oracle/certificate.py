"""CPU ORACLE (test infrastructure): checks of a trussness array that hold at any size.

The full oracle (the serial bucket peel) takes hours on the largest synthetic inputs,
so there the GPU result is checked against the definition of the k-truss
(Background section) through a certificate instead, on sampled edges:

* lower bound -- every edge e with trussness k lies in at least k - 2 triangles
  whose other two edges also have trussness >= k.  Then the edges of trussness
  >= k form a subgraph in which every edge has support >= k - 2, so it lies in
  the maximal one, and no trussness is overstated.
* upper bound -- a peeling order (rank: equal values mean removed together)
  that never removes an edge of lower trussness after one of higher trussness,
  and under which no edge e of trussness k had more than k - 2 triangles left
  when it was removed (other two edges of rank >= rank(e)).  Then no edge of
  trussness k can lie in the (k+1)-truss: the member of lowest rank of that
  subgraph would have had at least k - 1 triangles left when removed.

The bucket peel's removal steps and the level loop's round indices are both such
orders.  Both bounds are checked edge by edge from the CSR rows; the monotone
order check runs over all edges.
"""
from __future__ import annotations

import numpy as np

from . import edge_ids


def monotone_order(tau: np.ndarray, rank: np.ndarray) -> bool:
    """Every edge of lower trussness has a strictly lower rank than every edge of higher trussness.

    Holds iff all edges of one rank share one trussness and that trussness does not
    decrease as the rank grows.  O(m) with one array of the rank range.
    """
    tau = np.asarray(tau, np.int64)
    rank = np.asarray(rank, np.int64)
    if len(tau) == 0:
        return True
    if rank.min() < 0:
        return False
    per_rank = np.full(int(rank.max()) + 1, -1, np.int64)
    per_rank[rank] = tau  # one representative per rank
    if not np.array_equal(per_rank[rank], tau):
        return False
    present = per_rank[per_rank >= 0]
    return bool(np.all(np.diff(present) >= 0))


class Certificate:
    """Checks edges of one graph; builds the slot -> edge id map once."""

    def __init__(self, g):
        self.off = np.asarray(g.offsets, np.int64)
        self.adj = np.asarray(g.adj, np.int32)
        self.el, self.eid = edge_ids(g)

    def partners(self, e: int):
        """Edge ids (a, b) of the two other edges of every triangle on edge e."""
        u, v = int(self.el[e, 0]), int(self.el[e, 1])
        ou, ov = self.off[u], self.off[v]
        ru = self.adj[ou:self.off[u + 1]]
        rv = self.adj[ov:self.off[v + 1]]
        _, iu, iv = np.intersect1d(ru, rv, assume_unique=True, return_indices=True)
        return self.eid[ou + iu], self.eid[ov + iv]

    def check(self, tau: np.ndarray, rank: np.ndarray, edges) -> dict:
        """Lower and upper bound on the given edges; lists the edges that fail each."""
        bad_lo, bad_hi = [], []
        for e in np.asarray(edges, np.int64):
            a, b = self.partners(int(e))
            k = int(tau[e])
            if int(np.count_nonzero((tau[a] >= k) & (tau[b] >= k))) < k - 2:
                bad_lo.append(int(e))
            re = rank[e]
            if int(np.count_nonzero((rank[a] >= re) & (rank[b] >= re))) > k - 2:
                bad_hi.append(int(e))
        return {"checked": len(edges), "lower_bound_fails": bad_lo, "upper_bound_fails": bad_hi}


def sample_edges(tau: np.ndarray, n_uniform: int, per_value: int, seed: int = 1) -> np.ndarray:
    """A uniform sample plus up to per_value edges of every trussness value present.

    Linear passes only (no sort of all edges), so it scales to the full-size inputs.
    """
    tau = np.asarray(tau)
    rng = np.random.default_rng(seed)
    m = len(tau)
    if m == 0:
        return np.zeros(0, np.int64)
    uni = np.unique(rng.integers(0, m, size=min(n_uniform, m)))
    counts = np.bincount(tau)
    have = np.bincount(tau[uni], minlength=len(counts))
    short = (counts > 0) & (have < np.minimum(counts, per_value))
    picks = [uni]
    if short.any():
        cand = np.flatnonzero(short[tau])  # edges of the values the uniform sample left short
        for k in np.flatnonzero(short):
            ids = cand[tau[cand] == k]
            picks.append(rng.choice(ids, size=min(per_value, len(ids)), replace=False))
    return np.unique(np.concatenate(picks))


def verify(g, tau: np.ndarray, rank: np.ndarray, edges=None) -> dict:
    """Monotone order over all edges, both bounds on `edges` (all edges when None)."""
    tau = np.asarray(tau)
    rank = np.asarray(rank)
    cert = Certificate(g)
    if edges is None:
        edges = np.arange(len(tau))
    out = cert.check(tau, rank, edges)
    out["monotone"] = monotone_order(tau, rank)
    out["ok"] = out["monotone"] and not out["lower_bound_fails"] and not out["upper_bound_fails"]
    return out
