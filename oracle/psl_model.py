"""CPU ORACLE -- test infrastructure only.

A step-by-step model of PKT's level-synchronous peeling (PKT section, Algorithms 4
and 5) in which the per-edge "threads" of one sub-level run interleaved at random,
one shared-memory operation at a time.  Plain reads of a support value may return
any value the location has held since the sub-level began (the weakest coherence a
GPU's non-atomic loads give); read-modify-writes are atomic.

Rules modelled for a frontier edge e1 = (u, v) at level l and each common neighbour
w, with e2 = (v, w), e3 = (u, w):
  * skip the triangle if e2 or e3 was processed in an earlier sub-level;
  * for (x, y) in ((e2, e3), (e3, e2)): if S[x] > l and (y is not in the frontier,
    or e1 is the owner of the triangle -- the lower id of e1 and y by the paper's
    rule, the higher id by its alternative), then a = atomic_sub(S[x], 1);
    if a == l + 1, x joins the next frontier; if a <= l, atomic_add(S[x], 1).
The paper's listing prints only the first of the two symmetric blocks and the text
describes the other; both are modelled.  ``owner="none"`` and ``restore=False``
switch a rule off, so a test can show that it matters.
"""
from __future__ import annotations

import random

ALIVE, CURR, NEXT, PROC = 0, 1, 2, 3


class Sublevel:
    """Shared state of one sub-level and its random scheduler."""

    def __init__(self, S, state, rng, stale_reads=True):
        self.S = S
        self.state = state
        self.rng = rng
        self.stale = stale_reads
        self.hist = {}
        self.next = []

    def read_S(self, x):
        h = self.hist.setdefault(x, [self.S[x]])
        if self.stale:
            return self.rng.choice(h)
        return self.S[x]

    def _log(self, x):
        self.hist.setdefault(x, []).append(self.S[x])

    def atomic_sub(self, x):
        a = self.S[x]
        self.hist.setdefault(x, [a])
        self.S[x] = a - 1
        self._log(x)
        return a

    def atomic_add(self, x):
        self.S[x] += 1
        self._log(x)


def _thread(sh, e1, u, v, adj, eid, l, owner, restore):
    common = sorted(adj[u] & adj[v])
    for w in common:
        e3 = eid[(min(u, w), max(u, w))]
        e2 = eid[(min(v, w), max(v, w))]
        st2 = sh.state[e2]
        yield
        st3 = sh.state[e3]
        yield
        if st2 == PROC or st3 == PROC:
            continue
        for x, y in ((e2, e3), (e3, e2)):
            sx = sh.read_S(x)
            yield
            y_in_curr = sh.state[y] == CURR
            yield
            if owner == "lower":
                mine = (not y_in_curr) or e1 < y
            elif owner == "higher":
                mine = (not y_in_curr) or e1 > y
            else:
                mine = True
            if sx > l and mine:
                a = sh.atomic_sub(x)
                yield
                if a == l + 1:
                    sh.next.append(x)
                    sh.state[x] = NEXT
                    yield
                if a <= l and restore:
                    sh.atomic_add(x)
                    yield


def process_sublevel(edges, S, state, curr, l, rng, owner="lower", restore=True, stale_reads=True):
    """Run one sub-level with a random interleaving; returns the next frontier (list of ids).

    ``edges`` is the canonical edge list (index = edge id); S and state are mutated.
    """
    adj = {}
    for a, b in edges:
        adj.setdefault(a, set()).add(b)
        adj.setdefault(b, set()).add(a)
    eid = {e: i for i, e in enumerate(edges)}
    sh = Sublevel(S, state, rng, stale_reads)
    threads = []
    for e1 in curr:
        u, v = edges[e1]
        threads.append(_thread(sh, e1, u, v, adj, eid, l, owner, restore))
    live = list(threads)
    while live:
        t = rng.randrange(len(live))
        try:
            next(live[t])
        except StopIteration:
            live[t] = live[-1]
            live.pop()
    return sh.next


def pkt(edges, seed=0, owner="lower", restore=True, stale_reads=True, trace=None):
    """Full level-synchronous decomposition under random interleavings.

    Returns trussness in canonical edge order.  ``trace``, if a list, receives one
    (l, S_start, state_start, curr, S_end, next) tuple per sub-level.
    """
    rng = random.Random(seed)
    E = list(edges)
    m = len(E)
    adj = {}
    for a, b in E:
        adj.setdefault(a, set()).add(b)
        adj.setdefault(b, set()).add(a)
    S = [len(adj[a] & adj[b]) for a, b in E]
    state = [ALIVE] * m
    todo = m
    l = 0
    guard = 0
    while todo > 0:
        curr = [e for e in range(m) if state[e] == ALIVE and S[e] == l]
        for e in curr:
            state[e] = CURR
        while curr:
            guard += 1
            if guard > 4 * m + 10:
                raise RuntimeError("sub-level count exceeded its bound")
            todo -= len(curr)
            S_start, st_start = list(S), list(state)
            nxt = process_sublevel(E, S, state, curr, l, rng, owner, restore, stale_reads)
            if trace is not None:
                trace.append((l, S_start, st_start, list(curr), list(S), list(nxt)))
            for e in curr:
                state[e] = PROC
            for e in nxt:
                state[e] = CURR
            curr = nxt
        l += 1
    return [s + 2 for s in S]


def sublevel_closed_form(edges, S_start, state_start, curr, l):
    """Expected (S_end, next set) of one sub-level, from counting destroyed triangles.

    A triangle is destroyed in the sub-level if it has an edge in the frontier and no
    edge processed earlier.  Each non-frontier edge x of it loses one unit of support,
    floored at l: S_end[x] = max(l, S_start[x] - D[x]); x joins the next frontier iff
    S_start[x] > l >= S_start[x] - D[x].
    """
    curr_set = set(curr)
    adj = {}
    for a, b in edges:
        adj.setdefault(a, set()).add(b)
        adj.setdefault(b, set()).add(a)
    eid = {e: i for i, e in enumerate(edges)}
    D = [0] * len(edges)
    seen = set()
    for e1 in curr:
        u, v = edges[e1]
        for w in adj[u] & adj[v]:
            tri = tuple(sorted((u, v, w)))
            if tri in seen:
                continue
            seen.add(tri)
            a, b, c = tri
            ids = (eid[(a, b)], eid[(a, c)], eid[(b, c)])
            if any(state_start[x] == PROC for x in ids):
                continue
            for x in ids:
                if x not in curr_set:
                    D[x] += 1
    S_end = list(S_start)
    nxt = set()
    for x in range(len(edges)):
        if x in curr_set or state_start[x] == PROC:
            continue
        S_end[x] = max(l, S_start[x] - D[x]) if S_start[x] > l else S_start[x]
        if S_start[x] > l and S_start[x] - D[x] <= l:
            nxt.add(x)
    return S_end, nxt
