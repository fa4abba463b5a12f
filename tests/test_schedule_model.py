"""CPU model behind the work-queue guard (no GPU needed).

The persistent work queue relaxes in FIFO order with one in-queue flag per
vertex, drained by thousands of waves at once, so improvements spread in rounds.
The library refuses that schedule when a breadth-first probe from the sources is
still discovering vertices after 64 hop levels.  This model shows why the guard
keys on hop depth: relaxation in rounds expands each vertex about twice on a
shallow R-MAT graph, while on a weighted grid the expansions per vertex grow
with the side (the hop depth), so a 4096 x 4096 grid would take hundreds.
"""

import numpy as np

import graphgen

GUARD_LEVELS = 64


def csr(n, s, d, w):
    order = np.lexsort((d, s))
    s, d, w = s[order], d[order], w[order]
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, s + 1, 1)
    return np.cumsum(off), d, w


def round_relaxations(n, s, d, w, source):
    """Vertex expansions of label-correcting relaxation in rounds: every vertex
    improved in a round is expanded in the next (a wide FIFO queue, as when
    thousands of waves drain one queue).  Returns (expansions, distances)."""
    off, col, wt = csr(n, s, d, w)
    big = np.int64(1) << 62
    dist = np.full(n, big, np.int64)
    dist[source] = 0
    front = np.array([source])
    pops = 0
    while front.size:
        pops += front.size
        starts, ends = off[front], off[front + 1]
        idx = np.concatenate([np.arange(a, b) for a, b in zip(starts.tolist(), ends.tolist())])
        cand = dist[np.repeat(front, ends - starts)] + wt[idx]
        best = np.full(n, big, np.int64)
        np.minimum.at(best, col[idx], cand)
        front = np.nonzero(best < dist)[0]
        dist[front] = best[front]
    return pops, dist


def hop_levels(n, s, d, source, limit):
    """Levels of a breadth-first search from source, stopping at limit."""
    off, col, _ = csr(n, s, d, np.zeros(s.size, np.int32))
    seen = np.zeros(n, bool)
    seen[source] = True
    front = np.array([source])
    levels = 0
    while front.size and levels < limit:
        nxt = np.concatenate([col[off[u]:off[u + 1]] for u in front.tolist()]) if front.size else front
        nxt = np.unique(nxt[~seen[nxt]]) if nxt.size else nxt
        seen[nxt] = True
        front = nxt
        levels += 1
    return levels, bool(front.size)


def test_fifo_work_grows_with_hop_depth_on_grids():
    per_vertex = {}
    for side in (32, 128, 256):
        n, s, d, w = graphgen.grid4(side, side, 5, 1000)
        pops, _ = round_relaxations(n, s, d, w, 0)
        per_vertex[side] = pops / n
        _, deep = hop_levels(n, s, d, 0, GUARD_LEVELS)
        assert deep == (2 * (side - 1) > GUARD_LEVELS)
    # expansions per vertex grow about linearly with the side beyond the guard's
    # depth (side / 20 here, so hundreds per vertex on a 4096 x 4096 grid)
    assert per_vertex[32] < per_vertex[128] < per_vertex[256]
    assert per_vertex[256] > 3.0 * per_vertex[32]
    assert per_vertex[256] > 256 / 25


def test_fifo_work_is_flat_on_shallow_rmat():
    n, s, d, w = graphgen.rmat_directed(11, 16 << 11, 21)
    pops, dist = round_relaxations(n, s, d, w, 0)
    reached = int((dist < (1 << 62)).sum())
    levels, deep = hop_levels(n, s, d, 0, GUARD_LEVELS)
    assert not deep and levels < 16
    assert pops <= 4 * reached
