"""CPU model of the output positions the CSR merge tiles compute (no GPU needed).

The merge (Section 3.5) folds the diff level into the base rows and drops the
tombstones.  The tile kernel places entries without reading new row offsets: when
the merge runs, the diff level holds live entries only, so a live base entry i of
row r lands at

    i - (tombstones before i) + doff[r] + (diff entries of row r below it)

and a diff entry q of row r at

    (row start) + (q - doff[r]) + (live base entries of row r below it),
    row start = off[r] - (tombstones before off[r]) + doff[r],

where the tombstones before an index come from per-block counters (blocks of 256
base entries) plus a count inside the block.  This model checks both formulas
against the merge written as its definition (each row's live base entries and
diff entries sorted together, rows concatenated), on random rows with tombstones,
empty rows, rows with only diff entries and a hub row longer than several blocks.
"""

import numpy as np

BLOCK = 256  # base entries per tombstone counter block


def random_level(seed, n=3000):
    """Base rows (sorted columns, some tombstoned) and a diff level of live entries
    whose columns are absent from the same row's base part."""
    rng = np.random.default_rng(seed)
    deg = rng.poisson(4, n)
    deg[rng.random(n) < 0.2] = 0          # empty base rows
    deg[17] = 3 * BLOCK + 41              # a hub spanning several counter blocks
    base_rows, diff_rows, dead_rows = [], [], []
    for r in range(n):
        cols = np.sort(rng.choice(n, size=min(deg[r], n - 1), replace=False))
        dead = rng.random(cols.size) < 0.3
        free = np.setdiff1d(np.arange(n), cols)
        k = rng.poisson(1.5) if r % 7 else 0
        dcols = np.sort(rng.choice(free, size=min(k, free.size), replace=False))
        base_rows.append(cols)
        dead_rows.append(dead)
        diff_rows.append(dcols)
    off = np.concatenate([[0], np.cumsum([c.size for c in base_rows])])
    doff = np.concatenate([[0], np.cumsum([c.size for c in diff_rows])])
    col = np.concatenate(base_rows) if off[-1] else np.zeros(0, np.int64)
    dead = np.concatenate(dead_rows) if off[-1] else np.zeros(0, bool)
    dcol = np.concatenate(diff_rows) if doff[-1] else np.zeros(0, np.int64)
    return n, off, col, dead, doff, dcol


def merged_by_definition(n, off, col, dead, doff, dcol):
    """Output position of every live base entry and every diff entry."""
    pos_base, pos_diff = {}, {}
    o = 0
    for r in range(n):
        items = [(col[i], 0, i) for i in range(off[r], off[r + 1]) if not dead[i]]
        items += [(dcol[q], 1, q) for q in range(doff[r], doff[r + 1])]
        for c, kind, idx in sorted(items):
            (pos_base if kind == 0 else pos_diff)[idx] = o
            o += 1
    return pos_base, pos_diff, o


def tombstones_before(dead):
    """The tile kernel's count: per-block counters plus a count inside the block."""
    blocks = (dead.size + BLOCK - 1) // BLOCK
    per_block = np.array([dead[b * BLOCK:(b + 1) * BLOCK].sum() for b in range(blocks)], np.int64)
    tb = np.concatenate([[0], np.cumsum(per_block)])

    def count(i):
        b = i // BLOCK
        return int(tb[b] + dead[b * BLOCK:i].sum())

    return count


def test_merge_positions_match_the_definition():
    for seed in (1, 2, 3):
        n, off, col, dead, doff, dcol = random_level(seed)
        pos_base, pos_diff, total = merged_by_definition(n, off, col, dead, doff, dcol)
        assert total == int((~dead).sum()) + dcol.size
        tomb = tombstones_before(dead)
        for r in range(n):
            dl, dh = doff[r], doff[r + 1]
            row_start = off[r] - tomb(off[r]) + dl
            live = [i for i in range(off[r], off[r + 1]) if not dead[i]]
            for i in live:
                below = int(np.searchsorted(dcol[dl:dh], col[i]))
                assert i - tomb(i) + dl + below == pos_base[i], (seed, r, i)
            live_cols = np.array([col[i] for i in live], np.int64)
            for q in range(dl, dh):
                below = int(np.searchsorted(live_cols, dcol[q]))
                assert row_start + (q - dl) + below == pos_diff[q], (seed, r, q)


def test_positions_need_a_live_diff_level():
    """The formula takes doff[r] as the count of diff entries before row r, which
    holds only when every diff entry survives the merge: a killed diff entry left
    in the level shifts every later row by one (why the merge runs after the diff
    rebuild, which drops killed entries)."""
    n, off, col, dead, doff, dcol = random_level(4)
    pos_base, _, _ = merged_by_definition(n, off, col, dead, doff, dcol)
    # count one more (killed) diff entry in row 5: rows after it are placed one
    # slot too far by the formula
    doff_killed = doff.copy()
    doff_killed[6:] += 1
    tomb = tombstones_before(dead)
    r = next(r for r in range(6, n) if any(not dead[i] for i in range(off[r], off[r + 1])))
    i = next(i for i in range(off[r], off[r + 1]) if not dead[i])
    dl = doff_killed[r]
    below = int(np.searchsorted(dcol[doff[r]:doff[r + 1]], col[i]))
    assert i - tomb(i) + dl + below == pos_base[i] + 1
