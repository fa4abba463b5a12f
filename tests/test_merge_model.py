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


# ---- the tile kernel's own steps --------------------------------------------------
# A step-by-step copy of the merge tile kernel's index logic (partition, per-wave
# tombstone counts, the column before an entry taken from the neighbouring lane or
# the wave before, the row left open at the tile's end) and of the pass for rows
# with an empty base part.  Whether a tile's diff entries sit in LDS or are read
# from memory changes where the kernel reads them, not what it compares, so the
# copy reads them in one place; the inputs still include a row with more diff
# entries than any tile stages.  Every output slot must be written exactly once,
# with the entry the definition puts there.

ID_MASK, MARK, DEAD = 0x3FFFFFFF, 0x40000000, 0x80000000
THREADS, WAVE = 256, 64


def partition(off, n, m, items, nb):
    rows, edges = [], []
    for b in range(nb + 1):
        diag = min(b * items, n + m)
        lo, hi = max(diag - m, 0), min(diag, n)
        while lo < hi:
            p = (lo + hi) >> 1
            if off[p + 1] <= diag - p - 1:
                lo = p + 1
            else:
                hi = p
        rows.append(lo)
        edges.append(diag - lo)
    return rows, edges


def lower(dcol, lo, hi, v):
    while lo < hi:
        mid = (lo + hi) >> 1
        if (dcol[mid] & ID_MASK) < v:
            lo = mid + 1
        else:
            hi = mid
    return lo


def emulate_merge(n, off, col, w, doff, dcol, dw, items, keep=0xFFFFFFFF):
    m, dm = int(off[n]), int(doff[n])
    ipt, waves = items // THREADS, THREADS // WAVE
    dead = [(c & DEAD) != 0 for c in col]
    m2 = m - sum(dead) + dm
    out_c, out_w = [None] * m2, [None] * m2

    def put(o, c, wt):
        assert 0 <= o < m2 and out_c[o] is None, o
        out_c[o], out_w[o] = c & keep, wt

    nblk = (m + BLOCK - 1) // BLOCK
    tb = [0]
    for b in range(nblk):
        tb.append(tb[-1] + sum(dead[b * BLOCK:(b + 1) * BLOCK]))
    tb.append(tb[-1])
    nb = (n + m + items - 1) // items
    mp_row, mp_edge = partition(off, n, m, items, nb)
    for b in range(nb):
        r0, r1, e0 = mp_row[b], mp_row[b + 1], mp_edge[b]
        ne, nr = mp_edge[b + 1] - e0, r1 - r0
        dbase = int(doff[r0])
        ndt = int(doff[min(r1 + 1, n)]) - dbase
        assert ndt >= 0
        s_off, s_dlo, s_open = {}, {}, None
        for i in range(nr + 2):
            r = r0 + i
            if r > n:
                continue
            s_dlo[i] = int(doff[r]) - dbase
            if i <= nr:
                o = int(off[r]) - e0
                s_off[i] = -1 if o < 0 else o
            else:
                s_open = int(off[r])
        st = (e0 // BLOCK) * BLOCK
        pre = tb[e0 // BLOCK] + sum(dead[st:e0])
        c = [col[e0 + j] if j < ne else 0 for j in range(items)]
        wts = [w[e0 + j] if j < ne else 0 for j in range(items)]
        s_wd = [[sum(1 for l in range(WAVE) if c[u * THREADS + wv * WAVE + l] & DEAD) for wv in range(waves)]
                for u in range(ipt)]
        s_last = [[None] + [c[u * THREADS + wv * WAVE + WAVE - 1] for wv in range(waves)] for u in range(ipt)]
        s_last[0][0] = col[e0 - 1] if e0 > 0 else None

        def lo_of(v):
            return lower(dcol, dbase + s_dlo_lo, dbase + s_dlo_hi, v) - dbase

        for u in range(ipt):
            for t in range(THREADS):
                wv, l = t // WAVE, t % WAVE
                j = u * THREADS + t
                if j >= ne:
                    continue
                i = e0 + j
                lp = sum(1 for q in range(l) if c[u * THREADS + wv * WAVE + q] & DEAD)
                dead_g = pre + sum(s_wd[u][:wv]) + lp
                lo, hi = 0, nr
                while lo < hi:
                    mid = (lo + hi + 1) >> 1
                    if s_off[mid] <= j:
                        lo = mid
                    else:
                        hi = mid - 1
                ro = int(off[r0]) if lo == 0 else e0 + s_off[lo]
                cu = c[j]
                cur, is_dead = cu & ID_MASK, (cu & DEAD) != 0
                s_dlo_lo, s_dlo_hi = s_dlo[lo], s_dlo[lo + 1]
                base0 = i - dead_g + dbase + s_dlo_lo
                if s_dlo_lo == s_dlo_hi:
                    if not is_dead:
                        put(base0, cu, wts[j])
                    continue
                bq = lo_of(cur)
                if not is_dead:
                    put(base0 + (bq - s_dlo_lo), cu, wts[j])
                a = s_dlo_lo
                if i > ro:
                    if l > 0:
                        p = c[j - 1]
                    elif wv > 0:
                        p = s_last[u][wv]
                    elif u > 0:
                        p = s_last[u - 1][waves]
                    else:
                        p = s_last[0][0]
                    a = lo_of((p & ID_MASK) + 1)
                for q in range(a, bq):
                    put(base0 + (q - s_dlo_lo), dcol[dbase + q], dw[dbase + q])
                rend = e0 + s_off[lo + 1] if lo < nr else s_open
                if i == rend - 1:
                    after = 0 if is_dead else 1
                    for q in range(lo_of(cur + 1), s_dlo_hi):
                        put(base0 + after + (q - s_dlo_lo), dcol[dbase + q], dw[dbase + q])
            pre += sum(s_wd[u])
    # rows with an empty base part
    live_deg = [sum(1 for i in range(off[r], off[r + 1]) if not dead[i]) + int(doff[r + 1] - doff[r])
                for r in range(n)]
    off2 = np.concatenate([[0], np.cumsum(live_deg)])
    for jd in range(dm):
        r = int(np.searchsorted(doff, jd, side="right") - 1)
        if off[r] != off[r + 1]:
            continue
        put(int(off2[r]) + (jd - int(doff[r])), dcol[jd], dw[jd])
    assert all(x is not None for x in out_c)
    return out_c, out_w


def flagged_level(seed, n=700):
    """Rows as the merge meets them: sorted base ids with DEAD and MARK flags, a
    diff level of live ids (MARK on some) absent from the row's base part, empty
    rows, a hub spanning many tiles and a row with more diff entries than a tile
    stages."""
    rng = np.random.default_rng(seed)
    base, diff = [], []
    for r in range(n):
        k = 0 if rng.random() < 0.25 else int(rng.poisson(5))
        if r == 3:
            k = 2600
        ids = np.sort(rng.choice(n * 8, size=k, replace=False)).astype(np.int64)
        flags = np.where(rng.random(k) < 0.3, DEAD, np.where(rng.random(k) < 0.2, MARK, 0))
        free = np.setdiff1d(np.arange(n * 8), ids)
        kd = 300 if r == 5 else (int(rng.poisson(1.2)) if r % 5 else 0)
        dids = np.sort(rng.choice(free, size=kd, replace=False)).astype(np.int64)
        dflags = np.where(rng.random(kd) < 0.3, MARK, 0)
        base.append((ids | flags, rng.integers(1, 100, k)))
        diff.append((dids | dflags, rng.integers(1, 100, kd)))
    off = np.concatenate([[0], np.cumsum([b[0].size for b in base])])
    doff = np.concatenate([[0], np.cumsum([d[0].size for d in diff])])
    col = [int(x) for b in base for x in b[0]]
    w = [int(x) for b in base for x in b[1]]
    dcol = [int(x) for d in diff for x in d[0]]
    dw = [int(x) for d in diff for x in d[1]]
    return n, off, col, w, doff, dcol, dw


def merged_flagged(n, off, col, w, doff, dcol, dw, keep):
    out_c, out_w = [], []
    for r in range(n):
        items = [(col[i] & ID_MASK, col[i], w[i]) for i in range(off[r], off[r + 1]) if not col[i] & DEAD]
        items += [(dcol[q] & ID_MASK, dcol[q], dw[q]) for q in range(doff[r], doff[r + 1])]
        for _, c, wt in sorted(items):
            out_c.append(c & keep)
            out_w.append(wt)
    return out_c, out_w


def test_tile_kernel_steps_give_the_merge():
    for seed, items, keep in ((7, 512, 0xFFFFFFFF), (8, 1024, 0xFFFFFFFF), (9, 2048, ~MARK & 0xFFFFFFFF)):
        n, off, col, w, doff, dcol, dw = flagged_level(seed)
        got = emulate_merge(n, off, col, w, doff, dcol, dw, items, keep)
        want = merged_flagged(n, off, col, w, doff, dcol, dw, keep)
        assert got[0] == want[0] and got[1] == want[1], (seed, items)
