"""The radix sort and exclusive scan the batch canonicalisation and the CSR
maintenance use (dg_sort_pairs, dg_scan_exclusive), on device tensors, against
numpy: a stable sort by the low `bits` bits (values carry the input position, so
the order of equal keys is checked exactly) and a cumulative sum.  Sizes cover
the empty case, single elements, partial and exact tiles (2,048 keys per sort
tile, 4,096 values per scan tile) and many tiles; keys cover every digit count,
all-equal keys and heavy repeats."""
import sys

import numpy as np
import pytest

import paper_2507_11094_amd as dg

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 63, 64, 65, 2047, 2048, 2049, 3 * 4096 + 17, 100_000, 1 << 20]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def sort_check(keys: np.ndarray, bits: int):
    import torch

    n = keys.size
    vals = np.arange(n, dtype=np.int32)
    dk = torch.from_numpy(keys.view(np.int64)).cuda()
    dv = torch.from_numpy(vals).cuda()
    ko, vo = dg.dg_sort_pairs(dk, dv, bits)
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(keys & mask, kind="stable")
    assert np.array_equal(ko.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(vo.cpu().numpy(), vals[order])
    # inputs untouched
    assert np.array_equal(dk.cpu().numpy().view(np.uint64), keys)


@pytest.mark.parametrize("n", SIZES)
def test_sort_random_keys(n):
    rng = np.random.default_rng(1000 + n)
    keys = rng.integers(0, 2**63, size=n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=n,
                                                                                          dtype=np.uint64)
    for bits in (1, 8, 9, 44, 64):
        say("sort n", n, "bits", bits)
        sort_check(keys, bits)


@pytest.mark.parametrize("bits", [3, 17, 31, 40, 57])
def test_sort_repeats_and_skew(bits):
    rng = np.random.default_rng(bits)
    n = 50_000
    say("sort repeats/skew bits", bits)
    sort_check(rng.integers(0, 16, size=n, dtype=np.uint64), bits)             # heavy repeats
    sort_check(np.full(n, 0xABCDEF0123456789, dtype=np.uint64), bits)          # all equal
    row = rng.zipf(1.5, size=n).astype(np.uint64) % np.uint64(1 << 20)        # skewed rows of (row, col) keys
    col = rng.integers(0, 1 << 20, size=n, dtype=np.uint64)
    sort_check((row << np.uint64(20)) | col, bits)


@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 3 * 4096 + 1, 1_000_000, 10_000_000])
def test_scan_exclusive(n):
    import torch

    rng = np.random.default_rng(77 + n)
    x = rng.integers(0, 1000, size=n, dtype=np.int64)
    if n > 10:
        x[rng.integers(0, n, size=n // 10)] = 0
    say("scan n", n)
    got = dg.dg_scan_exclusive(torch.from_numpy(x).cuda()).cpu().numpy()
    want = np.concatenate([[0], np.cumsum(x)[:-1]]) if n else x
    assert np.array_equal(got, want)


def test_scan_large_values():
    import torch

    n = 123_457
    x = np.full(n, (1 << 30) + 7, dtype=np.int64)  # total ~2^47: near the documented bound
    say("scan large values")
    got = dg.dg_scan_exclusive(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.array_equal(got, np.arange(n, dtype=np.int64) * x[0])
