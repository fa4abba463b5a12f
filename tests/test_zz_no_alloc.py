"""dg_pr_read_noalloc: the no-allocation variant of dg_pr_read, called through
the C ABI and compared with dg_pr_read (bit for bit, and within max-abs 1e-10 of
the oracle) on two calls in a row, the second on a smaller graph; it allocates
nothing (the allocator hook sees no call), and a host read above its staging
limit is refused."""
import ctypes
import gc
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_11094_amd as dg

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def read_noalloc(q, out=None):
    lib = dg.load_library()
    it, cv = ctypes.c_int32(), ctypes.c_int32()
    if out is not None:
        dg._check(lib.dg_pr_read_noalloc(q.handle, ctypes.c_void_p(out.data_ptr()), ctypes.byref(it),
                                         ctypes.byref(cv), dg.DG_DEVICE_PTRS))
        return out.cpu().numpy(), it.value, bool(cv.value)
    rank = np.empty(q.graph.n, np.float64)
    dg._check(lib.dg_pr_read_noalloc(q.handle, rank.ctypes.data, ctypes.byref(it), ctypes.byref(cv), 0))
    return rank, it.value, bool(cv.value)


def test_noalloc_read_matches_read_twice_then_smaller():
    import torch

    gc.collect()
    hook = dg.use_torch_allocator()  # counts every device allocation of the library
    graphs = []
    try:
        for scale, inst in ((14, 60), (10, 61)):  # the second call on a smaller graph
            n, s, d, w = graphgen.rmat_directed(scale, 16 << scale, graphgen.config_seed(0, inst))
            b = graphgen.update_batch(n, s, d, int(0.01 * s.size), graphgen.config_seed(0, inst + 10))
            say("no-alloc PageRank read, R-MAT scale", scale)
            G = dg.Graph(n, s, d, w)
            graphs.append(G)
            q = G.pr_attach(0.85, 1e-9, 1000)
            G.apply(*b)
            torch.cuda.synchronize()
            before = hook.allocs
            got, it, cv = read_noalloc(q)
            dev = torch.empty(n, dtype=torch.float64, device="cuda:0")
            got_dev, _, _ = read_noalloc(q, dev)
            assert hook.allocs == before, "the no-allocation read allocated"
            want, it2, cv2 = q.read()  # the allocating read (stages through the library's buffer)
            assert (it, cv) == (it2, cv2)
            assert np.array_equal(got, want) and np.array_equal(got_dev, want)
            cs, cd, _, _ = oracle.apply(n, s, d, w, *b)
            pr, _, _ = oracle.pagerank(n, cs, cd, 0.85, 1e-9, 1000)
            assert float(np.max(np.abs(got - pr))) <= 1e-10
    finally:
        for G in graphs:
            G.close()
        dg.use_default_allocator()


def test_noalloc_host_read_limit():
    import torch

    n = dg.DG_NOALLOC_MAX_HOST_N + 1
    say("no-alloc host read refused above", dg.DG_NOALLOC_MAX_HOST_N)
    s = np.arange(0, n - 1, dtype=np.int32)
    G = dg.Graph(n, s, s + 1, np.ones(n - 1, np.int32))
    q = G.pr_attach(0.85, 1e-9, 1000)
    with pytest.raises(dg.DGError) as e:
        read_noalloc(q)
    assert e.value.code == dg.DG_EINVAL
    dev = torch.empty(n, dtype=torch.float64, device="cuda:0")
    got, _, _ = read_noalloc(q, dev)  # device output has no limit
    want, _, _ = q.read()
    assert np.array_equal(got, want)
    G.close()
