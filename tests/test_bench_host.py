"""Host logic of bench.py (CPU): the kernel hash that keeps stored counter
traffic from outliving the kernel it was measured on, the null reporting of
missing tallies, and the one-GPU guard."""
import importlib.util
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture
def csrc_copy(bench, tmp_path, monkeypatch):
    """A private copy of the kernel sources that the hash reads instead."""
    d = tmp_path / "csrc"
    shutil.copytree(bench.CSRC, d)
    monkeypatch.setattr(bench, "CSRC", str(d))
    return d


def edit(path, old, new):
    text = path.read_text()
    assert text.count(old) == 1, old
    path.write_text(text.replace(old, new))


def test_hash_tracks_body_helpers_and_constants(bench, csrc_copy):
    f = csrc_copy / "tc.hip"
    h0 = bench.kernel_sha1("tc.hip", "k_tc_delta")
    assert len(h0) == 40
    # a constant only the static count uses leaves the delta kernel's hash alone
    edit(f, "constexpr int TCF_CAP", "constexpr int  TCF_CAP")
    assert bench.kernel_sha1("tc.hip", "k_tc_delta") == h0
    # a constant the kernel uses
    edit(f, "constexpr int TC_CHUNK = ", "constexpr int TC_CHUNK = 2 * ")
    h1 = bench.kernel_sha1("tc.hip", "k_tc_delta")
    assert h1 != h0
    # a device function of the same file that the kernel calls
    edit(f, "if (x < f[0]) return -1;", "if (x < f[0]) return -1;  // below the first fence")
    h2 = bench.kernel_sha1("tc.hip", "k_tc_delta")
    assert h2 != h1
    # the kernel's own body
    edit(f, "uint64_t acc = 0, walked = 0, probes = 0;\n    const int64_t items",
         "uint64_t acc = 0, walked = 0, probes = 0;\n    // items\n    const int64_t items")
    assert bench.kernel_sha1("tc.hip", "k_tc_delta") != h2
    assert bench.kernel_sha1("tc.hip", "no_such_kernel") == ""


def test_template_kernel_hash_covers_its_parameter_line(bench, csrc_copy):
    h0 = bench.kernel_sha1("pagerank.hip", "k_pr_tiles")
    edit(csrc_copy / "pagerank.hip", "template <bool STREAM, int ITEMS>\n__global__ __launch_bounds__(MP_THREADS) void k_pr_tiles(",
         "template <bool STREAM, int  ITEMS>\n__global__ __launch_bounds__(MP_THREADS) void k_pr_tiles(")
    assert bench.kernel_sha1("pagerank.hip", "k_pr_tiles") != h0


def test_stale_or_foreign_traffic_is_null(bench, csrc_copy):
    for (kernel, workload), e in bench.MEASURED_TRAFFIC.items():
        order = e.get("vertex_order")
        if bench.kernel_sha1(e["source"], kernel) != e["sha1"]:
            continue  # already stale in this tree: reported as null, nothing to check
        want = round(e["fetch_kib"] * 1024 / e["fetch_factor"] + e["write_kib"] * 1024 / e["write_factor"])
        assert bench.traffic_for(kernel, workload, order) == want
        assert bench.traffic_for(kernel, workload + "-other") is None
        if order is not None:
            assert bench.traffic_for(kernel, workload, 1 - order) is None
    # any edit to the measured kernel makes every figure for it stale
    edit(csrc_copy / "tc.hip", "constexpr int TC_CHUNK = ", "constexpr int TC_CHUNK = 2 * ")
    assert bench.traffic_for("k_tc_delta", "rmat20-undirected-dynamic-tc", 0) is None


def test_gteps_null_without_a_tally(bench):
    assert bench.gteps_of([{"edges_traversed": 0}, {"edges_traversed": 0}], 1.0) is None
    assert bench.gteps_of([{"edges_traversed": 2_000_000_000}], 2.0) == 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "--gpus must be 1" in r.stderr
    assert r.stdout == ""
