"""Host-side parts of bench.py: the one-GPU guard, the switched-off workload and
the lookup of measured HBM traffic (no GPU needed)."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_batched64_is_switched_off():
    r = run_bench("--workload", "batched64")
    assert r.returncode == 2 and "switched off" in r.stderr and r.stdout == ""


def test_traffic_lookup_needs_matching_source_hash(tmp_path, monkeypatch):
    h = bench.product_source_hash()
    assert len(h) == 16
    os.makedirs(tmp_path / "profiles")
    (tmp_path / "profiles" / "traffic_w1.md").write_text(
        "# summary\n"
        f"`traffic k_subtree_expand w1 2.5e9 {h}`\n"
        "`traffic k_leaf_reduce w1 1.0e9 0123456789abcdef`\n")
    # the hash covers the sources under ROOT: point ROOT at a copy that also holds them
    csrc = tmp_path / "paper_1805_08998_amd" / "csrc"
    os.makedirs(csrc)
    for f in ("product.hip", "product_kernels.h", "multiply.cpp"):
        with open(os.path.join(ROOT, "paper_1805_08998_amd", "csrc", f), "rb") as src:
            (csrc / f).write_bytes(src.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_subtree_expand", "w1") == 2.5e9
    assert bench.measured_traffic("k_leaf_reduce", "w1") is None  # taken on other sources
    assert bench.measured_traffic("k_term_reduce", "w1") is None  # no line
    assert bench.measured_traffic("k_subtree_expand", "w2") is None  # no file
    (csrc / "multiply.cpp").write_bytes(b"changed")
    assert bench.measured_traffic("k_subtree_expand", "w1") is None  # sources changed since
