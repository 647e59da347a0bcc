"""The roofline bookkeeping of bench.py, without a GPU.

* The HBM traffic the headline's roofline object carries comes from the committed counter
  summary: FETCH_SIZE and WRITE_SIZE averages per dispatch, each scaled by what the same counter
  reads for a plain device copy of known size.  The stored bytes per launch must be that
  product, and bench.py must drop it (null) as soon as the tile-QR source differs from the one
  the counters were taken on.
* The roofline object itself: the kind with the largest device time, its algorithmic flops over
  its summed duration, priced at the MFMA peak of its precision (FP32 for FP32-bulk leaf tiles,
  applications and component GEMMs; FP64 otherwise and for every kind of an FP64 workload) or,
  for the Jacobi SVDs, at the FP64 vector peak ("alu").
"""
import hashlib
import importlib
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    try:
        return importlib.import_module("bench")
    finally:
        sys.path.remove(ROOT)


@pytest.mark.parametrize("kernel,workload", [("qr_factor_leaf", "graded_sum_r200"), ("qr_apply", "batched_uneven_256")])
def test_recorded_traffic_is_the_calibrated_counter_sum(bench, kernel, workload):
    text = open(os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")).read()
    fetch_kib, write_kib = map(float, re.search(r"FETCH_SIZE ([\d.]+) KiB,? .*?WRITE_SIZE ([\d.]+) KiB", text).groups())
    sf, sw = map(float, re.search(r"FETCH_SIZE (?:is )?scaled by (\d+\.\d+),? (?:and )?WRITE_SIZE by (\d+\.\d+)",
                                  text).groups())
    stored = int(re.search(r"traffic_bytes_per_launch: (\d+)", text).group(1))
    # the averages are printed to 0.1 KiB and the scale factors to 1e-4: the product agrees to
    # that rounding
    slack = 0.05 * (sf + sw) + 0.00005 * (fetch_kib + write_kib)
    assert abs(1024 * (fetch_kib * sf + write_kib * sw) - stored) <= 1024 * slack + 1
    src = open(os.path.join(ROOT, "paper_2211_08770_amd", "csrc", "qr.hip"), "rb").read()
    current = hashlib.sha256(src).hexdigest()[:16] in text
    assert bench.recorded_traffic(kernel, workload) == (stored if current else None)


def test_no_traffic_without_a_summary(bench):
    assert bench.recorded_traffic("qr_apply") is None            # no summary for that kind on the headline


def test_recorded_traffic_is_dropped_when_the_qr_source_changes(bench, tmp_path, monkeypatch):
    root = tmp_path / "repo"
    (root / "profiles").mkdir(parents=True)
    (root / "paper_2211_08770_amd" / "csrc").mkdir(parents=True)
    src = open(os.path.join(ROOT, "paper_2211_08770_amd", "csrc", "qr.hip"), "rb").read()
    summary = open(os.path.join(ROOT, "profiles", "qr_factor_leaf_graded_sum_r200_traffic.txt")).read()
    (root / "profiles" / "qr_factor_leaf_graded_sum_r200_traffic.txt").write_text(summary)
    monkeypatch.setattr(bench, "ROOT", str(root))
    (root / "paper_2211_08770_amd" / "csrc" / "qr.hip").write_bytes(src)
    same = bench.recorded_traffic("qr_factor_leaf")
    (root / "paper_2211_08770_amd" / "csrc" / "qr.hip").write_bytes(src + b"\n// changed\n")
    assert bench.recorded_traffic("qr_factor_leaf") is None
    # with the source the summary names, the value is read back
    if hashlib.sha256(src).hexdigest()[:16] in summary:
        assert same == int(re.search(r"traffic_bytes_per_launch: (\d+)", summary).group(1))


def test_roofline_object_prices_each_kind(bench):
    def prof(dominant, ms=2.0, flops=4e9):
        p = {k: {"ms": 0.1, "flops": 1e6, "bytes": 0.0, "launches": 1} for k in bench.KINDS}
        p[dominant] = {"ms": ms, "flops": flops, "bytes": 0.0, "launches": 4}
        return p

    r = bench.roofline_of(prof("qr_factor_leaf"))
    assert r["kernel"] == "qr_factor_leaf" and r["bound"] == "mfma" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(4e9 / 2e-3 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3, rel=1e-3)
    assert r["avg_launch_ms"] == pytest.approx(0.5)
    assert bench.roofline_of(prof("qr_factor_leaf"), bulk_fp32=False)["peak"] == 78.6
    assert bench.roofline_of(prof("qr_factor_node"))["peak"] == 78.6      # tree nodes are FP64
    assert bench.roofline_of(prof("tt_dot"))["peak"] == 78.6              # FP64 MFMA for either dtype
    assert bench.roofline_of(prof("contraction_gemm"))["peak"] == 157.3
    s = bench.roofline_of(prof("svd_jacobi"))
    assert s["bound"] == "alu" and s["peak"] == 78.6
    total = 2.0 + 0.1 * (len(bench.KINDS) - 1)
    assert s["share_of_kernel_time"] == pytest.approx(2.0 / total, rel=1e-3)
