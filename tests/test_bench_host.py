"""Host-side logic of bench.py (no GPU): the flop count against the oracle's
formulas, the choice of the dominant kernel class, and the lookup of the
committed HBM-traffic record (class, workload, kernel-source digest and
launch shape must all match)."""
import json
import os

import pytest

import bench
from oracle import randutv_ref as ref

WORKLOAD = "randUTV 8000x8000, b=256, q=1, U and V formed, sigma_j=exp(-j/800)+1e-10"


def test_flops_total_matches_the_paper_formula_plus_uv():
    for m, n, q in [(8000, 8000, 1), (8000, 8000, 2), (20000, 5000, 2), (500, 500, 1)]:
        assert bench.flops_total(m, n, q) == pytest.approx(ref.flops_paper(m, n, q) +
                                                           ref.flops_uv(m, n), rel=1e-15)
        assert bench.flops_total(m, n, q, form_uv=False) == pytest.approx(
            ref.flops_paper(m, n, q), rel=1e-15)


def test_dominant_class_rule():
    prof = {
        "gemm_nn_fp64_t64": (90.0, 1e12, 1e9, 100),   # also inside the panels: excluded
        "gemm_tn_fp64_t64": (80.0, 1e12, 1e9, 100),   # likewise
        "panel_qr": (70.0, 1e10, 1e9, 63),            # not a GEMM class
        "gemm_nt_fp64_t64": (30.0, 1e12, 1e9, 287),
        "gemm_nn_fp32_t128": (15.0, 1e12, 1e9, 46),
        "gemm_tn_bf16x3_t128": (40.0, 1e12, 1e9, 0),  # no launches: excluded
    }
    assert bench.dominant_class(prof) == "gemm_nt_fp64_t64"


def _committed_record():
    d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")
    for f in sorted(os.listdir(d)):
        if f.endswith(".md"):
            for line in open(os.path.join(d, f)):
                if line.startswith("traffic-record: "):
                    return json.loads(line[len("traffic-record: "):])
    return None


def test_traffic_record_lookup():
    rec = _committed_record()
    assert rec is not None
    alg = rec["algorithmic_bytes_per_launch"]
    if rec["kernel_sources_sha256"] == bench.kernel_sources_sha256():
        got = bench.traffic_record(rec["class"], rec["workload"], alg)
        assert got is not None and got["traffic_bytes_per_launch"] == rec["traffic_bytes_per_launch"]
        assert bench.traffic_record(rec["class"], rec["workload"], alg * 1.01) is not None
    # Another launch shape, class or workload never matches.
    assert bench.traffic_record(rec["class"], rec["workload"], alg * 1.5) is None
    assert bench.traffic_record("gemm_nn_fp32_t128", rec["workload"], alg) is None
    assert bench.traffic_record(rec["class"], rec["workload"] + " (other)", alg) is None
    assert rec["workload"] == WORKLOAD
