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
    """The top-time k_gemm class, no class excluded (the panels' own products
    are timed inside panel_qr); composite classes never qualify."""
    prof = {
        "panel_qr": (170.0, 1e10, 1e9, 63),           # not a GEMM class
        "small_svd": (120.0, 0.0, 0.0, 1),            # not a GEMM class
        "splitk_reduce": (100.0, 1e9, 1e9, 40),       # not a GEMM class
        "gemm_nn_fp64_t64_uv": (90.0, 1e12, 1e9, 100),
        "gemm_nt_fp64_t64": (30.0, 1e12, 1e9, 287),
        "gemm_nn_fp32_t128": (15.0, 1e12, 1e9, 46),
        "gemm_tn_bf16x3_t128": (400.0, 1e12, 1e9, 0),  # no launches: excluded
        "gemm_nn_bf16x3_t128": (4.0, 1e12, 1e9, 18),
    }
    assert bench.dominant_class(prof) == "gemm_nn_fp64_t64_uv"
    assert bench.dominant_class(prof, "bf16x3") == "gemm_nn_bf16x3_t128"
    assert bench.dominant_class(prof, "fp32") == "gemm_nn_fp32_t128"


def test_roofline_record_arithmetic():
    """achieved = algorithmic flops / event time; BF16x3 classes are priced as
    three BF16 MFMA products per flop against the BF16 peak."""
    prof = {"gemm_nt_fp64_t128": (10.0, 5e11, 2e9, 100),
            "gemm_tn_bf16x3_t128": (2.0, 1e12, 4e9, 10)}
    r = bench.roofline_of("gemm_nt_fp64_t128", prof, WORKLOAD)
    assert r["achieved"] == pytest.approx(50.0)
    assert r["frac"] == pytest.approx(50.0 / 78.6)
    assert r["avg_launch_us"] == pytest.approx(100.0)
    assert r["kernel"] == "k_gemm<PREC_FP64, false, true, 128, 128, 2, 4, 0>"
    assert bench.kernel_symbol("gemm_nt_fp64_t64_uv") == \
        "k_gemm<PREC_FP64, false, true, 64, 64, 2, 2, 2>"
    # BF16 classes of a split path name the pre-split instantiations they run.
    assert bench.kernel_symbol("gemm_nn_bf16x6_t128", "bf16x3_bf16x6") == (
        "k_gemm<PREC_BF16X6, false, false, 128, 128, 2, 2, 8> | "
        "k_gemm<PREC_BF16X6, false, false, 128, 128, 2, 2, 12>")
    assert bench.kernel_symbol("gemm_tn_bf16x3_t128", "bf16x3_bf16x6") == \
        "k_gemm<PREC_BF16X3, true, false, 128, 128, 2, 2, 8>"
    assert bench.kernel_symbol("gemm_tn_bf16x3_t128", "bf16x3") == (
        "k_gemm<PREC_BF16X3, true, false, 128, 128, 2, 2, 4> | "
        "k_gemm<PREC_BF16X3, true, false, 128, 128, 2, 2, 8>")
    prof["gemm_nt_fp64_t128@alone"] = (5.0, 5e11, 2e9, 100)
    r = bench.roofline_of("gemm_nt_fp64_t128", prof, WORKLOAD)
    assert r["achieved_alone"] == pytest.approx(100.0)
    assert r["frac_alone"] == pytest.approx(100.0 / 78.6)
    assert r["avg_launch_us_alone"] == pytest.approx(50.0)
    r = bench.roofline_of("gemm_tn_bf16x3_t128", prof, WORKLOAD)
    assert r["achieved"] == pytest.approx(500.0)
    assert r["frac"] == pytest.approx(1500.0 / 2500.0)
    assert r["algorithmic_gb_per_s"] == pytest.approx(2000.0)


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
