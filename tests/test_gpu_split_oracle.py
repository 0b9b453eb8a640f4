"""End-to-end tests of the split-precision paths against the FP64 oracle
(Figure "The algorithm randUTV"), at sizes where the thin products run on
the 128 x 128 GEMM tiles and with split-K (the launch classes of the
8000 x 8000 workload's first steps), and on a mid-size matrix through the
whole factorization.

The reference is always the oracle.  The tolerance is taken from the
oracle's own response to a seeded relative perturbation A o (1 + delta E)
at the split arithmetic's rounding level (delta = 2^-24 for FP32 and BF16x6
products, 2^-16 for BF16x3 sampling or products), times a margin of
10 sqrt(n / 2): a product's rounding acts on each step like such a
perturbation, amplified by the accumulation over K = n terms (about
sqrt(K / 2) relatively, for FP32 accumulation).  A wrong tile, transpose or
piece of the split gives errors of the order of the values themselves and
fails."""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import randutv_ref as ref  # noqa: E402
from paper_1703_00998_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "split_4096_b256.json")
# Rounding level each path's products carry: the coarser of its sampling and
# update arithmetic.
LEVEL = {"fp64": None, "fp32": "fp32", "bf16x3": "bf16", "bf16x3_fp32": "bf16",
         "bf16x3_bf16x6": "bf16"}
# 128 x 128 classes each path must launch at 4096 x 4096, b = 256.
T128 = {"fp64": ["gemm_tn_fp64_t128", "gemm_nn_fp64_t128", "gemm_nt_fp64_t128"],
        "fp32": ["gemm_tn_fp32_t128", "gemm_nn_fp32_t128", "gemm_nt_fp32_t128"],
        "bf16x3": ["gemm_tn_bf16x3_t128", "gemm_nn_bf16x3_t128", "gemm_nt_bf16x3_t128"],
        "bf16x3_fp32": ["gemm_tn_bf16x3_t128", "gemm_nn_bf16x3_t128", "gemm_nt_fp32_t128",
                        "gemm_nn_fp32_t128", "gemm_tn_fp32_t128"],
        "bf16x3_bf16x6": ["gemm_tn_bf16x3_t128", "gemm_nn_bf16x3_t128", "gemm_nt_bf16x6_t128",
                          "gemm_nn_bf16x6_t128", "gemm_tn_bf16x6_t128"]}

def margin(n):
    return 10.0 * math.sqrt(n / 2.0)


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_00998_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    A = wl.planted(4096, 4096, np.exp(-np.arange(1, 4097) / 512.0), seed=0)
    G = wl.gaussian_g(4096, 4096, 256, seed=1)
    # the regenerated input is the one the stored values were computed from
    assert abs(np.linalg.norm(A) / g["A_fro"] - 1) < 1e-12
    assert abs(A[0, 0] - g["A_00"]) <= 1e-14 and abs(A[-1, -1] - g["A_last"]) <= 1e-14
    return g, A, G


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x3_fp32", "bf16x3_bf16x6"])
def test_split_paths_4096_on_128_tiles_match_oracle(B, golden, prec):
    """4096 x 4096, sigma_j = exp(-j/512), b = 256, q = 1, three steps:
    diag(T)(0:768) and ||T(k:, k:)||_F at k = 256, 512, 768 against the
    oracle's, with the path's 128 x 128 kernel classes checked to have run."""
    g, A, G = golden
    print(f"split oracle 4096 {prec}", flush=True)
    T = B.colmajor(A)
    dG = B.colmajor(G)
    B.profile_begin()
    k = B.randutv_factor(T, dG, 256, 1, k_stop=768, prec=prec)
    torch.cuda.synchronize()
    prof = B.profile_end()
    assert k == 768
    ran = {c for c, v in prof.items() if v[3] > 0}
    missing = [c for c in T128[prec] if c not in ran]
    assert not missing, (missing, sorted(ran))
    d = torch.diagonal(T)[:768].cpu().numpy()
    tails = np.array([torch.linalg.norm(T[kk:, kk:]).item() for kk in (256, 512, 768)])
    d0, t0 = np.array(g["diag"]), np.array(g["tails"])
    if LEVEL[prec] is None:  # the FP64 path: the FP32 response scaled to FP64 rounding
        pert = g["perturbed_fp32"]
        scale = 2.0 ** -52 / pert["delta"]
    else:
        pert = g[f"perturbed_{LEVEL[prec]}"]
        scale = 1.0
    rd = np.abs(np.array(pert["diag"]) - d0).max() * scale
    rt = np.abs(np.array(pert["tails"]) - t0).max() * scale
    nA = g["A_fro"]
    tol_d = margin(4096) * rd + 1e-13 * nA
    tol_t = margin(4096) * rt + 1e-13 * nA
    ed, et = np.abs(d - d0).max(), np.abs(tails - t0).max()
    print(f"{prec}: |d - d_oracle| {ed:.2e} (tol {tol_d:.2e}), "
          f"|tail - tail_oracle| {et:.2e} (tol {tol_t:.2e})", flush=True)
    assert ed <= tol_d and et <= tol_t
    # the three diagonal blocks are each exactly diagonal and descending
    Th = T[:768, :768].cpu().numpy()
    assert np.all(np.tril(Th, -1) == 0.0)
    for s0 in (0, 256, 512):
        blk = Th[s0:s0 + 256, s0:s0 + 256]
        assert np.all(blk - np.diag(np.diag(blk)) == 0.0)
        assert np.all(np.diff(np.diag(blk)) <= 0.0)


@pytest.fixture(scope="module")
def mid():
    """1024 x 768, sigma_j = exp(-j/200), b = 64, q = 1: the oracle's
    factorization and its response to perturbations at both levels."""
    m, n, b, q = 1024, 768, 64, 1
    A = wl.planted(m, n, np.exp(-np.arange(1, n + 1) / 200.0), seed=0)
    G = wl.gaussian_g(m, n, b, seed=1)
    _, T0, _, _ = ref.randutv(A, b, q, G, form_u=False, form_v=False)
    E = np.random.default_rng(7).standard_normal(A.shape)
    resp = {}
    for name, delta in (("fp32", 2.0 ** -24), ("bf16", 2.0 ** -16)):
        _, Tp, _, _ = ref.randutv(A * (1.0 + delta * E), b, q, G, form_u=False, form_v=False)
        resp[name] = np.abs(np.diag(Tp) - np.diag(T0)).max()
    return A, G, T0, resp


@pytest.mark.parametrize("prec,bound", [("fp32", 1e-6), ("bf16x3_fp32", 1e-6),
                                        ("bf16x3_bf16x6", 1e-6), ("bf16x3", 3e-5)])
def test_split_paths_whole_factorization_match_oracle(B, mid, prec, bound):
    """The whole 1024 x 768 factorization (every step, the final block and
    the small SVDs): diag(T) against the oracle's within the margin times
    the oracle's response at the path's rounding level; the residual within
    the path's bound (BF16x3 updates carry about 2^-17 relative error, so
    they cannot reach 1e-6); U, V orthogonal to FP64 rounding (built in FP64
    from FP64 reflectors); T exactly upper triangular with diagonal blocks."""
    A, G, T0, resp = mid
    m, n = A.shape
    b, q = 64, 1
    print(f"split whole factorization {prec}", flush=True)
    T = B.colmajor(A)
    U, V = B.empty_colmajor(m, m), B.empty_colmajor(n, n)
    k = B.randutv_factor(T, B.colmajor(G), b, q, U=U, V=V, prec=prec)
    assert k == n
    Ad = torch.as_tensor(A, device="cuda")
    res = (torch.linalg.norm(Ad - U @ (T @ V.T)) / torch.linalg.norm(Ad)).item()
    eye = lambda k: torch.eye(k, dtype=torch.float64, device="cuda")  # noqa: E731
    ou = torch.linalg.norm(U.T @ U - eye(m)).item()
    ov = torch.linalg.norm(V.T @ V - eye(n)).item()
    Th = T.cpu().numpy()
    ed = np.abs(np.diag(Th) - np.diag(T0)).max()
    tol = margin(m) * resp[LEVEL[prec]] + 1e-13 * np.linalg.norm(A)
    print(f"{prec}: residual {res:.2e}, |d - d_oracle| {ed:.2e} (tol {tol:.2e})", flush=True)
    assert res <= bound
    assert ou <= 1e-12 * math.sqrt(m) and ov <= 1e-12 * math.sqrt(n)
    assert ed <= tol
    assert np.all(np.tril(Th, -1) == 0.0)
    for s0 in range(0, n, b):
        blk = Th[s0:s0 + b, s0:s0 + b]
        assert np.all(blk - np.diag(np.diag(blk)) == 0.0)
