"""GPU tests of the thin GEMM on its 128 x 128 tiles, in every arithmetic and
transpose case, including the exact launch shapes of the 8000 x 8000, b = 256
factorization's first step (sampling Y = X^T G and Z = X Y with split-K,
the right update W = T Vh and T -= W2 Vh^T, the left update C = Uh^T T and
T -= Uh C2; Section 5.4's "applications of A to thin matrices").  The
library's own kernel timing names the instantiation that ran, so each case
first asserts that the 128 x 128 kernel (not the 64 x 64 one) was used.
References are numpy FP64 products; the full-size cases compare sampled
rows (spread over every row tile, the ragged last one included) against
those rows computed on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_00998_amd import binding
    binding.lib()
    return binding


# Per-entry bound of a split-precision product (as in test_gpu_kernels):
# |err_ij| <= alpha ||a_i|| ||b_j|| (4 u_split + 8 * 2^-24 sqrt(K)).
U_SPLIT = {"fp64": 0.0, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16, "bf16x6": 2.0 ** -24}


def _run(B, prec, ta, tb, M, N, K, alpha, beta, seed, rows=None):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((K, M) if ta else (M, K))
    Bm = rng.standard_normal((N, K) if tb else (K, N))
    if prec != "fp64":
        A *= np.exp(rng.uniform(-2, 2, size=A.shape))
    C0 = rng.standard_normal((M, N))
    dA, dB, dC = B.colmajor(A), B.colmajor(Bm), B.colmajor(C0)
    ws = B.workspace(8 * M * N * 8)
    torch.cuda.synchronize()
    B.profile_begin()
    B.randutv_gemm(dC, dA, dB, ta=ta, tb=tb, alpha=alpha, beta=beta, prec=prec, work=ws)
    torch.cuda.synchronize()
    prof = B.profile_end()
    op = ("t" if ta else "n") + ("t" if tb else "n")
    cls = f"gemm_{op}_{prec}_t128"
    assert prof.get(cls, (0, 0, 0, 0))[3] == 1, {k: v[3] for k, v in prof.items() if v[3]}
    Aop = A.T if ta else A
    Bop = Bm.T if tb else Bm
    if rows is None:
        rows = np.arange(M)
    got = dC[torch.as_tensor(rows, device=dC.device)].cpu().numpy()
    ref = alpha * (Aop[rows] @ Bop) + beta * C0[rows]
    err = np.abs(got - ref)
    if prec == "fp64":
        tol = np.sqrt(K) * 1e-14 * (np.abs(ref).max() + 1)
        assert err.max() <= tol, (err.max(), tol)
    else:
        scale = np.outer(np.linalg.norm(Aop[rows], axis=1), np.linalg.norm(Bop, axis=0))
        tol = abs(alpha) * scale * (4 * U_SPLIT[prec] + 8 * 2.0 ** -24 * np.sqrt(K))
        assert np.all(err <= tol + 1e-14 * (np.abs(ref) + 1)), float((err / (tol + 1e-300)).max())
        if prec == "bf16x3":  # far better than one BF16 product (2^-9)
            assert float((err / (abs(alpha) * scale + 1e-300)).max()) < 2.0 ** -12
        if prec == "bf16x6":  # below the BF16x3 split's 2^-16 (catches a dropped m*m, h*l)
            assert float((err / (abs(alpha) * scale + 1e-300)).max()) < 2.0 ** -17
    return prof[cls]


# Shapes large enough for 128 x 128 tiles: 2560 x 2560 outputs (400 tiles),
# and a thin 3072 x 256 output with K = 4096 split over blockIdx.z.
MEDIUM = [(2560, 2560, 256), (3072, 256, 4096), (2600, 2500, 300)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("M,N,K", MEDIUM)
def test_t128_tiles_all_cases(B, M, N, K, ta, tb, prec):
    print(f"t128 {prec} M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    _run(B, prec, ta, tb, M, N, K, 0.75, -0.5, M * 3 + N * 7 + K + 2 * ta + tb)


# The first step of the 8000 x 8000, b = 256 factorization (m_i = n_i = 8000,
# n_i - b = 7744), with the alpha / beta the driver passes.
HEADLINE = [
    (True, False, 8000, 256, 8000, 1.0, 0.0),    # Y = X^T G (and Y = X^T Z)
    (False, False, 8000, 256, 8000, 1.0, 0.0),   # Z = X Y, and W = T(:, J) Vh
    (False, True, 8000, 8000, 256, -1.0, 1.0),   # T(:, J) -= W2 Vh^T
    (True, False, 256, 7744, 8000, 1.0, 0.0),    # C = Uh^T T(I, J3)
    (False, False, 8000, 7744, 256, -1.0, 1.0),  # T(I, J3) -= Uh C2
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("ta,tb,M,N,K,alpha,beta", HEADLINE)
def test_t128_headline_launch_shapes(B, ta, tb, M, N, K, alpha, beta, prec):
    print(f"t128 headline {prec} M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(11)
    tiles = np.arange(0, M, 128)
    rows = np.unique(np.concatenate([tiles + rng.integers(0, 128, tiles.size), [M - 1]]))
    rows = rows[rows < M]
    _run(B, prec, ta, tb, M, N, K, alpha, beta, 5 + M + N + K, rows=rows)
