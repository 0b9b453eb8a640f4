"""GPU parity of the over-sampled factorization (randutv_factor_p; the Remark on
over-sampling in Section 5.3 and the over-sampled step of Appendix A.2)
against the FP64 oracle with the same p, through the C ABI.

Each randomized step draws b + p samples and takes the Householder QR of the
b dominant left singular vectors of the extended sample.  The cases cover
several tiles and ragged tails, the last randomized step with fewer than
b + p columns left (the zero-padded SVD), b + p above one 128-column HR block
and at its 256 limit, a wide input, an early stop, the split-precision
paths, and a rank-deficient input (invariants only: the singular vectors of
a zero singular value are not unique).

Tolerance.  Keeping the b dominant of b + p singular vectors makes each step
as sensitive as the gap between the b-th and (b+1)-th singular values of its
sample, and later steps inherit earlier steps' perturbations through the
trailing matrix, so the factors can move far more than rounding under a
rounding-sized change of A (500 x 400, b = 48, p = 16: V moves by 4e-10
under a 1e-15 relative perturbation, against 4e-13 with p = 0).  Both
sides are backward stable, so their difference is about the condition times
their rounding.  Each test measures that condition on the oracle alone (its
response to a seeded random perturbation of relative size 1e-15) and allows
100 times the response (the GPU path's rounding is blocked and reordered,
up to a few times 1e-15), with the p = 0 tests' bounds as the floor."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import randutv_ref as ref  # noqa: E402
from paper_1703_00998_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_00998_amd import binding
    binding.lib()
    return binding


def _np(t):
    return t.detach().cpu().numpy()


def _factor(B, A, b, q, p, G, prec="fp64", **kw):
    m, n = A.shape
    T = B.colmajor(A)
    U = B.empty_colmajor(m, m)
    V = B.empty_colmajor(n, n)
    k = B.randutv_factor(T, B.colmajor(G), b, q, U=U, V=V, prec=prec, p=p, **kw)
    torch.cuda.synchronize()
    return U, T, V, k


def _residual(A, U, T, V):
    Ad = torch.as_tensor(A, device="cuda")
    return (torch.linalg.norm(Ad - U @ (T @ V.T)) / torch.linalg.norm(Ad)).item()


def _orth(Q):
    n = Q.shape[1]
    return torch.linalg.norm(Q.T @ Q - torch.eye(n, dtype=Q.dtype, device=Q.device)).item()


def _sensitivity(A, b, q, G, p, **kw):
    """Oracle-only condition estimate: max |change| of U and V, and of T
    relative to ||A||_F, when A moves by a seeded random perturbation of
    Frobenius norm 1e-15 ||A||_F."""
    rng = np.random.default_rng(12345)
    E = rng.standard_normal(A.shape)
    E *= 1e-15 * np.linalg.norm(A) / np.linalg.norm(E)
    U1, T1, V1, _ = ref.randutv(A, b, q, G, p=p, **kw)
    U2, T2, V2, _ = ref.randutv(A + E, b, q, G, p=p, **kw)
    nA = np.linalg.norm(A)
    return (U1, T1, V1), (np.abs(U1 - U2).max(), np.abs(V1 - V2).max(),
                          np.abs(T1 - T2).max() / nA)


def _tols(sens):
    dU, dV, dT = sens
    return max(1e-9, 100 * dU), max(1e-9, 100 * dV), max(1e-10, 100 * dT)


def _case(m, n, b, p):
    sig = np.exp(-np.arange(1, min(m, n) + 1) / max(2.0 * b, 4.0))
    A = wl.planted(m, n, sig, seed=0)
    G = wl.gaussian_g(m, n, b, seed=1, p=p)
    return A, G


# (m, n, b, p, q).  300 x 260, b = 32, p = 8: the last randomized step has
# 36 < 40 columns (padded SVD); 500 x 400, b = 48, p = 16: exactly 64 = b + p;
# 600 x 600, b = 128, p = 20: b + p = 148 spans two HR blocks; 700 x 600,
# b = 200, p = 56: b + p = 256.
CASES = [(300, 260, 32, 8, 1), (500, 400, 48, 16, 1), (257, 257, 32, 10, 2),
         (600, 600, 128, 20, 1), (700, 600, 200, 56, 1), (400, 300, 16, 1, 0),
         (200, 500, 32, 8, 1)]


@pytest.mark.parametrize("m,n,b,p,q", CASES)
def test_oversampled_matches_oracle(B, m, n, b, p, q):
    """T, U, V elementwise against the oracle (same sign rules on the
    extended sample's singular vectors and on the Householder reflectors),
    and the UTV invariants."""
    print(f"oversampled factor m={m} n={n} b={b} p={p} q={q}", flush=True)
    A, G = _case(m, n, b, p)
    assert G.shape[1] == B.g_cols(m, n, b, p)
    (Uo, To, Vo), sens = _sensitivity(A, b, q, G, p)
    tu, tv, tt = _tols(sens)
    print(f"tolerances U {tu:.1e} V {tv:.1e} T/||A|| {tt:.1e}", flush=True)
    U, T, V, k = _factor(B, A, b, q, p, G)
    assert k == min(m, n)
    nA = np.linalg.norm(A)
    np.testing.assert_allclose(_np(T), To, rtol=0, atol=tt * nA)
    np.testing.assert_allclose(_np(U), Uo, rtol=0, atol=tu)
    np.testing.assert_allclose(_np(V), Vo, rtol=0, atol=tv)
    assert _residual(A, U, T, V) <= 1e-13
    assert _orth(U) <= 1e-12 * math.sqrt(m) and _orth(V) <= 1e-12 * math.sqrt(n)
    assert np.all(np.tril(_np(T), -1) == 0.0)


def test_oversampled_early_stop(B):
    """k_stop = 2b with p = 12: the reduced part agrees with the oracle
    stopped the same way."""
    m, n, b, p, q = 400, 350, 32, 12, 1
    A, G = _case(m, n, b, p)
    (Uo, To, Vo), sens = _sensitivity(A, b, q, G, p, k_stop=2 * b)
    tu, _, tt = _tols(sens)
    U, T, V, k = _factor(B, A, b, q, p, G, k_stop=2 * b)
    assert k == 2 * b
    np.testing.assert_allclose(_np(T)[:k, :k], To[:k, :k], rtol=0,
                               atol=tt * np.linalg.norm(A))
    np.testing.assert_allclose(_np(U)[:, :k], Uo[:, :k], rtol=0, atol=tu)
    assert _residual(A, U, T, V) <= 1e-13


@pytest.mark.parametrize("prec,bound", [("fp32", 1e-6), ("bf16x3_fp32", 1e-6)])
def test_oversampled_split_paths(B, prec, bound):
    """1024 x 768, b = 64, p = 10 on the split-precision paths: residual
    within the path's bound, U and V orthogonal to FP64 rounding, T upper
    triangular with diagonal blocks."""
    m, n, b, p, q = 1024, 768, 64, 10, 1
    sig = np.exp(-np.arange(1, n + 1) / 200.0)
    A = wl.planted(m, n, sig, seed=0)
    G = wl.gaussian_g(m, n, b, seed=1, p=p)
    print(f"oversampled split path {prec}", flush=True)
    U, T, V, k = _factor(B, A, b, q, p, G, prec=prec)
    assert k == n
    assert _residual(A, U, T, V) <= bound
    assert _orth(U) <= 1e-12 * math.sqrt(m) and _orth(V) <= 1e-12 * math.sqrt(n)
    Th = _np(T)
    assert np.all(np.tril(Th, -1) == 0.0)
    for s0 in range(0, n, b):
        blk = Th[s0:s0 + b, s0:s0 + b]
        assert np.all(blk - np.diag(np.diag(blk)) == 0.0)


def test_oversampled_rank_deficient_invariants(B):
    """Rank 20 < b = 32 with p = 8: the sample has rank 20, so the b dominant
    left singular vectors are not unique; check what holds for any choice:
    A = U T V^T, U and V orthogonal, T upper triangular, and the first
    diagonal block holding the 20 singular values of A."""
    m, n, b, p, q = 300, 256, 32, 8, 1
    sig = np.linspace(1.0, 0.5, 20)
    A = wl.planted(m, n, sig, seed=0)
    G = wl.gaussian_g(m, n, b, seed=1, p=p)
    U, T, V, k = _factor(B, A, b, q, p, G)
    assert k == n
    assert _residual(A, U, T, V) <= 1e-13
    assert _orth(U) <= 1e-12 * math.sqrt(m) and _orth(V) <= 1e-12 * math.sqrt(n)
    Th = _np(T)
    assert np.all(np.tril(Th, -1) == 0.0)
    np.testing.assert_allclose(np.diag(Th)[:20], sig, rtol=0, atol=1e-12)
    assert np.linalg.norm(Th[20:, 20:]) <= 1e-12
