"""GPU parity of the lower-triangular variant (randutv_factor_lower: A =
U L V^T, Section 1 lets the middle factor be upper or lower triangular;
computed as randUTV of A^T) against the oracle's randutv_lower through the
C ABI: U, L, V elementwise on tall, wide and square shapes with ragged
tails, an early stop, a split-precision path, and the invariants at
3000 x 2000."""
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


def _run(B, A, G, b, q, **kw):
    m, n = A.shape
    T = B.colmajor(A)
    U = B.empty_colmajor(m, m)
    V = B.empty_colmajor(n, n)
    k = B.randutv_factor_lower(T, B.colmajor(G), b, q, U=U, V=V, **kw)
    torch.cuda.synchronize()
    return U, T, V, k


@pytest.mark.parametrize("shape,b,q", [((300, 200), 32, 1), ((200, 300), 32, 1),
                                       ((257, 257), 64, 2), ((130, 500), 16, 0)])
def test_lower_matches_oracle(B, shape, b, q):
    m, n = shape
    print(f"lower m={m} n={n} b={b} q={q}", flush=True)
    sig = np.exp(-np.arange(1, min(m, n) + 1) / max(2.0 * b, 4.0))
    A = wl.planted(m, n, sig, seed=0)
    G = wl.gaussian_g(n, m, b, seed=1)
    Uo, Lo, Vo, ko = ref.randutv_lower(A, b, q, G)
    U, L, V, k = _run(B, A, G, b, q)
    assert k == ko == min(m, n)
    nA = np.linalg.norm(A)
    np.testing.assert_allclose(_np(L), Lo, rtol=0, atol=1e-10 * nA)
    np.testing.assert_allclose(_np(U), Uo, rtol=0, atol=1e-9)
    np.testing.assert_allclose(_np(V), Vo, rtol=0, atol=1e-9)
    assert np.all(np.triu(_np(L), 1) == 0.0)


def test_lower_early_stop(B):
    m, n, b, q = 400, 300, 32, 1
    sig = np.exp(-np.arange(1, n + 1) / 40.0)
    A = wl.planted(m, n, sig, seed=0)
    G = wl.gaussian_g(n, m, b, seed=1)
    Uo, Lo, Vo, ko = ref.randutv_lower(A, b, q, G, k_stop=2 * b)
    U, L, V, k = _run(B, A, G, b, q, k_stop=2 * b)
    assert k == ko == 2 * b
    np.testing.assert_allclose(_np(L)[:k, :k], Lo[:k, :k], rtol=0, atol=1e-10 * np.linalg.norm(A))
    Ad = torch.as_tensor(A, device="cuda")
    assert (torch.linalg.norm(Ad - U @ (L @ V.T)) / torch.linalg.norm(Ad)).item() <= 1e-13


@pytest.mark.parametrize("prec,bound", [("fp64", 1e-13), ("bf16x3_fp32", 1e-6)])
def test_lower_invariants_3000x2000(B, prec, bound):
    m, n, b, q = 3000, 2000, 128, 1
    sig = np.exp(-np.arange(1, n + 1) / 300.0)
    A = wl.planted(m, n, sig, seed=0)
    G = wl.gaussian_g(n, m, b, seed=1)
    U, L, V, k = _run(B, A, G, b, q, prec=prec)
    assert k == n
    Ad = torch.as_tensor(A, device="cuda")
    assert (torch.linalg.norm(Ad - U @ (L @ V.T)) / torch.linalg.norm(Ad)).item() <= bound
    eye_m = torch.eye(m, dtype=torch.float64, device="cuda")
    assert torch.linalg.norm(U.T @ U - eye_m).item() <= 1e-12 * math.sqrt(m)
    assert torch.linalg.norm(V.T @ V - eye_m[:n, :n]).item() <= 1e-12 * math.sqrt(n)
    Lh = _np(L)
    assert np.all(np.triu(Lh, 1) == 0.0)
    d = np.diag(Lh)
    assert np.all(np.cumsum(d ** 2) <= np.cumsum(sig ** 2) * (1 + 1e-9))
