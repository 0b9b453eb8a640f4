"""The economy U (RANDUTV_ECON_U: U's first min(m, n) columns, m x min(m, n))
against the FP64 oracle's full U through the C ABI: tall inputs with ragged
last blocks, an early stop (U(:, 0:k) is the left factor of the rank-k
approximation, Section 1.1 advantage (ii)), over-sampling, and the
20000 x 5000 early-stop workload with U and V formed in O(mnk) storage."""
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


@pytest.mark.parametrize("m,n,b,q,k_stop,p", [(600, 300, 32, 1, 0, 0), (777, 500, 64, 2, 0, 0),
                                                (1000, 400, 64, 1, 128, 0), (500, 300, 32, 1, 0, 8)])
def test_econ_u_matches_oracle(B, m, n, b, q, k_stop, p):
    print(f"econ U m={m} n={n} b={b} q={q} k_stop={k_stop} p={p}", flush=True)
    sig = np.exp(-np.arange(1, n + 1) / (2.0 * b))
    A = wl.planted(m, n, sig, seed=0)
    G = wl.gaussian_g(m, n, b, seed=1, p=p)
    Uo, To, Vo, ko = ref.randutv(A, b, q, G, p=p, k_stop=k_stop)
    T = B.colmajor(A)
    U = B.empty_colmajor(m, n)
    V = B.empty_colmajor(n, n)
    k = B.randutv_factor(T, B.colmajor(G), b, q, U=U, V=V, k_stop=k_stop, p=p)
    assert k == ko
    nA = np.linalg.norm(A)
    tol = 1e-9 if p == 0 else 1e-7
    np.testing.assert_allclose(_np(U), Uo[:, :n], rtol=0, atol=tol)
    np.testing.assert_allclose(_np(V), Vo, rtol=0, atol=tol)
    np.testing.assert_allclose(_np(T), To, rtol=0, atol=tol * nA)
    Ug = U.double()
    assert torch.linalg.norm(Ug.T @ Ug - torch.eye(n, dtype=torch.float64, device="cuda")).item() \
        <= 1e-13 * math.sqrt(m) * 10
    Ad = torch.as_tensor(A, device="cuda")
    if k == n:  # A = U T(0:n, :) V^T
        res = torch.linalg.norm(Ad - U @ (T[:n] @ V.T)).item() / nA
        assert res <= 1e-13
    else:  # the rank-k approximation U_k T(0:k, :) V^T
        Ak = U[:, :k] @ (T[:k] @ V.T)
        Ak_o = Uo[:, :k] @ To[:k] @ Vo.T
        np.testing.assert_allclose(_np(Ak), Ak_o, rtol=0, atol=1e-10 * nA)


def test_econ_u_early_stop_20000x5000_workload(B):
    """20000 x 5000 (rank 300 + noise 1e-8 ||A||), b = 128, q = 2,
    tol = 1e-6, with U (20000 x 5000, economy) and V formed: k = 384, and
    ||A - U_k T(0:k, :) V^T||_F / ||A||_F is the noise left behind."""
    A, _ = wl.config_matrix("c4_20000x5000")
    m, n, b, q = 20000, 5000, 128, 2
    dA = B.colmajor(A)
    nA = float(np.linalg.norm(A))
    del A
    G = B.colmajor(wl.gaussian_g(m, n, b, seed=1))
    T = dA.clone().T.contiguous().T
    U = B.empty_colmajor(m, n)
    V = B.empty_colmajor(n, n)
    k = B.randutv_factor(T, G, b, q, U=U, V=V, tol=1e-6)
    assert k == 384
    Uk = U[:, :k]
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    assert torch.linalg.norm(Uk.T @ Uk - eye).item() <= 1e-12
    err = torch.linalg.norm(dA - Uk @ (T[:k] @ V.T)).item() / nA
    tail = torch.linalg.norm(T[k:, k:]).item() / nA
    print(f"econ U 20000x5000: k={k}, ||A - A_k|| / ||A|| = {err:.3e} (trailing {tail:.3e})",
          flush=True)
    assert abs(err - tail) <= 1e-3 * tail  # A - A_k = U(:, k:) T(k:, k:) V(:, k:)^T
    assert 0.9e-8 <= err <= 1.0e-8
