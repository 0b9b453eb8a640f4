"""GPU parity of the rank-k accuracy study (Section 6.2): the errors
e_k = ||A - A_k|| of the library's factor against those of the oracle's on
Matrices 1-3 with q = 0, 1, 2, and at the study's full size (4000 x 4000,
b = 100) the properties that hold for any correct factorization:
Eckart-Young (no rank-k error below the optimal one), the first block's
diagonal below the singular values, and Ky Fan's bound on the leading
diagonal entries."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import bench  # noqa: E402
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


def _gpu_T(B, A, G, b, q):
    T = B.colmajor(A)
    B.randutv_factor(T, B.colmajor(G), b, q)
    torch.cuda.synchronize()
    return T


@pytest.mark.parametrize("q", [0, 1, 2])
@pytest.mark.parametrize("name", list(wl.STUDY_SPECTRA))
def test_study_errors_match_oracle(B, name, q):
    """400 x 400, b = 40.  Tolerance on each e_k: 100 times the Frobenius
    change of the oracle's T under a seeded 1e-15 relative perturbation of A
    (both factorizations are backward stable; any e_k moves by at most the
    Frobenius norm of T's change), never below 1e-10 ||A||_F."""
    n, b = 400, 40
    print(f"study parity {name} q={q}", flush=True)
    sig = wl.STUDY_SPECTRA[name](n)
    A = wl.planted(n, n, sig, seed=0)
    G = wl.gaussian_g(n, n, b, seed=1)
    _, To, _, _ = ref.randutv(A, b, q, G, form_u=False, form_v=False)
    E = np.random.default_rng(12345).standard_normal(A.shape)
    E *= 1e-15 * np.linalg.norm(A) / np.linalg.norm(E)
    _, Tp, _, _ = ref.randutv(A + E, b, q, G, form_u=False, form_v=False)
    nA = np.linalg.norm(A)
    tol = max(1e-10 * nA, 100 * np.linalg.norm(To - Tp))
    ks = bench.study_ks(n, b)
    eo = bench.rank_k_errors(torch, torch.tensor(To), sig, ks)
    eg = bench.rank_k_errors(torch, _gpu_T(B, A, G, b, q), sig, ks)
    np.testing.assert_allclose(eg["fro"], eo["fro"], rtol=0, atol=tol)
    np.testing.assert_allclose(eg["spec"], eo["spec"], rtol=0, atol=tol)
    assert np.all(eg["spec"] >= eg["opt_spec"] * (1 - 1e-12))
    assert np.all(eg["fro"] >= eg["opt_fro"] * (1 - 1e-12))


def test_study_full_size_bounds(B):
    """Matrix 3 (gap) at 4000 x 4000, b = 100, q = 1: the bounds that hold at
    any size, on the Frobenius errors at every rank and the spectral errors
    around the gap."""
    n, b, q = 4000, 100, 1
    sig = wl.gap_sigma(n)
    A = wl.planted(n, n, sig, seed=0)
    G = wl.gaussian_g(n, n, b, seed=1)
    T = _gpu_T(B, A, G, b, q)
    ks = [150, 151]
    e = bench.rank_k_errors(torch, T, sig, ks,
                            norm2=lambda th, M: th.linalg.matrix_norm(M, ord=2).item())
    assert np.all(e["fro"] >= e["opt_fro"] * (1 - 1e-12))
    assert np.all(e["spec"] >= e["opt_spec"] * (1 - 1e-12))
    # The study's bidiagonalization estimate agrees with the dense SVD.
    for k, want in zip(ks, e["spec"]):
        assert abs(bench.spectral_norm(torch, T[k:, k:]) - want) <= 1e-6 * want
    d = torch.diagonal(T).cpu().numpy()
    assert np.all(d[:b] <= sig[:b] * (1 + 1e-12))                    # first block
    assert np.all(np.cumsum(d ** 2) <= np.cumsum(sig ** 2) * (1 + 1e-12))  # Ky Fan
    assert abs(e["fro"][0] - np.linalg.norm(A)) <= 1e-12 * np.linalg.norm(A)
