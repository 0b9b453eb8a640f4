"""The rank-k error metrics of the accuracy study (Section 6.2, eqs.
def_error, Ak_randUTV, rel_error) computed from T alone, checked on the CPU
against their definitions: e_k = ||A - U(:, 1:k) T(1:k, :) V^T|| formed
densely from the oracle's factors, in the spectral and Frobenius norms, and
the optimal errors against numpy's singular values.  Also the study spectra
(Matrices 1-3) against their stated formulas."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import bench  # noqa: E402
from oracle import randutv_ref as ref  # noqa: E402
from paper_1703_00998_amd import workloads as wl  # noqa: E402


@pytest.mark.parametrize("name,q", [("fast_decay", 0), ("s_shape", 1), ("gap", 2)])
def test_rank_k_errors_match_definition(name, q):
    n, b = 200, 20
    sig = wl.STUDY_SPECTRA[name](n)
    A = wl.planted(n, n, sig, seed=0)
    G = wl.gaussian_g(n, n, b, seed=1)
    U, T, V, _ = ref.randutv(A, b, q, G)
    ks = bench.study_ks(n, b)
    e = bench.rank_k_errors(torch, torch.tensor(T), sig, ks)
    fro = np.array([np.linalg.norm(A - U[:, :k] @ T[:k, :] @ V.T) for k in range(n)])
    spec = np.array([np.linalg.norm(A - U[:, :k] @ T[:k, :] @ V.T, 2) for k in ks])
    nA = np.linalg.norm(A)
    np.testing.assert_allclose(e["fro"], fro, rtol=0, atol=1e-13 * nA)
    np.testing.assert_allclose(e["spec"], spec, rtol=0, atol=1e-13 * nA)
    s = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(e["opt_spec"], s[np.asarray(ks)], rtol=1e-12, atol=0)
    opt_f = np.array([np.sqrt(np.sum(s[k:] ** 2)) for k in range(n)])
    np.testing.assert_allclose(e["opt_fro"], opt_f, rtol=1e-12, atol=0)
    # Eckart-Young: no rank-k approximation beats the truncated SVD.
    assert np.all(e["spec"] >= e["opt_spec"] * (1 - 1e-12))
    assert np.all(e["fro"] >= e["opt_fro"] * (1 - 1e-12))


def test_study_spectra():
    n = 4000
    f = wl.fast_decay_sigma(n)
    assert f[0] == 1.0 and abs(f[-1] - 1e-5) < 1e-18
    assert np.allclose(np.diff(np.log(f)), np.log(1e-5) / (n - 1))
    g = wl.gap_sigma(n)
    assert g[149] == 1 / 150 and abs(g[150] - 0.1 / 151) < 1e-18   # sigma_151 = 0.1 sigma_150 (ratio 150/151)
    s = wl.s_shape_sigma(n)
    assert 0.999 < s[0] <= 1.0 and abs(s[-1] - 1e-2) < 1e-6
    assert np.all(np.diff(s) <= 0) and np.all(np.diff(s[: n // 4]) < 0)
    ks = bench.study_ks(n, 100)
    assert 150 in ks and 151 - 1 in ks and min(ks) > 0 and max(ks) < n


@pytest.mark.parametrize("name", ["fast_decay", "gap"])
def test_spectral_norm_lanczos_path(name):
    """The bidiagonalization path of spectral_norm (blocks above its direct
    limit) against LAPACK's 2-norm, on trailing blocks of a 700 x 700
    randUTV factor."""
    n, b = 700, 50
    sig = wl.STUDY_SPECTRA[name](n)
    A = wl.planted(n, n, sig, seed=0)
    G = wl.gaussian_g(n, n, b, seed=1)
    _, T, _, _ = ref.randutv(A, b, 1, G, form_u=False, form_v=False)
    Tt = torch.tensor(T)
    for k in (0, 100, 149, 150, 151, 300):
        want = np.linalg.norm(T[k:, k:], 2)
        got = bench.spectral_norm(torch, Tt[k:, k:], direct_max=64)
        assert abs(got - want) <= 1e-12 * want, (k, got, want)
