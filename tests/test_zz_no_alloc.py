"""randutv_factor_noalloc (the factorization on the library's own static
device workspace, for callers that cannot allocate) against randutv_factor
on the same inputs: two calls in a row, the second smaller, each compared
elementwise (the same kernels in the same order, so the results agree to
the last bit), with its status through k_out; and the size limit of the
static workspace.  Named to be collected last."""
import ctypes

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


def _inputs(wl, m, n, b, seed):
    sig = np.exp(-np.arange(1, min(m, n) + 1) / (2.0 * b))
    return wl.planted(m, n, sig, seed=seed), wl.gaussian_g(m, n, b, seed=seed + 1)


def _factor_both(B, A, G, b, q):
    m, n = A.shape
    dG = B.colmajor(G)
    T1, T2 = B.colmajor(A), B.colmajor(A)
    U1, U2 = B.empty_colmajor(m, m), B.empty_colmajor(m, m)
    V1, V2 = B.empty_colmajor(n, n), B.empty_colmajor(n, n)
    k1 = B.randutv_factor(T1, dG, b, q, U=U1, V=V1)
    # Through the C ABI directly: no workspace argument.
    L = B.lib()
    k2 = ctypes.c_int64(-1)
    st = L.randutv_factor_noalloc(m, n, b, q, ctypes.c_void_p(T2.data_ptr()), m,
                                  ctypes.c_void_p(dG.data_ptr()), m,
                                  ctypes.c_void_p(U2.data_ptr()), m,
                                  ctypes.c_void_p(V2.data_ptr()), n, 0, 0.0, 0, 3,
                                  ctypes.byref(k2),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    assert k2.value == k1 == min(m, n)
    for a, c in ((T1, T2), (U1, U2), (V1, V2)):
        np.testing.assert_array_equal(a.cpu().numpy(), c.cpu().numpy())
    res = torch.linalg.norm(B.colmajor(A) - U2 @ (T2 @ V2.T)).item() / np.linalg.norm(A)
    assert res < 1e-13


def test_noalloc_matches_factor_twice_second_smaller(B):
    from paper_1703_00998_amd import workloads as wl
    print("noalloc: 1500 x 1200, b = 128, q = 1", flush=True)
    A, G = _inputs(wl, 1500, 1200, 128, 0)
    _factor_both(B, A, G, 128, 1)
    print("noalloc: 300 x 200, b = 32, q = 2", flush=True)
    A, G = _inputs(wl, 300, 200, 32, 4)
    _factor_both(B, A, G, 32, 2)


def test_noalloc_rejects_sizes_beyond_its_workspace(B):
    m = n = 4000
    T = B.empty_colmajor(m, n)
    U, V = B.empty_colmajor(m, m), B.empty_colmajor(n, n)
    G = B.empty_colmajor(m, 3840)
    with pytest.raises(B.RandUTVError, match="-901"):
        B.randutv_factor_noalloc(T, G, 256, 1, U=U, V=V)
