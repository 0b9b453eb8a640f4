"""GPU unit tests of the building blocks behind the C ABI: the MFMA thin GEMM,
the cooperative Householder panel QR with its compact-WY factor, and the
batched small SVD.  References are independent (numpy / LAPACK via scipy,
run on the host)."""
import numpy as np
import pytest
import scipy.linalg

torch = pytest.importorskip("torch")

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


GEMM_SHAPES = [(64, 64, 16), (100, 70, 130), (257, 33, 1500), (8, 300, 7), (1, 1, 1),
               (130, 256, 4100), (33, 17, 0),
               (2100, 200, 1100), (3000, 256, 700), (240, 2300, 1200),  # thin-output tiles
               (128, 128, 128), (128, 128, 512), (16, 128, 37), (127, 3, 513)]  # small-product path edges


@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_fp64_matches_numpy(B, M, N, K, ta, tb):
    """Thin product C = alpha op(A) op(B) + beta C (Section 5.4's BLAS-3 work):
    FP64 MFMA result within a few ulps * K of the FP64 numpy product,
    including ragged tiles and split-K."""
    print(f"gemm fp64 M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    Bm = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = 0.75 * ((A.T if ta else A) @ (Bm.T if tb else Bm)) - 0.5 * C0
    dA, dB, dC = B.colmajor(A), B.colmajor(Bm), B.colmajor(C0)
    ws = B.workspace(8 * M * N * 8)
    B.randutv_gemm(dC, dA, dB, ta=ta, tb=tb, alpha=0.75, beta=-0.5, work=ws)
    torch.cuda.synchronize()
    got = _np(dC)
    scale = np.sqrt(max(K, 1)) * 1e-15 * 10
    np.testing.assert_allclose(got, ref, rtol=0, atol=scale * (np.abs(ref).max() + 1))


SPLIT_TOL = {"fp32": 2 ** -24, "bf16x3": 2 ** -16, "bf16x6": 2 ** -24}


@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_gemm_split_precision_error_bound(B, M, N, K, ta, tb, prec):
    """Split-precision products (FP64 in and out): each entry's error is
    bounded by a few units of the arithmetic's rounding times |a_i||b_j|
    (FP32: operand rounding 2^-24 plus FP32 accumulation; BF16x3: the dropped
    lo*lo term and the BF16 representation error, 2^-16 together; BF16x6:
    three pieces carry x32's 24 bits, and the dropped m*l, l*m, l*l terms are
    below 2^-23), plus the accumulation's sqrt(K) growth.  A lane-layout or
    piece mistake gives errors of order |a_i||b_j| (or 2^-8, 2^-16 of it)
    and fails."""
    print(f"gemm {prec} M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 5 + N * 11 + K + {"fp32": 7, "bf16x3": 13, "bf16x6": 17}[prec])
    A = rng.standard_normal((K, M) if ta else (M, K))
    Bm = rng.standard_normal((N, K) if tb else (K, N))
    A *= np.exp(rng.uniform(-3, 3, size=A.shape))  # spread of magnitudes
    C0 = rng.standard_normal((M, N))
    Aop = A.T if ta else A
    Bop = Bm.T if tb else Bm
    ref = 0.75 * (Aop @ Bop) - 0.5 * C0
    dA, dB, dC = B.colmajor(A), B.colmajor(Bm), B.colmajor(C0)
    ws = B.workspace(8 * M * N * 8)
    B.randutv_gemm(dC, dA, dB, ta=ta, tb=tb, alpha=0.75, beta=-0.5, prec=prec, work=ws)
    torch.cuda.synchronize()
    got = _np(dC)
    scale = np.outer(np.linalg.norm(Aop, axis=1), np.linalg.norm(Bop, axis=0))
    tol = 0.75 * scale * (4 * SPLIT_TOL[prec] + 8 * 2 ** -24 * np.sqrt(max(K, 1)))
    err = np.abs(got - ref)
    assert np.all(err <= tol + 1e-14 * (np.abs(ref) + 1)), float((err / (tol + 1e-300)).max())
    if prec == "bf16x3" and K >= 16:
        # much better than one BF16 product: the error must sit well below 2^-9
        assert float((err / (0.75 * scale + 1e-300)).max()) < 2 ** -12
    if prec == "bf16x6" and K >= 16:
        # FP32-like: below the BF16x3 split's 2^-16 (a dropped m*m or h*l term fails)
        assert float((err / (0.75 * scale + 1e-300)).max()) < 2 ** -17


def _larft(V, tau):
    """Host reference compact-WY factor by the column recurrence
    T(0:j,j) = -tau_j T(0:j,0:j) V(:,0:j)^T v_j, T(j,j) = tau_j."""
    nb = tau.size
    T = np.zeros((nb, nb))
    for j in range(nb):
        T[:j, j] = -tau[j] * (T[:j, :j] @ (V[:, :j].T @ V[:, j]))
        T[j, j] = tau[j]
    return T


@pytest.mark.parametrize("Mp,nb", [(40, 7), (300, 32), (1000, 64), (257, 256), (5000, 256),
                                   (8000, 256), (129, 128), (20000, 128), (64, 64), (17, 1)])
def test_panel_qr_matches_lapack(B, Mp, nb):
    """Unpivoted Householder QR (Section 2.4 eq. unpivQR) against LAPACK dgeqrf
    (same dlarfg convention): R, tau and reflector tails; the compact-WY factor
    against the host recurrence, and I - V Tw V^T against dorgqr's Q."""
    print(f"panel Mp={Mp} nb={nb}", flush=True)
    rng = np.random.default_rng(Mp + nb)
    A = rng.standard_normal((Mp, nb))
    if nb >= 8:
        A[:, 3] *= 1e-6  # graded columns
    qr, tau_ref, _, info = scipy.linalg.lapack.dgeqrf(np.asfortranarray(A))
    assert info == 0
    dP = B.colmajor(A)
    dtau = torch.zeros(nb, dtype=torch.float64, device="cuda")
    dTw = B.colmajor(np.full((nb, nb), np.nan))
    fallback = B.randutv_panel_qr(dP, dtau, dTw)
    torch.cuda.synchronize()
    # kappa <= ~1e6 here: the CholeskyQR2 + reconstruction path must take it
    assert not fallback
    P, tau, Tw = _np(dP), _np(dtau), _np(dTw)
    nA = np.linalg.norm(A)
    np.testing.assert_allclose(np.triu(P[:nb]), np.triu(qr[:nb]), rtol=0, atol=1e-13 * nA)
    np.testing.assert_allclose(tau, tau_ref, rtol=0, atol=1e-13)
    V = np.tril(P, -1)[:, :nb] + np.eye(Mp, nb)
    Vref = np.tril(qr, -1)[:, :nb] + np.eye(Mp, nb)
    np.testing.assert_allclose(V, Vref, rtol=0, atol=1e-11)
    assert np.all(np.tril(Tw, -1) == 0.0)
    Tref = _larft(V, tau)
    np.testing.assert_allclose(Tw, Tref, rtol=0, atol=1e-12 * (np.abs(Tref).max() + 1))
    Q = np.eye(Mp, nb) - V @ (Tw @ V[:nb, :].T)
    Qref = scipy.linalg.lapack.dorgqr(qr, tau_ref)[0][:, :nb]
    np.testing.assert_allclose(Q, Qref, rtol=0, atol=1e-12)


def test_panel_qr_zero_and_rank_deficient(B):
    """tau = 0 when the part below the diagonal is zero (dlarfg), also with a
    negative diagonal entry; exact-zero columns give identity reflectors."""
    Mp, nb = 300, 16
    A = np.zeros((Mp, nb))
    A[0, 0] = -2.0
    rng = np.random.default_rng(1)
    A[:, 5] = rng.standard_normal(Mp)
    A[:, 9] = rng.standard_normal(Mp)
    qr, tau_ref, _, _ = scipy.linalg.lapack.dgeqrf(np.asfortranarray(A))
    dP = B.colmajor(A)
    dtau = torch.zeros(nb, dtype=torch.float64, device="cuda")
    dTw = B.colmajor(np.zeros((nb, nb)))
    assert B.randutv_panel_qr(dP, dtau, dTw)  # rank deficient: column-by-column path
    torch.cuda.synchronize()
    tau = _np(dtau)
    assert tau[0] == 0.0 and _np(dP)[0, 0] == -2.0
    np.testing.assert_allclose(tau, tau_ref, atol=1e-14)
    assert np.all(np.isfinite(_np(dP))) and np.all(np.isfinite(_np(dTw)))


def _stack(mats, ld):
    out = np.zeros((len(mats), ld, ld))
    for i, M in enumerate(mats):
        n = M.shape[0]
        out[i, :n, :n] = M.T  # [i] holds the column-major storage (transpose)
    return torch.as_tensor(out, device="cuda")


def test_small_svd_matches_numpy(B):
    """The small SVD of Figure randUTV: singular values against LAPACK,
    Us diag(D) Vs^T = R, orthogonality, canonical signs."""
    rng = np.random.default_rng(4)
    sizes = [1, 2, 5, 32, 33, 64, 128, 256]
    mats = [np.triu(rng.standard_normal((n, n))) for n in sizes]
    mats[3] = mats[3] * np.exp(-np.arange(32) / 4.0)  # graded columns
    ld = 256
    R = _stack(mats, ld)
    Us, D, Vs, st = B.randutv_small_svd(R, sizes)
    torch.cuda.synchronize()
    assert st == 0
    for i, (n, M) in enumerate(zip(sizes, mats)):
        u = _np(Us[i]).T[:n, :n]
        v = _np(Vs[i]).T[:n, :n]
        d = _np(D[i])[:n]
        s = np.linalg.svd(M, compute_uv=False)
        np.testing.assert_allclose(d, s, rtol=1e-13 * n, atol=1e-15 * s[0])
        np.testing.assert_allclose(u @ np.diag(d) @ v.T, M, atol=1e-13 * s[0] * np.sqrt(n))
        assert np.linalg.norm(u.T @ u - np.eye(n)) < 1e-13 * n
        assert np.linalg.norm(v.T @ v - np.eye(n)) < 1e-13 * n
        for j in range(n):
            assert v[np.argmax(np.abs(v[:, j])), j] > 0


def test_small_svd_zero_and_rank_deficient(B):
    """Zero singular values: Us is completed to an orthogonal matrix."""
    n = 24
    rng = np.random.default_rng(9)
    Z = np.zeros((n, n))
    L = rng.standard_normal((n, 3)) @ rng.standard_normal((3, n))
    R = _stack([Z, np.triu(L)], n)
    Us, D, Vs, st = B.randutv_small_svd(R, [n, n])
    torch.cuda.synchronize()
    assert st == 0
    for i, M in enumerate([Z, np.triu(L)]):
        u = _np(Us[i]).T
        v = _np(Vs[i]).T
        d = _np(D[i])
        assert np.linalg.norm(u.T @ u - np.eye(n)) < 1e-12
        assert np.linalg.norm(v.T @ v - np.eye(n)) < 1e-12
        np.testing.assert_allclose(u @ np.diag(d) @ v.T, M, atol=1e-12 * (np.abs(M).max() + 1))


def _panel_quality(B, P0):
    Mp, nb = P0.shape
    dP = B.colmajor(P0)
    dtau = torch.zeros(nb, dtype=torch.float64, device="cuda")
    dTw = B.colmajor(np.zeros((nb, nb)))
    fallback = B.randutv_panel_qr(dP, dtau, dTw)
    torch.cuda.synchronize()
    P, T = _np(dP), _np(dTw)
    V = np.tril(P, -1)[:, :nb] + np.eye(Mp, nb)
    R = np.triu(P[:nb])
    X = np.random.default_rng(0).standard_normal((Mp, 8))
    HX = X - V @ (T @ (V.T @ X))
    orth = np.abs(HX.T @ HX - X.T @ X).max() / np.abs(X.T @ X).max()
    Q = np.eye(Mp, nb) - V @ (T @ V[:nb].T)
    res = np.linalg.norm(P0 - Q @ R) / np.linalg.norm(P0)
    return orth, res, fallback


@pytest.mark.parametrize("case", ["sampling_c2", "zero_col", "tiny_block", "graded", "near_dup",
                                  "sampling_c3", "gaussian", "scaled_1e150"])
def test_panel_qr_backward_stable_on_hard_panels(B, case):
    """Householder QR is backward stable whatever the conditioning (Section 2.4
    eq. unpivQR): on graded / rank-deficient / nearly dependent panels the
    compact-WY product I - V Tw V^T must stay orthogonal to ~eps and
    reproduce the panel, including a sampling matrix (X^T X) X^T G of the
    4000 x 4000, sigma_j = j^-1.5 workload (condition ~1e10)."""
    from paper_1703_00998_amd import workloads as wl
    rng = np.random.default_rng(1)
    if case == "sampling_c2":
        A, _ = wl.config_matrix("c2_4000")
        G = wl.gaussian_g(4000, 4000, 128, seed=1)
        P0 = A.T @ (A @ (A.T @ G[:, :128]))
    elif case == "sampling_c3":
        # sampling matrix of a 3000 x 3000, sigma_j = exp(-j/800) matrix (the
        # 8000 x 8000 workload's decay), b = 256, q = 1: well conditioned
        sig = np.exp(-np.arange(1, 3001) / 800.0) + 1e-10
        A = wl.planted(3000, 3000, sig, seed=0)
        G = wl.gaussian_g(3000, 3000, 256, seed=1)
        P0 = A.T @ (A @ (A.T @ G[:, :256]))
    elif case == "gaussian":
        P0 = rng.standard_normal((5000, 200))
    elif case == "scaled_1e150":
        P0 = 1e150 * rng.standard_normal((2000, 64))
    else:
        P0 = rng.standard_normal((3000, 128))
        if case == "zero_col":
            P0[:, 20] = 0.0
        elif case == "tiny_block":
            P0[:, 16:32] *= 1e-9
        elif case == "graded":
            P0 *= np.exp(-np.arange(128) / 4.0)
        else:
            P0[:, 40] = 3 * P0[:, 39] + 1e-12 * rng.standard_normal(3000)
    orth, res, fallback = _panel_quality(B, P0)
    print(f"panel {case}: orth {orth:.2e} res {res:.2e} fallback {fallback}", flush=True)
    assert orth < 1e-14 and res < 1e-14, (orth, res)
    # kappa > ~3e6 must go column by column; well-conditioned panels must not
    assert fallback == (case not in ("sampling_c3", "gaussian", "scaled_1e150"))


@pytest.mark.parametrize("case", ["graded_8000x256", "near_dup_200_3000x256"])
def test_panel_qr_nb256_fallback_matches_dgeqrf(B, case):
    """Panels 256 wide are two 128-column blocks on the reconstruction path;
    an ill-conditioned one goes to the column-by-column kernel on all 256
    columns, whether the first block already flags (graded columns, kappa ~
    1e14) or only the second (a near-duplicate column at index 200).  The
    result is LAPACK's dgeqrf factorization (Section 2.4, eq. unpivQR):
    R, tau and the reflectors agree elementwise wherever they are well
    determined (all columns for the graded panel, whose QR only rescales
    R's columns; the 200 columns before the near-duplicate one), and the
    compact-WY product stays orthogonal and reproduces the panel."""
    rng = np.random.default_rng(2)
    if case == "graded_8000x256":
        P0 = rng.standard_normal((8000, 256)) * np.exp(-np.arange(256) / 8.0)
        ncmp = 256
    else:
        P0 = rng.standard_normal((3000, 256))
        P0[:, 200] = 3 * P0[:, 199] + 1e-12 * rng.standard_normal(3000)
        ncmp = 200
    Mp, nb = P0.shape
    dP = B.colmajor(P0)
    dtau = torch.zeros(nb, dtype=torch.float64, device="cuda")
    dTw = B.colmajor(np.zeros((nb, nb)))
    fallback = B.randutv_panel_qr(dP, dtau, dTw)
    torch.cuda.synchronize()
    assert fallback
    qr, tau_ref, _, info = scipy.linalg.lapack.dgeqrf(np.asfortranarray(P0))
    assert info == 0
    P, tau, T = _np(dP), _np(dtau), _np(dTw)
    R, Rr = np.triu(P[:nb]), np.triu(qr[:nb])
    V, Vr = np.tril(P, -1)[:, :nb], np.tril(qr, -1)[:, :nb]
    scale = np.abs(Rr).max(axis=0)  # column scale of R
    np.testing.assert_allclose(R[:, :ncmp] / scale[:ncmp], Rr[:, :ncmp] / scale[:ncmp],
                               rtol=0, atol=1e-12)
    np.testing.assert_allclose(tau[:ncmp], tau_ref[:ncmp], rtol=0, atol=1e-12)
    np.testing.assert_allclose(V[:, :ncmp], Vr[:, :ncmp], rtol=0, atol=1e-11)
    Vf = V + np.eye(Mp, nb)
    X = rng.standard_normal((Mp, 8))
    HX = X - Vf @ (T @ (Vf.T @ X))
    assert np.abs(HX.T @ HX - X.T @ X).max() / np.abs(X.T @ X).max() < 1e-14
    Q = np.eye(Mp, nb) - Vf @ (T @ Vf[:nb].T)
    assert np.linalg.norm(P0 - Q @ R) / np.linalg.norm(P0) < 1e-14
