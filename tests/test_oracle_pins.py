"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own code.

Each test names the passage of the paper (section / equation / figure) whose
consequence it checks.  Library routines (LAPACK via numpy/scipy) are only run
here as independent references.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import randutv_ref as ref
from paper_1703_00998_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(np.float64).eps


def _factor(A, b, q, seed_g=1, **kw):
    m, n = A.shape
    G = wl.gaussian_g(m, n, b, seed=seed_g)
    return G, ref.randutv(A, b, q, G, **kw)


def _check_utv(A, U, T, V, k, b, tol=1e-13):
    m, n = A.shape
    nA = np.linalg.norm(A)
    assert np.linalg.norm(A - U @ T @ V.T) / nA <= tol
    assert np.linalg.norm(U.T @ U - np.eye(m)) <= tol * math.sqrt(m) * 10
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= tol * math.sqrt(n) * 10
    # Exact zeros below the diagonal in the first k columns, and off the
    # diagonal inside each diagonal block (Figure randUTV: T(I3,J2) = 0 and
    # T(I2,J2) = D_small).
    for j in range(k):
        assert np.all(T[j + 1:, j] == 0.0)
        blk = (j // b) * b
        assert np.all(T[blk:j, j] == 0.0)
    d = np.diag(T)[:k]
    assert np.all(d >= 0.0)
    for s0 in range(0, k, b):
        blkd = d[s0:min(s0 + b, k)]
        assert np.all(np.diff(blkd) <= 0.0)
    # ||T||_F = ||A||_F (orthogonal invariance).
    assert abs(np.linalg.norm(T) - nA) <= 1e-13 * nA


# ---------------------------------------------------------------- Householder
def test_house_qr_matches_lapack_dgeqrf():
    """Section 2.4 eq. unpivQR: unpivoted Householder QR.  LAPACK dgeqrf uses
    the dlarfg sign convention; the oracle's reflectors, tau and R must agree."""
    rng = np.random.default_rng(5)
    for (p, c) in [(40, 7), (33, 33), (9, 4), (64, 16)]:
        B = rng.standard_normal((p, c))
        refl, R = ref.house_qr(B)
        qr, tau, _, info = scipy.linalg.lapack.dgeqrf(np.asfortranarray(B))
        assert info == 0
        k = min(p, c)
        np.testing.assert_allclose(R, np.triu(qr[:k, :]), rtol=0, atol=1e-13 * np.abs(B).max() * p)
        for j, (v, t) in enumerate(refl):
            assert abs(t - tau[j]) <= 1e-14 * 4
            np.testing.assert_allclose(v[1:], qr[j + 1:, j], rtol=0, atol=1e-13)
            assert v[0] == 1.0


def test_householder_special_cases():
    """dlarfg convention corners: x2 = 0 gives tau = 0 and beta = alpha, also for
    alpha < 0; alpha = 0 with x2 != 0 takes sign(0) = +1 (beta < 0)."""
    v, tau, beta = ref.householder(np.array([-3.0, 0.0, 0.0]))
    assert tau == 0.0 and beta == -3.0 and np.array_equal(v, [1.0, 0.0, 0.0])
    v, tau, beta = ref.householder(np.array([0.0, 3.0, 4.0]))
    assert beta == -5.0 and abs(tau - 1.0) < 1e-15
    x = np.array([2.0, -1.0, 2.0])
    v, tau, beta = ref.householder(x)
    Hx = x - tau * v * (v @ x)
    np.testing.assert_allclose(Hx, [beta, 0, 0], atol=1e-15)
    assert beta == -3.0
    # single entry: nothing below the diagonal, identity reflector
    v, tau, beta = ref.householder(np.array([-2.0]))
    assert tau == 0.0 and beta == -2.0


def test_reflector_products_match_lapack_full_q():
    """The complement matters for later steps (Section 5.2: V and U are
    products of b Householder reflectors).  apply_right(I, refl) must equal
    LAPACK's full orthogonal factor (dgeqrf + dorgqr) of the same matrix, and
    apply_left must apply its transpose."""
    rng = np.random.default_rng(6)
    Y = rng.standard_normal((30, 8))
    refl, _ = ref.house_qr(Y)
    Qfull, _ = scipy.linalg.qr(Y, mode="full")
    Qo = ref.apply_right(np.eye(30), refl)
    np.testing.assert_allclose(Qo, Qfull, atol=1e-14 * 30)
    C = rng.standard_normal((30, 11))
    np.testing.assert_allclose(ref.apply_left(C.copy(), refl), Qfull.T @ C, atol=1e-13)


def test_small_svd_canonical_signs_and_order():
    """Section 2.2 eq. defSVD: sigma descending, >= 0; canonical signs: the
    largest-magnitude entry of each v_j is positive."""
    rng = np.random.default_rng(7)
    R = np.triu(rng.standard_normal((12, 12)))
    Us, D, Vs = ref.small_svd(R)
    np.testing.assert_allclose(Us @ np.diag(D) @ Vs.T, R, atol=1e-13)
    assert np.all(np.diff(D) <= 0) and np.all(D >= 0)
    for j in range(12):
        assert Vs[np.argmax(np.abs(Vs[:, j])), j] > 0


# ------------------------------------------------------------- whole method
def _jacobi_singular_values(A, sweeps=40):
    """Brute-force one-sided (Hestenes) Jacobi: singular values of A, written
    independently of numpy's SVD, for tiny matrices."""
    W = np.array(A, dtype=np.float64, copy=True)
    n = W.shape[1]
    for _ in range(sweeps):
        off = 0.0
        for p in range(n - 1):
            for qq in range(p + 1, n):
                a = W[:, p] @ W[:, p]
                bb = W[:, qq] @ W[:, qq]
                g = W[:, p] @ W[:, qq]
                if g == 0.0:
                    continue
                off = max(off, abs(g) / math.sqrt(a * bb))
                zeta = (bb - a) / (2.0 * g)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = c * t
                wp = W[:, p].copy()
                W[:, p] = c * wp - s * W[:, qq]
                W[:, qq] = s * wp + c * W[:, qq]
        if off < 1e-15:
            break
    return np.sort(np.linalg.norm(W, axis=0))[::-1]


def test_planted_graded_spectrum_diag_matches_jacobi():
    """Section 4.1 objective (i) and Theorem: with a large gap between blocks
    of singular values and q = 1, each diagonal block of T reproduces the
    planted sigma to ~eps*||A|| (the subspace error is (gap)^(2q+1) ~ 1e-14).
    Checked against an independent brute-force Jacobi SVD of A."""
    n, b = 24, 8
    rng = np.random.default_rng(11)
    sig = np.concatenate([np.sort(1 + rng.random(8))[::-1],
                          1e-5 * np.sort(1 + rng.random(8))[::-1],
                          1e-10 * np.sort(1 + rng.random(8))[::-1]])
    A = wl.planted(n, n, sig, seed=3)
    sj = _jacobi_singular_values(A)
    np.testing.assert_allclose(sj, sig, rtol=0, atol=50 * EPS * sig[0])
    G, (U, T, V, k) = _factor(A, b, 1)
    _check_utv(A, U, T, V, k, b)
    d = np.diag(T)
    assert np.all(np.abs(d - sj) <= 100 * EPS * sig[0] + 1e-9 * sj)


def test_q_matters_on_graded_spectrum():
    """The power iteration is really applied: with q = 0 the first block is
    only accurate to (gap)^1-ish, far worse than with q = 1."""
    n, b = 24, 8
    sig = np.concatenate([np.linspace(2, 1, 8), np.linspace(2e-2, 1e-2, 8),
                          np.linspace(2e-4, 1e-4, 8)])
    A = wl.planted(n, n, sig, seed=4)
    _, (_, T0, _, _) = _factor(A, b, 0)
    _, (_, T1, _, _) = _factor(A, b, 1)
    _, (_, T2, _, _) = _factor(A, b, 2)
    e0 = np.max(np.abs(np.diag(T0)[:8] - sig[:8]))
    e1 = np.max(np.abs(np.diag(T1)[:8] - sig[:8]))
    e2 = np.max(np.abs(np.diag(T2)[:8] - sig[:8]))
    assert e1 < e0 * 1e-2 and e2 < e1 * 1e-2


def test_b_ge_n_is_exact_svd():
    """Figure randUTV: with b >= n there is one step and it is the final SVD
    branch, so diag(T) are the singular values (tall input: economic QR+SVD,
    Remark on the economic SVD)."""
    rng = np.random.default_rng(12)
    for (m, n) in [(20, 20), (35, 12), (12, 35)]:
        A = rng.standard_normal((m, n))
        G = np.zeros((m, 0))
        U, T, V, k = ref.randutv(A, 32, 1, G)
        s = np.linalg.svd(A, compute_uv=False)
        np.testing.assert_allclose(np.diag(T), s, rtol=1e-14 * 10, atol=1e-15)
        _check_utv(A, U, T, V, k, 32)
        assert k == min(m, n)
        assert np.all(T[n:, :] == 0.0)
        assert np.all(T[:, m:] == 0.0)  # wide input: [diag(sigma), 0] (Remark on m < n)


def test_rank_le_b_captured_in_first_block():
    """rank(A) <= b: the range finder captures the whole range (Section 2.5),
    so T11 = diag(sigma) and the rest of T is ~eps*||A||."""
    m, n, b = 60, 40, 8
    sig = np.array([5.0, 3.0, 2.0, 1.5, 1.0, 0.5])
    A = wl.planted(m, n, sig, seed=9)
    G, (U, T, V, k) = _factor(A, b, 1)
    np.testing.assert_allclose(np.diag(T)[:6], sig, rtol=1e-13)
    assert np.linalg.norm(T[:, 6:]) <= 1e-13 * 5


def test_theorem_step_one_identities():
    """Theorem (Section 5.3), eq. approx1 and approx2, after ONE step:
    ||[T12;T22]||_F = ||A - A Q Q^T||_F with Q = orth((A^T A)^q A^T G_1), and
    ||T22||_F = ||A - W W^T A||_F with W = orth(A Y); also diag(T11) = sigma(A Q).
    Q, W and sigma(AQ) come from numpy's QR / SVD of independently formed
    sampling matrices."""
    m, n, b, q = 50, 40, 8, 1
    A = wl.planted(m, n, np.exp(-np.arange(1, 41) / 6.0), seed=2)
    G = wl.gaussian_g(m, n, b, seed=1)
    U, T, V, k = ref.randutv(A, b, q, G, k_stop=b)
    assert k == b
    G1 = G[:, :b]
    Y = A.T @ G1
    for _ in range(q):
        Y = A.T @ (A @ Y)
    Q, _ = np.linalg.qr(Y)
    W, _ = np.linalg.qr(A @ Y)
    e1 = np.linalg.norm(A - A @ Q @ Q.T)
    e2 = np.linalg.norm(A - W @ (W.T @ A))
    assert abs(np.linalg.norm(T[:, b:]) - e1) <= 1e-12 * e1 + 1e-14
    assert abs(np.linalg.norm(T[b:, b:]) - e2) <= 1e-12 * e2 + 1e-14
    np.testing.assert_allclose(np.diag(T)[:b], np.linalg.svd(A @ Q, compute_uv=False), rtol=1e-13)
    # Partial factorization is still exact: A = U T V^T.
    assert np.linalg.norm(A - U @ T @ V.T) <= 1e-13 * np.linalg.norm(A)


def _dense_lapack_randutv(A, b, q, G, p=0):
    """Independent dense re-implementation of the blocked method with LAPACK
    primitives and explicit m x m / n x n orthogonal factors (the O(n^4)
    style of Figure randUTVmatlab, with the economic left transform of the
    Remark on tall SVDs so that complements are Householder ones, and the
    LQ of the Remark on the case m < n for a wide last block)."""
    m, n = A.shape
    T = A.copy()
    U = np.eye(m)
    V = np.eye(n)
    s = min(-(-m // b), -(-n // b))
    for i in range(s):
        r0 = i * b
        X = T[r0:, r0:]
        Mi, Ni = X.shape
        if r0 + b < m and r0 + b < n:
            Gi = G[:Mi, i * (b + p):(i + 1) * (b + p)]
            Y = X.T @ Gi
            for _ in range(q):
                Y = X.T @ (X @ Y)
            if p > 0:  # dominant b left singular vectors (signs as for the small SVDs)
                Zy, _, Wyt = scipy.linalg.svd(Y, full_matrices=False, lapack_driver="gesvd")
                for j in range(b):
                    if Wyt[j, np.argmax(np.abs(Wyt[j, :]))] < 0:
                        Zy[:, j] *= -1
                Y = Zy[:, :b]
            Vq, _ = scipy.linalg.qr(Y, mode="full")
            XV = X @ Vq
            Uq, R = scipy.linalg.qr(XV[:, :b], mode="full")
            Us, D, Vst = np.linalg.svd(R[:b, :b])
            Vs = Vst.T
            for j in range(b):
                if Vs[np.argmax(np.abs(Vs[:, j])), j] < 0:
                    Vs[:, j] *= -1
                    Us[:, j] *= -1
            UU = Uq.copy()
            UU[:, :b] = Uq[:, :b] @ Us
            VV = Vq.copy()
            VV[:, :b] = Vq[:, :b] @ Vs
        elif Mi < Ni:
            # Wide last block: LQ of the rows via LAPACK's QR of X^T, then the
            # SVD of the Mi x Mi lower-triangular factor (signs normalised on
            # that SVD's right singular vectors).
            Qt, Rt = scipy.linalg.qr(X.T, mode="full")
            Us, D, Vlt = np.linalg.svd(Rt[:Mi, :Mi].T)
            Vl = Vlt.T
            for j in range(D.size):
                if Vl[np.argmax(np.abs(Vl[:, j])), j] < 0:
                    Vl[:, j] *= -1
                    Us[:, j] *= -1
            VV = Qt.copy()
            VV[:, :Mi] = Qt[:, :Mi] @ Vl
            UU = Us
        else:
            Uf, D, Vft = np.linalg.svd(X, full_matrices=True)
            Vs = Vft.T
            for j in range(D.size):
                if Vs[np.argmax(np.abs(Vs[:, j])), j] < 0:
                    Vs[:, j] *= -1
                    Uf[:, j] *= -1
            UU, VV = Uf, Vs
        T[r0:, r0:] = UU.T @ X @ VV
        T[:r0, r0:] = T[:r0, r0:] @ VV
        U[:, r0:] = U[:, r0:] @ UU
        V[:, r0:] = V[:, r0:] @ VV
    return U, T, V


@pytest.mark.parametrize("shape,b,q", [((48, 48), 8, 1), ((57, 41), 8, 2), ((40, 37), 6, 0)])
def test_oracle_matches_dense_lapack_version(shape, b, q):
    """Figure randUTV vs a dense LAPACK-primitive implementation of the same
    steps on tiny inputs: elementwise agreement of U, T, V (same packed G)."""
    m, n = shape
    A = wl.planted(m, n, np.exp(-np.arange(1, n + 1) / 10.0), seed=8)
    G = wl.gaussian_g(m, n, b, seed=1)
    U, T, V, k = ref.randutv(A, b, q, G)
    U2, T2, V2 = _dense_lapack_randutv(A, b, q, G)
    # Columns of U beyond n are a complement of the range (not unique across
    # the two final-step routes); compare the first n.
    np.testing.assert_allclose(T, T2, atol=1e-11)
    np.testing.assert_allclose(V, V2, atol=1e-10)
    np.testing.assert_allclose(U[:, :n], U2[:, :n], atol=1e-10)
    _check_utv(A, U, T, V, k, b)


@pytest.mark.parametrize("shape,b,q", [((41, 57), 8, 2), ((37, 40), 6, 0), ((30, 90), 8, 1)])
def test_wide_matches_dense_lapack_version(shape, b, q):
    """m < n (Remark on the case m < n): the first s-1 steps as for tall
    input, the last one an LQ of the block row followed by the small SVD.
    Against the dense LAPACK-primitive version: U, and the first m columns
    of T and V (the columns beyond are a Householder complement in one route
    and LAPACK's in the other, so not comparable); plus the UTV invariants."""
    m, n = shape
    A = wl.planted(m, n, np.exp(-np.arange(1, m + 1) / 10.0), seed=8)
    G = wl.gaussian_g(m, n, b, seed=1)
    U, T, V, k = ref.randutv(A, b, q, G)
    assert k == m
    U2, T2, V2 = _dense_lapack_randutv(A, b, q, G)
    np.testing.assert_allclose(T[:, :m], T2[:, :m], atol=1e-11)
    np.testing.assert_allclose(V[:, :m], V2[:, :m], atol=1e-10)
    np.testing.assert_allclose(U, U2, atol=1e-10)
    _check_utv(A, U, T, V, k, b)
    assert np.all(np.tril(T, -1) == 0.0)


@pytest.mark.parametrize("shape,b,q,p", [((48, 40), 8, 1, 4), ((60, 60), 8, 2, 8), ((40, 56), 8, 0, 3)])
def test_oversampling_matches_dense_lapack_version(shape, b, q, p):
    """Over-sampling (Appendix A.2, Figure stepUTVoversampling): against the
    dense LAPACK-primitive version (LAPACK's gesvd for the extended sample's
    singular vectors, LAPACK QR for the reflectors): T, V and the first
    min(m, n) columns of U elementwise, and the UTV invariants."""
    m, n = shape
    A = wl.planted(m, n, np.exp(-np.arange(1, min(m, n) + 1) / 10.0), seed=8)
    G = wl.gaussian_g(m, n, b, seed=1, p=p)
    U, T, V, k = ref.randutv(A, b, q, G, p=p)
    U2, T2, V2 = _dense_lapack_randutv(A, b, q, G, p)
    r = min(m, n)
    np.testing.assert_allclose(T[:, :r], T2[:, :r], atol=1e-11)
    np.testing.assert_allclose(V[:, :r], V2[:, :r], atol=1e-10)
    np.testing.assert_allclose(U[:, :r], U2[:, :r], atol=1e-10)
    _check_utv(A, U, T, V, k, b)


def test_oversampling_step_one_identities():
    """Theorem (Section 5.3) with the over-sampled basis: after one step,
    ||T(:, b:)||_F = ||A - A Q Q^T||_F and diag(T11) = sigma(A Q) for Q an
    orthonormal basis of the b dominant left singular vectors of the extended
    sample (A^T A)^q A^T G_1 (b + p columns), here from numpy's QR of those
    vectors; and the captured norm is no worse than the optimal rank-b one
    (Eckart-Young)."""
    m, n, b, q, p = 50, 40, 8, 1, 5
    A = wl.planted(m, n, np.exp(-np.arange(1, 41) / 6.0), seed=2)
    G = wl.gaussian_g(m, n, b, seed=1, p=p)
    U, T, V, k = ref.randutv(A, b, q, G, p=p, k_stop=b)
    assert k == b
    Y = A.T @ G[:, :b + p]
    for _ in range(q):
        Y = A.T @ (A @ Y)
    Zy, _, _ = np.linalg.svd(Y, full_matrices=False)
    Q, _ = np.linalg.qr(Zy[:, :b])
    e1 = np.linalg.norm(A - A @ Q @ Q.T)
    assert abs(np.linalg.norm(T[:, b:]) - e1) <= 1e-12 * e1 + 1e-14
    np.testing.assert_allclose(np.diag(T)[:b], np.linalg.svd(A @ Q, compute_uv=False), rtol=1e-13)
    sig = np.linalg.svd(A, compute_uv=False)
    assert e1 >= np.sqrt(np.sum(sig[b:] ** 2)) * (1 - 1e-12)


def test_oversampling_rank_le_b_equals_plain():
    """rank(A) <= b: with or without over-sampling the first step's sample
    spans the whole row space, so both capture A in the first block:
    diag(T11) = sigma and the rest of T vanishes."""
    m, n, b = 60, 40, 8
    sig = np.array([5.0, 3.0, 2.0, 1.5, 1.0, 0.5])
    A = wl.planted(m, n, sig, seed=9)
    for p in (0, 6):
        G = wl.gaussian_g(m, n, b, seed=1, p=p)
        U, T, V, k = ref.randutv(A, b, 1, G, p=p)
        np.testing.assert_allclose(np.diag(T)[:6], sig, rtol=1e-13)
        assert np.linalg.norm(T[:, 6:]) <= 1e-13 * 5
        _check_utv(A, U, T, V, k, b)


def test_c1_invariants_and_logdet_golden():
    """500 x 500, b = 32, q = 1 workload: UTV invariants and the closed-form
    log-determinant sum_k log T_kk = sum_j log sigma_j = -2505 (golden)."""
    gold = json.load(open(os.path.join(GOLDEN, "logdet_c1.json")))
    A, sig = wl.config_matrix("c1_500")
    G, (U, T, V, k) = _factor(A, 32, 1)
    assert k == 500
    _check_utv(A, U, T, V, k, 32)
    ld = np.sum(np.log(np.diag(T)))
    assert abs(ld - gold["sum_log_diag"]) <= 1e-8 * abs(gold["sum_log_diag"])
    # Majorization (Ky Fan): partial sums of T_jj^2 never exceed those of sigma^2.
    d2 = np.cumsum(np.diag(T) ** 2)
    s2 = np.cumsum(sig ** 2)
    assert np.all(d2 <= s2 * (1 + 1e-13))
    # First block: T_kk <= sigma_k (singular values of A V1 are <= those of A).
    assert np.all(np.diag(T)[:32] <= sig[:32] * (1 + 1e-13))
    # Eckart-Young lower bound and Theorem (b): ||A - A_k||_F = ||T(k:,k:)||_F.
    for kk in (32, 128, 256):
        Uk = U[:, :kk]
        Ak = Uk @ (T[:kk, :] @ V.T)
        err = np.linalg.norm(A - Ak)
        assert abs(err - np.linalg.norm(T[kk:, kk:])) <= 1e-12 * np.linalg.norm(A)
        assert err >= np.sqrt(np.sum(sig[kk:] ** 2)) * (1 - 1e-12)


def test_early_stop_rank_and_residual():
    """Section 1.1 (ii): incremental factorization halts once the trailing
    block is below tolerance.  Scaled-down early-stop workload: rank-30
    planted (sigma_j = 1/j) plus noise of norm 1e-8 ||A_p||_F, b = 16, q = 2,
    tol = 1e-6: the first multiple of b >= 30 is 32."""
    m, n, b = 400, 120, 16
    sig = 1.0 / np.arange(1, 31)
    Ap = wl.planted(m, n, sig, seed=0)
    rng = np.random.default_rng(2)
    E = rng.standard_normal((m, n))
    E *= 1e-8 * np.linalg.norm(sig) / np.linalg.norm(E)
    A = Ap + E
    G = wl.gaussian_g(m, n, b, seed=1)
    U, T, V, k = ref.randutv(A, b, 2, G, tol=1e-6)
    assert k == 32
    assert np.linalg.norm(A - U @ T @ V.T) <= 1e-13 * np.linalg.norm(A)
    rel = np.linalg.norm(T[k:, k:]) / np.linalg.norm(A)
    assert 0.8e-8 <= rel <= 1.0e-8
    # k_stop gives the same prefix
    U2, T2, V2, k2 = ref.randutv(A, b, 2, G, k_stop=32)
    assert k2 == 32
    np.testing.assert_array_equal(T2, T)


def test_flop_formula_golden_ratios():
    """Section 5.4: (5+2q) m n^2 - (3+2q) n^3/3, which for square matrices is
    3, 4, 5 times the QR cost for q = 0, 1, 2 (golden), and agrees with the
    exact per-step sum of the thin products to within a few percent."""
    gold = json.load(open(os.path.join(GOLDEN, "flop_ratios.json")))
    n = 8000
    qr = 2 * n ** 3 - 2 * n ** 3 / 3
    for q, r in gold["ratio_by_q"].items():
        assert abs(ref.flops_paper(n, n, int(q)) / qr - r) < 1e-12
    for (m, n, b, q) in [(8000, 8000, 256, 1), (4000, 4000, 128, 1), (8000, 8000, 256, 2)]:
        exact = 0.0
        for i in range(ref.num_random_steps(m, n, b)):
            Mi, Ni = m - i * b, n - i * b
            exact += (2 * q + 1) * 2 * Mi * Ni * b + 4 * m * Ni * b + 4 * Mi * (Ni - b) * b
        assert abs(exact / ref.flops_paper(m, n, q) - 1) < 0.05


def _uv_forward_flops(m, n, b):
    """Flops of forming U and V by forward accumulation, summed step by step
    over the partitions of Figure randUTV (m >= n): each step applies its
    block of w = |J2| reflectors, which act on rows I2 u I3 (m_i of them) of
    U's trailing columns and rows J2 u J3 (n_i) of V's, to all m rows of U
    and n rows of V (U(:,[I2,I3]) and V(:,[J2,J3]) times the orthogonal
    factor): two thin products each in the compact WY form, 4 m m_i w + 2 m
    w^2 and 4 n n_i w + 2 n w^2; then the small-SVD rotations of the step,
    U(:,I2) Us and V(:,J2) Vs, 2 m w^2 + 2 n w^2.  The last step (no
    randomization) applies the QR reflectors of its tall block to U only
    (its square case has none), then its rotations."""
    tot = 0.0
    for i in range(ref.num_steps(m, n, b)):
        r0 = i * b
        w = min(r0 + b, n) - r0
        mi, ni = m - r0, n - r0
        if r0 + b < m and r0 + b < n:
            tot += 4 * m * mi * w + 2 * m * w * w + 4 * n * ni * w + 2 * n * w * w
            tot += 2 * m * w * w + 2 * n * w * w
        else:
            c = ni
            if mi > c:
                tot += 4 * m * mi * c + 2 * m * c * c
            tot += 2 * m * c * c + 2 * n * c * c
    return tot


@pytest.mark.parametrize("m,n", [(8000, 8000), (4000, 4000), (20000, 5000), (6000, 2000)])
def test_flops_uv_is_leading_order_of_per_step_sum(m, n):
    """flops_uv (4 m^2 n - 2 m n^2 + 2 n^3, the U and V formation of Figure
    randUTV by forward accumulation) is the leading-order term of the exact
    per-step sum: with a tiny block size (b = 4) the two agree to well under
    1 %, and at the workloads' block sizes they differ by the O(b/n) terms
    the formula drops (below 3 b / n relatively)."""
    exact = _uv_forward_flops(m, n, 4)
    assert abs(ref.flops_uv(m, n) / exact - 1.0) < 0.005
    for b in (128, 256):
        exact = _uv_forward_flops(m, n, b)
        assert 0.0 < 1.0 - ref.flops_uv(m, n) / exact < 3.0 * b / n


def test_approx_equals_truncated_factor():
    """eq. Ak_randUTV and Theorem (b): A_k = U(:,1:k) T(1:k,:) V^T = U_k U_k^T A,
    and it does not depend on the small SVD rotations (skipped in approx)."""
    m, n, b, q, k = 64, 48, 8, 1, 16
    A = wl.planted(m, n, np.exp(-np.arange(1, n + 1) / 8.0), seed=5)
    G = wl.gaussian_g(m, n, b, seed=1)
    Ak, Uk = ref.approx(A, G, b, q, k)
    U, T, V, kk = ref.randutv(A, b, q, G)
    Ak2 = U[:, :k] @ T[:k, :] @ V.T
    np.testing.assert_allclose(Ak, Ak2, atol=1e-13)
    np.testing.assert_allclose(Uk.T @ Uk, np.eye(k), atol=1e-14)


def test_complex_step_tangent_matches_finite_differences():
    """The oracle's tangent (complex step through approx) against FP64 central
    finite differences of the real oracle, 64 x 48, k = b = 8, q = 1."""
    m, n, b, q, k = 64, 48, 8, 1, 8
    A = wl.planted(m, n, np.exp(-np.arange(1, n + 1) / 100.0), seed=0)
    G = wl.gaussian_g(m, n, b, seed=1)
    rng = np.random.default_rng(3)
    dA = rng.standard_normal((m, n))
    J = ref.approx_jvp(A, G, b, q, k, dA)
    h = 1e-6
    fp, _ = ref.approx(A + h * dA, G, b, q, k)
    fm, _ = ref.approx(A - h * dA, G, b, q, k)
    fd = (fp - fm) / (2 * h)
    assert np.linalg.norm(J - fd) <= 1e-7 * np.linalg.norm(J)
    # Two steps (k = 2b): the complement of step 1 enters; still smooth.
    k2 = 16
    J2 = ref.approx_jvp(A, G, b, q, k2, dA)
    fp, _ = ref.approx(A + h * dA, G, b, q, k2)
    fm, _ = ref.approx(A - h * dA, G, b, q, k2)
    assert np.linalg.norm(J2 - (fp - fm) / (2 * h)) <= 1e-6 * np.linalg.norm(J2)


def test_zero_matrix():
    """Degenerate input: A = 0 gives T = 0 with every reflector the identity
    (tau = 0) and U = V = I (no NaN)."""
    A = np.zeros((20, 16))
    G = wl.gaussian_g(20, 16, 4, seed=1)
    U, T, V, k = ref.randutv(A, 4, 1, G)
    assert np.all(T == 0.0) and np.all(np.isfinite(U)) and np.all(np.isfinite(V))
    np.testing.assert_allclose(U.T @ U, np.eye(20), atol=1e-15)


# --------------------------------------------------------------------------
# Randomized SVD (Section 2.5, Remark RSVD, eqs. panda1, panda2).
# --------------------------------------------------------------------------
def _rsvd_case(m=120, n=90, decay=8.0, seed=4):
    sig = np.exp(-np.arange(1, min(m, n) + 1) / decay)
    return wl.planted(m, n, sig, seed=seed), sig


@pytest.mark.parametrize("k,p,q", [(10, 0, 0), (10, 0, 2), (12, 6, 1), (30, 10, 1)])
def test_rsvd_matches_dense_lapack_version(k, p, q):
    """The oracle's RSVD against a dense re-implementation on LAPACK
    primitives (scipy's dgeqrf/dorgqr Q of the sample, whose reflectors use
    the same dlarfg convention, and gesdd of B), with the same sign rule."""
    A, _ = _rsvd_case()
    G = np.random.default_rng(1).standard_normal((A.shape[0], k + p))
    U, D, V, Q = ref.rsvd(A, k, q, G, p=p)
    Y = A.T @ G
    for _ in range(q):
        Y = A.T @ (A @ Y)
    Ql, _ = scipy.linalg.qr(Y, mode="economic")
    # Householder QR is backward stable, so two orderings of its rounding give
    # Q's that differ by about eps * cond(Y).
    tol = max(1e-12, 1e-14 * np.linalg.cond(Y))
    np.testing.assert_allclose(Q, Ql, rtol=0, atol=tol)
    Ub, Db, Wt = scipy.linalg.svd(A @ Ql, full_matrices=False, lapack_driver="gesdd")
    for j in range(k):
        if Wt[j, np.argmax(np.abs(Wt[j]))] < 0:
            Wt[j] *= -1
            Ub[:, j] *= -1
    np.testing.assert_allclose(D, Db[:k], rtol=1e-12)
    np.testing.assert_allclose(U, Ub[:, :k], rtol=0, atol=max(1e-10, tol))
    np.testing.assert_allclose(V, Ql @ Wt[:k].T, rtol=0, atol=max(1e-10, tol))


def test_rsvd_error_equals_range_finder_error():
    """Remark RSVD: stage two is exact, so A - U D V^T = A - A Q Q^T (p = 0)
    in both norms; with p > 0, U D V^T is the best rank-k approximation of
    A Q Q^T (Eckart-Young on B = A Q)."""
    A, _ = _rsvd_case()
    m, n = A.shape
    k = 15
    G = np.random.default_rng(1).standard_normal((m, k + 8))
    U, D, V, Q = ref.rsvd(A, k, 1, G[:, :k])
    E1 = A - (U * D) @ V.T
    E2 = A - A @ Q @ Q.T
    assert abs(np.linalg.norm(E1) - np.linalg.norm(E2)) <= 1e-13 * np.linalg.norm(A)
    assert abs(np.linalg.norm(E1, 2) - np.linalg.norm(E2, 2)) <= 1e-13 * np.linalg.norm(A)
    U, D, V, Q = ref.rsvd(A, k, 1, G, p=8)
    P = A @ Q @ Q.T
    Up, Dp, Vpt = np.linalg.svd(P)
    best = (Up[:, :k] * Dp[:k]) @ Vpt[:k]
    np.testing.assert_allclose((U * D) @ V.T, best, rtol=0, atol=1e-12 * np.linalg.norm(A))
    # U, V orthonormal; D descending and nonnegative.
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= 1e-13 and np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-13
    assert np.all(np.diff(D) <= 0) and D[-1] >= 0


def test_rsvd_exact_on_rank_le_k():
    """rank(A) = 7 <= k = 10: the range finder captures the row space, so
    U D V^T = A and D holds the singular values (then zeros)."""
    sig = np.array([4.0, 3.0, 2.0, 1.0, 0.5, 0.25, 0.125])
    A = wl.planted(80, 60, sig, seed=3)
    G = np.random.default_rng(1).standard_normal((80, 10))
    U, D, V, _ = ref.rsvd(A, 10, 0, G)
    np.testing.assert_allclose(D[:7], sig, rtol=1e-13)
    assert np.all(np.abs(D[7:]) <= 1e-13)
    np.testing.assert_allclose((U * D) @ V.T, A, rtol=0, atol=1e-13 * 4)


def test_rsvd_range_matches_randutv_first_step():
    """Section 5.3 (connection between RSVD and randUTV): with k = b and the
    same G_1, RSVD's Q spans randUTV's first block of V, so the RSVD error
    equals ||T(:, b:)||_F after randUTV's first step, and D equals the first
    diagonal block of T (sigma(A Q) in both)."""
    m, n, b, q = 60, 50, 8, 1
    A = wl.planted(m, n, np.exp(-np.arange(1, 51) / 6.0), seed=2)
    G = wl.gaussian_g(m, n, b, seed=1)
    _, T, _, k = ref.randutv(A, b, q, G, k_stop=b)
    U, D, V, Q = ref.rsvd(A, b, q, G[:, :b])
    e = np.linalg.norm(A - (U * D) @ V.T)
    assert abs(e - np.linalg.norm(T[:, b:])) <= 1e-12 * e
    np.testing.assert_allclose(D, np.diag(T)[:b], rtol=1e-12)


# --------------------------------------------------------------------------
# Lower-triangular middle factor (Section 1: upper or lower, as preferred).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,b,q", [((60, 40), 8, 1), ((40, 60), 8, 1), ((50, 50), 16, 2)])
def test_lower_variant_invariants(shape, b, q):
    """A = U L V^T with U, V orthogonal, L lower triangular with diagonal
    blocks, its diagonal nonnegative and descending inside each block, and
    Ky Fan's bound on the leading diagonal entries."""
    m, n = shape
    sig = np.exp(-np.arange(1, min(m, n) + 1) / 6.0)
    A = wl.planted(m, n, sig, seed=3)
    G = wl.gaussian_g(n, m, b, seed=1)
    U, L, V, k = ref.randutv_lower(A, b, q, G)
    assert k == min(m, n)
    assert np.linalg.norm(A - U @ L @ V.T) <= 1e-13 * np.linalg.norm(A)
    assert np.linalg.norm(U.T @ U - np.eye(m)) <= 1e-13 and np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-13
    assert np.all(np.triu(L, 1) == 0.0)
    d = np.diag(L)
    for s0 in range(0, min(m, n), b):
        blk = L[s0:s0 + b, s0:s0 + b]
        assert np.all(blk - np.diag(np.diag(blk)) == 0.0)
        db = d[s0:s0 + b]
        assert np.all(db >= 0) and np.all(np.diff(db) <= 0)
    assert np.all(np.cumsum(d ** 2) <= np.cumsum(sig ** 2) * (1 + 1e-12))


def test_lower_variant_b_ge_min_is_svd():
    """b >= min(m, n): one step, the final SVD, so L = [diag(sigma), 0] and
    U L V^T is an SVD of A."""
    sig = np.array([3.0, 2.0, 1.5, 0.7, 0.2])
    A = wl.planted(9, 5, sig, seed=4)
    G = wl.gaussian_g(5, 9, 8, seed=1)
    U, L, V, k = ref.randutv_lower(A, 8, 1, G)
    np.testing.assert_allclose(np.diag(L), sig, rtol=1e-13)
    assert np.linalg.norm(L[:5, :5] - np.diag(sig)) <= 1e-13 * 3
    assert np.linalg.norm(L[5:, :]) == 0.0
    assert np.linalg.norm(A - U @ L @ V.T) <= 1e-13 * 3
