"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and builds test matrices with planted
singular values (Section 6.2, "Matrix 1 ... obtained by performing an
unpivoted QR factorization on a random Gaussian matrix").  It holds none of
randUTV's arithmetic, so both the GPU path and the CPU oracle consume its
output without sharing any of the method.

Every matrix is returned as a float64 numpy array in column-major (Fortran)
order, the layout of the C ABI.
"""
from __future__ import annotations

import numpy as np

__all__ = ["haar", "planted", "gaussian_g", "g_cols", "config_matrix",
           "CONFIGS", "fast_decay_sigma", "gap_sigma", "s_shape_sigma", "STUDY_SPECTRA"]


def haar(rng, n, k):
    """n x k matrix with orthonormal columns: QR of a Gaussian, columns
    scaled by sign(diag R) so that the law is Haar."""
    Z = rng.standard_normal((n, k))
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def planted(m, n, sigma, seed=0):
    """A = X diag(sigma) Y^T with X (m x r), Y (n x r) Haar, r = len(sigma).
    X is drawn before Y from numpy.random.default_rng(seed)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.size
    rng = np.random.default_rng(seed)
    X = haar(rng, m, r)
    Y = haar(rng, n, r)
    return np.asfortranarray((X * sigma) @ Y.T)


def g_cols(m, n, b, p=0):
    """Columns of the packed Gaussian: b + p per step whose I3 and J3 are
    both nonempty (m >= n: ceil(n/b) - 1 such steps)."""
    s = min(-(-m // b), -(-n // b))
    return (b + p) * sum(1 for i in range(s) if i * b + b < m and i * b + b < n)


def gaussian_g(m, n, b, seed=1, cols=None, p=0):
    """Packed N(0,1) matrix G, m x g_cols(m,n,b,p); step i uses the leading
    m - i*b rows of column block i (b + p columns wide)."""
    c = g_cols(m, n, b, p) if cols is None else cols
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, c)))


def fast_decay_sigma(n, beta=1e-5):
    """Matrix 1 of Section 6.2: d_j = beta^((j-1)/(n-1))."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return beta ** ((j - 1) / (n - 1))


def gap_sigma(n):
    """Matrix 3 of Section 6.2: 1/j for j <= 150, 0.1/j after."""
    j = np.arange(1, n + 1, dtype=np.float64)
    return np.where(j <= 150, 1.0 / j, 0.1 / j)


def s_shape_sigma(n, floor=1e-2):
    """Matrix 2 of Section 6.2 (S-shaped decay: near 1, a rapid drop, then
    level at 1e-2; the paper gives only a plot).  Reading: log10 sigma_j
    follows a logistic step from 0 to log10(floor), centred at j = n/8 with
    width n/80, so sigma_1 ~ 1 and sigma_n ~ 1e-2."""
    j = np.arange(1, n + 1, dtype=np.float64)
    s = 1.0 / (1.0 + np.exp(-(j - n / 8.0) / (n / 80.0)))
    return 10.0 ** (np.log10(floor) * s)


# Spectra of the rank-k accuracy study (Section 6.2; Matrix 4, the boundary
# integral operator, needs a discretization that is not part of this code).
STUDY_SPECTRA = {"fast_decay": fast_decay_sigma, "s_shape": s_shape_sigma,
                 "gap": gap_sigma}


def _sigma_exp(n, scale):
    j = np.arange(1, n + 1, dtype=np.float64)
    return np.exp(-j / scale)


# Workloads: (m, n, b, q, spectrum).  The spectra follow the configurations the
# repository is measured on; C4 adds Gaussian noise (see config_matrix).
CONFIGS = {
    "c1_500": dict(m=500, n=500, b=32, q=1,
                   sigma=lambda: _sigma_exp(500, 50.0)),
    "c2_4000": dict(m=4000, n=4000, b=128, q=1,
                    sigma=lambda: np.arange(1, 4001, dtype=np.float64) ** -1.5),
    "c3_8000": dict(m=8000, n=8000, b=256, q=1,
                    sigma=lambda: _sigma_exp(8000, 800.0) + 1e-10),
    "c4_20000x5000": dict(m=20000, n=5000, b=128, q=2,
                          sigma=lambda: 1.0 / np.arange(1, 301, dtype=np.float64)),
    "c5_2048x1024": dict(m=2048, n=1024, b=64, q=1,
                         sigma=lambda: _sigma_exp(1024, 100.0)),
}


def config_matrix(name, seed=0, noise_seed=2):
    """(A, sigma) for a named workload.  For the rank-300 early-stop case the
    planted part gets i.i.d. Gaussian noise E scaled to
    ||E||_F = 1e-8 ||A_planted||_F."""
    cfg = CONFIGS[name]
    sigma = cfg["sigma"]()
    A = planted(cfg["m"], cfg["n"], sigma, seed=seed)
    if name.startswith("c4"):
        rng = np.random.default_rng(noise_seed)
        E = rng.standard_normal(A.shape)
        E *= 1e-8 * np.linalg.norm(sigma) / np.linalg.norm(E)
        A = np.asfortranarray(A + E)
    return A, sigma
