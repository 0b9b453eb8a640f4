"""Plain, slow FP64 CPU oracle for randUTV (Martinsson, Quintana-Orti, Heavner,
"randUTV: A blocked randomized algorithm for computing a rank-revealing UTV
factorization", arXiv:1703.00998).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product path (the
HIP library and its Python binding) never calls it, and the two share no code.

The oracle follows the blocked algorithm of the paper's Figure "The algorithm
randUTV" (Section 5.2) in the paper's order and notation, one Householder
reflector at a time (BLAS-2 style, no compact-WY blocking), with numpy used
only for vector/matrix primitives (products, and the LAPACK SVD of the small
b x b diagonal block, which the paper also obtains from a library `svd`).

Conventions the paper leaves open (each is listed with its reading in the
design notes of the repository):
  * Householder sign: LAPACK dlarfg convention (`householder` below).
  * SVD of the b x b block: singular values descending; each pair (u_j, v_j) is
    sign-normalised so that the largest-magnitude entry of v_j is positive
    (ties: lowest index) (`small_svd`).
  * Random matrices: step i (0-based) uses the leading m - i*b rows of column
    block i of one packed m x (s_r*(b+p)) Gaussian matrix G (`g_slab`).
  * Over-sampling (p > 0): the b dominant left singular vectors of the
    extended sampling matrix, signs normalised as for the small SVDs.
  * The QR factorization of the sampling matrix is unpivoted Householder QR
    (Section 4.3; Figure randUTV).
  * The right transform touches all m rows of T (Figure randUTV: the whole
    block column J2 u J3, rows I1 included).
  * Early stop: after step i, stop when ||T(I3,J3)||_F <= tol*||A||_F or when
    (i+1)*b >= k_stop (Section 1.1, advantage (ii)).
  * Lower-triangular middle factor (`randutv_lower`): randUTV of A^T,
    transposed.
  * Randomized SVD (`rsvd`, Remark RSVD): the b dominant triplets of the
    rank-(b+p) factorization when over-sampling; signs as for the small SVDs.

All routines are written without complex conjugation (``x @ x`` instead of
``|x|^2``, ``.T`` instead of ``.conj().T``, branch decisions on ``.real``) so
that `approx` can be run on complex input for a complex-step tangent
(`approx_jvp`); for real input this changes nothing.
"""
from __future__ import annotations

import math
import numpy as np

__all__ = [
    "householder", "house_qr", "apply_right", "apply_left", "small_svd",
    "top_left_singular_vectors",
    "num_steps", "num_random_steps", "g_slab", "randutv", "approx",
    "approx_jvp", "rsvd", "randutv_lower", "flops_paper", "flops_uv",
]


# --------------------------------------------------------------------------
# Section 2.4 (eq. unpivQR, eq. WYrepresentation): Householder reflectors.
# --------------------------------------------------------------------------
def householder(x):
    """Return (v, tau, beta) with (I - tau v v^T) x = beta e_1 and v[0] = 1.

    LAPACK dlarfg convention: with x = (alpha, x2),
      * if x2 == 0: tau = 0, beta = alpha (H = I, even when alpha < 0);
      * else beta = -sign(alpha) * ||x|| (sign(0) = +1), tau = (beta-alpha)/beta,
        v = (1, x2 / (alpha - beta)).
    """
    alpha = x[0]
    x2 = x[1:]
    xnorm2 = x2 @ x2 if x2.size else 0.0 * alpha
    v = np.zeros_like(x)
    v[0] = 1.0
    if np.real(xnorm2) == 0.0:
        return v, 0.0 * alpha, alpha
    sgn = 1.0 if np.real(alpha) >= 0.0 else -1.0
    beta = -sgn * np.sqrt(alpha * alpha + xnorm2)
    tau = (beta - alpha) / beta
    v[1:] = x2 / (alpha - beta)
    return v, tau, beta


def house_qr(B):
    """Unpivoted Householder QR of B (p x c), one column at a time.

    Returns (refl, R) where refl[j] = (v_j, tau_j) acts on rows j: of B and
    B = H_0 H_1 ... H_{k-1} [R; 0] with H_j = I - tau_j v_j v_j^T embedded at
    rows j:, k = min(p, c).  R is the k x c upper-trapezoidal factor.
    """
    B = np.array(B, copy=True)
    p, c = B.shape
    k = min(p, c)
    refl = []
    for j in range(k):
        v, tau, beta = householder(B[j:, j])
        if c > j + 1:
            w = v @ B[j:, j + 1:]
            B[j:, j + 1:] -= tau * np.outer(v, w)
        B[j, j] = beta
        B[j + 1:, j] = 0.0
        refl.append((v, tau))
    return refl, np.triu(B[:k, :])


def apply_right(C, refl):
    """In place C <- C H_0 H_1 ... H_{k-1} (C's columns are the reflectors' rows)."""
    for j, (v, tau) in enumerate(refl):
        w = C[:, j:] @ v
        C[:, j:] -= tau * np.outer(w, v)
    return C


def apply_left(C, refl):
    """In place C <- (H_0 H_1 ... H_{k-1})^T C = H_{k-1} ... H_0 C."""
    for j, (v, tau) in enumerate(refl):
        w = v @ C[j:, :]
        C[j:, :] -= tau * np.outer(v, w)
    return C


# --------------------------------------------------------------------------
# Section 2.2 (eq. defSVD), Figure randUTV: SVD of the small diagonal block.
# --------------------------------------------------------------------------
def small_svd(R):
    """Full SVD R = Us diag(D) Vs^T of a small square or tall block.

    Singular values descending and >= 0 (LAPACK).  Each pair (u_j, v_j) is
    flipped so that the largest-magnitude entry of v_j is positive (first
    index on ties).  For a tall p x c input, Us is p x p (full).
    """
    Us, D, Vt = np.linalg.svd(R, full_matrices=True)
    Vs = Vt.T.copy()
    Us = Us.copy()
    for j in range(D.size):
        idx = int(np.argmax(np.abs(Vs[:, j])))
        if Vs[idx, j] < 0.0:
            Vs[:, j] = -Vs[:, j]
            Us[:, j] = -Us[:, j]
    return Us, D, Vs


# --------------------------------------------------------------------------
# Figure randUTV: partitions and the random input.
# --------------------------------------------------------------------------
def num_steps(m, n, b):
    """Number of steps s = min(ceil(m/b), ceil(n/b)) of Figure randUTV."""
    return min(-(-m // b), -(-n // b))


def num_random_steps(m, n, b):
    """Steps whose I3 and J3 are both nonempty (the randomized branch)."""
    return sum(1 for i in range(num_steps(m, n, b))
               if i * b + b < m and i * b + b < n)


def g_slab(G, m, b, i, p=0):
    """G_i: the leading m - i*b rows of column block i (b + p columns wide)
    of the packed G."""
    w = b + p
    return G[: m - i * b, i * w:(i + 1) * w]


def top_left_singular_vectors(Y, b):
    """The b dominant left singular vectors of the n_i x (b+p) matrix Y
    (Appendix A.2, Figure stepUTVoversampling: the leading b left singular
    vectors of the economic SVD of Y), each pair (z_j, w_j) sign-normalised like `small_svd` (the
    largest-magnitude entry of the right singular vector w_j positive)."""
    Z, _, Wt = np.linalg.svd(Y, full_matrices=False)
    Z = Z[:, :b].copy()
    for j in range(b):
        idx = int(np.argmax(np.abs(Wt[j, :])))
        if Wt[j, idx] < 0.0:
            Z[:, j] = -Z[:, j]
    return Z


# --------------------------------------------------------------------------
# Figure randUTV (Section 5.2): the blocked algorithm.
# --------------------------------------------------------------------------
def randutv(A, b, q, G, *, p=0, form_u=True, form_v=True, k_stop=0, tol=0.0,
            small_svds=True):
    """The blocked randUTV of Section 5.2 (Figure randUTV): A = U T V^T.

    A: m x n (any shape).  G: m x (num_random_steps*(b+p)) packed Gaussian.
    p > 0 over-samples (Remark "Oversampling" in Section 5.3, Appendix A.2,
    Figure stepUTVoversampling): each step draws b+p samples, and the
    Householder QR is taken of the b dominant left singular vectors of the
    extended sampling matrix instead of the sampling matrix itself.
    Returns U (m x m or None), T (m x n), V (n x n or None), and k, the
    number of leading columns driven to triangular form (= min(m, n) unless
    the factorization stopped early).  With m < n the last step takes the
    SVD of the wide block row through an LQ of its rows (Remark on the case
    m < n, Section 5.2).

    small_svds=False skips the b x b SVD of each randomized step (the
    diagonal blocks are then left as the R factors of the panel QR).  This is
    only used by `approx`, whose result does not depend on those rotations.
    """
    A = np.asarray(A)
    m, n = A.shape
    if b < 1 or q < 0 or p < 0:
        raise ValueError("randutv oracle: b >= 1, q >= 0 and p >= 0 required")
    dt = np.result_type(A.dtype, np.float64)
    T = np.array(A, dtype=dt, copy=True)
    U = np.eye(m, dtype=dt) if form_u else None
    V = np.eye(n, dtype=dt) if form_v else None
    normA = math.sqrt(float(np.real(np.sum(A * A))))
    s = num_steps(m, n, b)
    k_done = min(m, n)
    for i in range(s):
        r0 = i * b
        r1 = min(r0 + b, m)          # I2 = r0:r1, I3 = r1:m
        c1 = min(r0 + b, n)          # J2 = r0:c1, J3 = c1:n
        if r1 < m and c1 < n:
            # The sampling matrix (X^T X)^q X^T G_i of the trailing block X.
            X = T[r0:, r0:]
            Gi = g_slab(G, m, b, i, p)
            Y = X.T @ Gi
            for _ in range(q):
                Y = X.T @ (X @ Y)
            if p > 0:
                Y = top_left_singular_vectors(Y, b)
            # Right transform: the Householder reflectors of Y act on the
            # trailing columns of T (all rows) and of V.
            reflV, _ = house_qr(Y)
            apply_right(T[:, r0:], reflV)
            if form_v:
                apply_right(V[:, r0:], reflV)
            # Left transform: the Householder QR of the new block column J2
            # (rows I2 u I3) acts on U's trailing columns and, transposed,
            # on the trailing rows of T right of the block; below the
            # block's R the column is zero.
            reflU, R = house_qr(T[r0:, r0:c1])
            if form_u:
                apply_right(U[:, r0:], reflU)
            apply_left(T[r0:, c1:], reflU)
            T[r0:, r0:c1] = 0.0
            T[r0:r1, r0:c1] = R
            if small_svds:
                # SVD of the diagonal block; its rotations fold into block
                # row I2, block column J2 and the matching columns of U, V.
                Us, D, Vs = small_svd(R)
                T[r0:r1, r0:c1] = np.diag(D)
                T[r0:r1, c1:] = Us.T @ T[r0:r1, c1:]
                if form_u:
                    U[:, r0:r1] = U[:, r0:r1] @ Us
                T[:r0, r0:c1] = T[:r0, r0:c1] @ Vs
                if form_v:
                    V[:, r0:c1] = V[:, r0:c1] @ Vs
            # Early stop (Section 1.1 (ii)): halt once the trailing block is small.
            if (k_stop > 0 and c1 >= k_stop) or (
                    tol > 0.0 and
                    math.sqrt(float(np.real(np.sum(T[r1:, c1:] * T[r1:, c1:]))))
                    <= tol * normA):
                k_done = c1
                break
        else:
            # Last block: SVD of T([I2,I3],[J2,J3]); economic (QR first) if tall
            # (Remark on the economic SVD of a tall matrix, Section 4.4).
            X = np.array(T[r0:, r0:])
            p, c = X.shape
            if p < c:
                # Fewer rows than columns (Remark on the case m < n): an
                # unpivoted QR of the rows, X^T = H [R; 0], so X = [R^T, 0] H^T,
                # then the SVD of the p x p lower-triangular L = R^T.  The right
                # transform is H diag(Vs, I): its reflectors act on the
                # columns of T (all rows above the block) and of V.
                reflV, R = house_qr(X.T)
                Us, D, Vs = small_svd(R[:p, :p].T)
                apply_right(T[:r0, r0:], reflV)
                T[:r0, r0:r0 + p] = T[:r0, r0:r0 + p] @ Vs
                if form_v:
                    apply_right(V[:, r0:], reflV)
                    V[:, r0:r0 + p] = V[:, r0:r0 + p] @ Vs
                if form_u:
                    U[:, r0:] = U[:, r0:] @ Us
                T[r0:, r0:] = 0.0
                T[r0:, r0:r0 + p] = np.diag(D)
                continue
            if p == c:
                Us, D, Vs = small_svd(X)
                if form_u:
                    U[:, r0:] = U[:, r0:] @ Us
            else:
                reflU, R = house_qr(X)
                Us, D, Vs = small_svd(R[:c, :c])
                if form_u:
                    apply_right(U[:, r0:], reflU)
                    U[:, r0:r0 + c] = U[:, r0:r0 + c] @ Us
            T[r0:, r0:] = 0.0
            T[r0:r0 + c, r0:r0 + c] = np.diag(D)
            T[:r0, r0:] = T[:r0, r0:] @ Vs
            if form_v:
                V[:, r0:] = V[:, r0:] @ Vs
    return U, T, V, k_done


# --------------------------------------------------------------------------
# Section 1 (the middle factor may be taken lower triangular): A = U L V^T.
# --------------------------------------------------------------------------
def randutv_lower(A, b, q, G, **kw):
    """[U, L, V, k] with L lower triangular, from randUTV of A^T:
    A^T = U' T V'^T gives A = V' T^T U'^T, so U = V', L = T^T, V = U'.
    G is the packed Gaussian of the n x m problem (n rows).  k counts the
    leading rows of L in lower-triangular form."""
    U1, T1, V1, k = randutv(np.asarray(A).T, b, q, G, **kw)
    return V1, T1.T.copy(), U1, k


# --------------------------------------------------------------------------
# Section 6.2 eq. Ak_randUTV, Theorem part (b): truncated approximation.
# --------------------------------------------------------------------------
def approx(A, G, b, q, k):
    """A_k = U(:,1:k) T(1:k,:) V^T = U_k U_k^T A after k/b steps (k % b == 0).

    The equality U_k T(1:k,:) V^T = U_k U_k^T A follows from A = U T V^T with
    U orthogonal.  U_k U_k^T does not depend on the b x b rotations Us of each
    step (they mix columns inside one block), so the SVDs are skipped.
    Returns (A_k, U_k).
    """
    m, n = np.shape(A)
    if k % b != 0 or k <= 0 or k >= min(m, n):
        raise ValueError("approx oracle: k must be a positive multiple of b below min(m, n)")
    U, _, _, kd = randutv(A, b, q, G, form_u=True, form_v=False, k_stop=k,
                          small_svds=False)
    if kd != k:
        raise ValueError("approx oracle: factorization did not reach k")
    Uk = U[:, :k]
    return Uk @ (Uk.T @ A), Uk


def approx_jvp(A, G, b, q, k, dA, h=1e-30):
    """Directional derivative of A -> A_k along dA (G fixed), by complex step.

    d/dt A_k(A + t dA) at t = 0 equals Im(A_k(A + i h dA)) / h up to O(h^2),
    with no subtractive cancellation, so h can be tiny; valid wherever no
    Householder sign decision (sign of alpha) flips along the path.
    """
    Ac = np.asarray(A, dtype=np.complex128) + 1j * h * np.asarray(dA, dtype=np.float64)
    Ak, _ = approx(Ac, np.asarray(G, dtype=np.float64), b, q, k)
    return np.imag(Ak) / h


# --------------------------------------------------------------------------
# Section 2.5, Remark RSVD (eqs. panda1, panda2) and Remark on over-sampling:
# the two-stage randomized SVD on the same building blocks.
# --------------------------------------------------------------------------
def rsvd(A, k, q, G, p=0):
    """Rank-k randomized SVD A ~ U diag(D) V^T.

    Stage one, the range finder of Section 2.5: Y = (A^T A)^q A^T G with G
    of size m x (k+p), Q = the orthonormal factor of Y's unpivoted
    Householder QR (n x (k+p)).  Stage two, Remark RSVD: B = A Q, the
    economic SVD B = Ub diag(Db) Vb^T (signs as in `small_svd`: the
    largest-magnitude entry of each right singular vector positive), then
    U = Ub, V = Q Vb.  With over-sampling (p > 0) the rank-(k+p) result is
    truncated to its k dominant triplets.  Returns (U m x k, D (k,),
    V n x k, Q n x (k+p)).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    c = k + p
    if k < 1 or p < 0 or q < 0 or c > min(m, n):
        raise ValueError("rsvd oracle: 1 <= k, 0 <= p, k + p <= min(m, n), q >= 0")
    Y = A.T @ G[:, :c]
    for _ in range(q):
        Y = A.T @ (A @ Y)
    refl, _ = house_qr(Y)
    Q = apply_right(np.eye(n), refl)[:, :c]     # H_0 ... H_{c-1} [I; 0]
    B = A @ Q
    Ub, Db, Wt = np.linalg.svd(B, full_matrices=False)
    W = Wt.T.copy()
    for j in range(c):
        idx = int(np.argmax(np.abs(W[:, j])))
        if W[idx, j] < 0.0:
            W[:, j] = -W[:, j]
            Ub[:, j] = -Ub[:, j]
    return Ub[:, :k].copy(), Db[:k].copy(), Q @ W[:, :k], Q


# --------------------------------------------------------------------------
# Section 5.4: flop counts.
# --------------------------------------------------------------------------
def flops_paper(m, n, q):
    """(5+2q) m n^2 - (3+2q) n^3 / 3: randUTV without forming U and V."""
    return (5 + 2 * q) * m * n * n - (3 + 2 * q) * n ** 3 / 3.0


def flops_uv(m, n):
    """Forming U and V by forward accumulation (Figure randUTV: U's and V's
    trailing columns times each step's orthogonal factor), m >= n: the sum
    over steps of 4 m m_i b + 4 n n_i b, to leading order
    4 m^2 n - 2 m n^2 + 2 n^3 (the O(b/n) terms are dropped)."""
    return 4.0 * m * m * n - 2.0 * m * n * n + 2.0 * n ** 3
