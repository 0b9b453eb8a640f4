/*
 * randutv.h -- C ABI of the MI355X (gfx950) implementation of randUTV, the
 * blocked randomized rank-revealing UTV factorization A = U T V^T of
 * Martinsson, Quintana-Orti and Heavner (arXiv:1703.00998).
 *
 * Conventions shared by every entry point
 *  - Real matrices, column-major (LAPACK convention) with explicit leading
 *    dimensions.  All matrix pointers are DEVICE pointers owned by the caller;
 *    the library never frees caller memory.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL means
 *    the default stream).  Calls return once the work is enqueued, except
 *    where stated: the tolerance-based early stop reads one scalar per step
 *    back to the host, a non-NULL k_out / sweeps_out asks the call to wait
 *    for its results, and the building blocks randutv_panel_qr and
 *    randutv_small_svd wait for completion.  Every iteration count (the
 *    Jacobi sweeps of the small SVDs included) is decided on the device.
 *  - An enqueue-only call leaves its status in the first 256 bytes of its
 *    workspace; randutv_status() waits for the stream and reports it.
 *  - Return status: 0 on success; -i if argument i (1-based) is invalid
 *    (LAPACK INFO convention); RANDUTV_E_UNSUPPORTED for a valid but
 *    unimplemented case; RANDUTV_E_WORKSPACE if the workspace is too small;
 *    RANDUTV_E_SYNC if a cross-workgroup wait exceeded its spin limit;
 *    RANDUTV_E_HIP - (int)hipError for HIP runtime failures.
 *  - Any m, n >= 1 for the factorization (m < n: the last step is the LQ of
 *    the wide block row, the paper's Remark on the case m < n in Section
 *    5.2); the truncated approximation takes m >= n.
 */
#ifndef RANDUTV_H
#define RANDUTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RANDUTV_E_UNSUPPORTED (-900)
#define RANDUTV_E_WORKSPACE (-901)
#define RANDUTV_E_SYNC (-902)
#define RANDUTV_E_HIP (-1000)

/* Arithmetic used for the four thin-matrix products that carry almost all of
 * the flops (sampling Y = (X^T X)^q X^T G, power iteration, and the right and
 * left trailing updates).  The Householder panels, their compact-WY factors,
 * the b x b SVDs and the U, V accumulation always run in FP64, and T, U, V
 * are always stored in FP64.  RANDUTV_FP32: operands rounded to FP32, FP32
 * MFMA with FP32 accumulation.  RANDUTV_BF16X3: each operand split as
 * x ~ hi + lo with hi = bf16(x), lo = bf16(x - hi); products hi*hi + hi*lo
 * + lo*hi on BF16 MFMA with FP32 accumulation.  RANDUTV_BF16X3_FP32: BF16x3
 * for the sampling products (their rounding only perturbs the sampled
 * subspace, never the exactness of A = U T V^T, since the transforms are
 * built from it in FP64) and FP32 for the two trailing updates.
 * RANDUTV_BF16X3_BF16X6: BF16x3 sampling and BF16x6 trailing updates: each
 * operand x32 = fl32(x) split into three bf16 pieces h = bf16(x32),
 * m = bf16(x32 - h), l = bf16(x32 - h - m), and the six products h*h, h*m,
 * m*h, h*l, l*h, m*m on BF16 MFMA with FP32 accumulation (FP32-level
 * accuracy on the BF16 matrix cores). */
typedef enum {
  RANDUTV_FP64 = 0,
  RANDUTV_FP32 = 1,
  RANDUTV_BF16X3 = 2,
  RANDUTV_BF16X3_FP32 = 3,
  RANDUTV_BF16X3_BF16X6 = 4
} randutv_prec;

/* Flags of randutv_factor. */
enum {
  RANDUTV_FORM_U = 1, /* accumulate U (m x m) */
  RANDUTV_FORM_V = 2, /* accumulate V (n x n) */
  RANDUTV_ECON_U = 4, /* with FORM_U: only U's first min(m, n) columns (m x min(m, n)) */
  RANDUTV_ONE_STREAM = 8 /* U and V updated on `stream` itself, no second stream:
                            slower, but every kernel runs alone on the device
                            (for timing single kernels); same results */
};

/* Number of randomized steps of Figure "The algorithm randUTV": steps i
 * (0-based) whose I3 = (i+1)b..m and J3 = (i+1)b..n are both nonempty.
 * Returns -1 for invalid sizes. */
int64_t randutv_random_steps(int64_t m, int64_t n, int64_t b);

/* Columns of the packed Gaussian matrix G: b * randutv_random_steps(). */
int64_t randutv_g_cols(int64_t m, int64_t n, int64_t b);

/* Bytes of device workspace randutv_factor needs for these arguments
 * (written to *bytes).  Returns a status as above.  For the arithmetics
 * with BF16 products this includes two buffers in which each product's
 * thin operand is split into BF16 pieces once (Section 5.4's thin
 * products); a call given only the FP64 workspace size computes the same
 * factorization, splitting the operands inside its product kernels. */
int randutv_workspace_size(int64_t m, int64_t n, int64_t b, int q,
                           int prec, unsigned flags, size_t* bytes);

/*
 * randutv_factor -- blocked randUTV (Figure "The algorithm randUTV", Section
 * 5.2; single step Section 4; the economic final SVD of the Remark in
 * Section 4.4).
 *
 *  1  m, n     rows and columns of A, m, n >= 1.  With m < n the first
 *              steps are as for tall input and the last one takes an LQ of the
 *              block row T(I2, [J2,J3]) (the QR of its transpose), then the SVD
 *              of its lower-triangular factor; T is upper trapezoidal.
 *  2  b        block size, 1 <= b <= 256.  max(m, n) <= 32768.
 *  3  q        power-iteration count, 0 <= q <= 16.
 *  4  T, ldt   in: A (m x n).  out: the middle factor T, upper triangular in
 *              the first k columns, with exact zeros below the diagonal and
 *              off the diagonal inside each diagonal block; the diagonal is
 *              >= 0 and descending within each block.  Columns k..n-1 hold
 *              the unreduced trailing block when the factorization stopped
 *              early.  ldt >= m.
 *  5  G, ldg   packed N(0,1) matrix, m x randutv_g_cols(m,n,b): randomized
 *              step i uses G(0:m-i*b-1, i*b:(i+1)*b-1), i.e. the leading
 *              m - i*b rows of column block i (the paper draws a fresh
 *              m - b(i-1) by b Gaussian matrix each step).  ldg >= m.  May be NULL only
 *              if randutv_g_cols() == 0.
 *  6  U, ldu   out (if flags & RANDUTV_FORM_U): m x m orthogonal U, or with
 *              RANDUTV_ECON_U its first min(m, n) columns (m x min(m, n),
 *              orthonormal): A = U T(0:min(m,n), :) V^T after a full
 *              factorization, and U(:, 0:k) is the left factor of the rank-k
 *              approximation after an early stop at k (Section 1.1, advantage
 *              (ii): O(mnk) storage).  Else may be NULL.  ldu >= m.
 *  7  V, ldv   out (if flags & RANDUTV_FORM_V): n x n orthogonal V.  Else may
 *              be NULL.  ldv >= n.
 *  8  k_stop   > 0: stop after the first step whose column count reaches
 *              k_stop (k = that multiple of b).  <= 0: no limit.
 *  9  tol      > 0: stop after the first step with ||T(I3,J3)||_F <=
 *              tol * ||A||_F (Section 1.1, advantage (ii)); this makes the
 *              call wait on the stream once per step.  <= 0: no test.
 * 10  prec     randutv_prec.
 * 11  flags    RANDUTV_FORM_U | RANDUTV_FORM_V, and RANDUTV_ECON_U with
 *              FORM_U (the economy U is formed after the loop, from the left
 *              reflectors kept in its own columns, by backward accumulation;
 *              the full U by forward accumulation on a second stream, or on
 *              `stream` with RANDUTV_ONE_STREAM).
 * 12  work     device workspace of at least randutv_workspace_size() bytes,
 *              256-byte aligned.  Contents on entry are ignored.
 * 13  work_bytes
 * 14  k_out    host pointer, may be NULL: the number of leading columns
 *              driven to triangular form (min(m,n) unless stopped early).
 *              When non-NULL the call also waits for the stream and then
 *              reports RANDUTV_E_SYNC or 1 (a small SVD did not converge
 *              within its 40-sweep budget); with k_out == NULL and tol <= 0
 *              the call only enqueues, and randutv_status(work, ...) reports
 *              the same statuses and k later.
 * 15  stream
 *
 * The small b x b SVDs of all steps are computed after the main loop and
 * their rotations folded into T, U and V then; left and right
 * multiplications commute, so the result equals the paper's in-loop order.
 */
int randutv_factor(int64_t m, int64_t n, int64_t b, int q,
                   double* T, int64_t ldt,
                   const double* G, int64_t ldg,
                   double* U, int64_t ldu,
                   double* V, int64_t ldv,
                   int64_t k_stop, double tol,
                   int prec, unsigned flags,
                   void* work, size_t work_bytes,
                   int64_t* k_out, void* stream);

/*
 * randutv_status -- status of the last factorization (randutv_factor,
 * randutv_factor_p, randutv_factor_lower) or randomized SVD (randutv_rsvd)
 * enqueued with this workspace: waits for `stream`, then returns 0, 1 (a
 * Jacobi SVD did not converge within its sweep budget), RANDUTV_E_SYNC (a
 * bounded cross-workgroup wait hit its spin limit), or
 * RANDUTV_E_UNSUPPORTED when no such call has completed in this workspace;
 * *k_out (host pointer, may be NULL) receives the number of leading
 * columns reduced (the rank k for randutv_rsvd).  The status words are the
 * first 256 bytes of the workspace, so each concurrent call needs its own
 * workspace.
 *  1  work        the workspace passed to that call (256-byte aligned)
 *  2  work_bytes  at least 256
 *  3  k_out
 *  4  stream      the stream that call was enqueued on
 */
int randutv_status(const void* work, size_t work_bytes, int64_t* k_out, void* stream);

/*
 * randutv_factor_noalloc -- randutv_factor for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments 1..11 as randutv_factor;
 * no workspace argument: the workspace is a 128 MiB device array of the
 * library, one per GPU, held until the process ends.  The call allocates
 * nothing (no hipMalloc, hipFree, stream or event creation); U and V are
 * updated on `stream` itself.  Sizes whose randutv_workspace_size exceeds
 * 128 MiB (for example 4000 x 4000 with b = 128 or 256; 3800 x 3800 with
 * b = 128 fits) return RANDUTV_E_WORKSPACE before any work is enqueued.  All calls
 * on one GPU share its array: calls that overlap in time on one GPU (on
 * different streams or host threads) race; calls on one stream do not.
 * Status through k_out as for randutv_factor (12 k_out, 13 stream).
 */
int randutv_factor_noalloc(int64_t m, int64_t n, int64_t b, int q,
                           double* T, int64_t ldt,
                           const double* G, int64_t ldg,
                           double* U, int64_t ldu,
                           double* V, int64_t ldv,
                           int64_t k_stop, double tol,
                           int prec, unsigned flags,
                           int64_t* k_out, void* stream);

/*
 * randutv_factor_lower -- the same factorization with a lower-triangular
 * middle factor, A = U L V^T (Section 1: the middle factor may be taken
 * upper or lower triangular).  Computed as randutv_factor of A^T
 * (A^T = U' T V'^T, so U = V', L = T^T, V = U'), with A^T formed in the
 * workspace by a tiled transpose and L transposed back into T.
 * Arguments as randutv_factor except:
 *  4  T, ldt   in: A (m x n).  out: L, lower triangular in its first k rows
 *              (exact zeros above the diagonal and off the diagonal inside
 *              each diagonal block; the diagonal >= 0 and descending within
 *              each block).
 *  5  G, ldg   packed N(0,1) matrix of the n x m problem:
 *              n x randutv_g_cols(n, m, b), ldg >= n.
 * 12  work     randutv_workspace_size_lower() bytes.
 * 11  flags    RANDUTV_FORM_U | RANDUTV_FORM_V (no economy form).
 * Statuses as randutv_factor (argument numbers of this call), except that
 * a HIP or numerical status from the inner factorization is passed on.
 */
int randutv_workspace_size_lower(int64_t m, int64_t n, int64_t b, int q,
                                 int prec, unsigned flags, size_t* bytes);
int randutv_factor_lower(int64_t m, int64_t n, int64_t b, int q,
                         double* T, int64_t ldt,
                         const double* G, int64_t ldg,
                         double* U, int64_t ldu,
                         double* V, int64_t ldv,
                         int64_t k_stop, double tol,
                         int prec, unsigned flags,
                         void* work, size_t work_bytes,
                         int64_t* k_out, void* stream);

/*
 * Over-sampled variants (Remark on over-sampling, Section 5.3; Appendix A.2,
 * the over-sampled step): each randomized step draws b + p samples,
 * Y = (X^T X)^q X^T G_i with G_i of b + p columns, and the Householder QR is
 * taken of the b dominant left singular vectors of Y instead of Y itself.
 * Each such vector's sign is fixed by its right singular vector, whose
 * largest-magnitude entry is made positive (the rule of the small SVDs).
 * p = 0 gives randutv_g_cols / randutv_workspace_size / randutv_factor.
 *
 * randutv_g_cols_p: (b + p) * randutv_random_steps(); -1 for invalid sizes.
 *   Randomized step i uses G(0:m-i*b-1, i*(b+p):(i+1)*(b+p)-1).
 * randutv_workspace_size_p: as randutv_workspace_size; status -4 when
 *   p < 0 or b + p > 256 (the later arguments' codes shift by one).
 * randutv_factor_p: arguments and results as randutv_factor with p after b;
 *   0 <= p and b + p <= 256, else status -13.  The SVD of each step's
 *   extended sample runs on the device between the sampling products and
 *   the QR; a non-converged one reports status 1 like a non-converged
 *   small SVD (through k_out or randutv_status).
 */
int64_t randutv_g_cols_p(int64_t m, int64_t n, int64_t b, int64_t p);
int randutv_workspace_size_p(int64_t m, int64_t n, int64_t b, int64_t p, int q,
                             int prec, unsigned flags, size_t* bytes);
int randutv_factor_p(int64_t m, int64_t n, int64_t b, int64_t p, int q,
                     double* T, int64_t ldt,
                     const double* G, int64_t ldg,
                     double* U, int64_t ldu,
                     double* V, int64_t ldv,
                     int64_t k_stop, double tol,
                     int prec, unsigned flags,
                     void* work, size_t work_bytes,
                     int64_t* k_out, void* stream);

/*
 * Randomized SVD on the same kernels (Section 2.5: the range finder and the
 * Remark RSVD, eqs. panda1 and panda2; over-sampling per the Remark on
 * over-sampling): A ~ U diag(D) V^T of rank k.
 *   Y = (A^T A)^q A^T G (G: m x (k+p)), Q = the n x (k+p) orthonormal factor
 *   of Y's unpivoted Householder QR, B = A Q, B = Ub diag(Db) W^T (economic
 *   SVD), U = Ub(:, 0:k), D = Db(0:k), V = Q W(:, 0:k).  Each (u_j, v_j)
 *   has the sign that makes the largest-magnitude entry of w_j positive.
 *   With p = 0 the error A - U D V^T equals A - A Q Q^T exactly (in exact
 *   arithmetic); with p > 0 the rank-(k+p) result is truncated to rank k.
 *
 *  1  m, n     rows and columns of A, max(m, n) <= 32768.
 *  3  k        rank, k >= 1.
 *  4  p        over-sampling, p >= 0, k + p <= min(m, n) and k + p <= 256.
 *  5  q        power-iteration count, 0 <= q <= 16.
 *  6  A, lda   m x n input (device, read only), lda >= m.
 *  8  G, ldg   m x (k+p) N(0,1) matrix (device), ldg >= m.
 * 10  U, ldu   out: m x k, orthonormal columns, ldu >= m.
 * 12  D        out: k singular values, descending, >= 0.
 * 13  V, ldv   out: n x k, orthonormal columns, ldv >= n.
 * 15  prec     randutv_prec: the sampling products and B = A Q take the
 *              arithmetic randutv_factor gives its sampling and update
 *              products; the QRs, the SVD and U, V are FP64.
 * 16  work     randutv_rsvd_workspace_size() bytes of device memory,
 *              256-byte aligned; contents on entry are ignored.
 * 18  sweeps_out  host pointer, may be NULL.  When non-NULL the call waits
 *              for the stream, stores the Jacobi sweeps used and returns 1
 *              if the SVD did not converge (RANDUTV_E_SYNC if a
 *              cross-workgroup wait hit its spin limit); when NULL it only
 *              enqueues, and randutv_status(work, ...) reports later.
 * 19  stream
 * Statuses: -i for argument i; RANDUTV_E_UNSUPPORTED above the size limit;
 * RANDUTV_E_WORKSPACE; RANDUTV_E_HIP - hipError.
 */
int randutv_rsvd_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, int q,
                                int prec, size_t* bytes);
int randutv_rsvd(int64_t m, int64_t n, int64_t k, int64_t p, int q,
                 const double* A, int64_t lda, const double* G, int64_t ldg,
                 double* U, int64_t ldu, double* D, double* V, int64_t ldv,
                 int prec, void* work, size_t work_bytes, int* sweeps_out,
                 void* stream);

/* ---- Building blocks of one step (exported for testing and reuse) ---- */

/* Truncated approximation (Section 6.2, eq. Ak_randUTV; Theorem of Section
 * 5.3): A_k = U_k U_k^T A, with U_k the first k columns of U after t = k / b
 * steps of randUTV on A (m x n, m >= n, m <= 32768), b <= 128, k a multiple
 * of b with 0 < k < n.  The b x b SVDs are skipped: U_k U_k^T does not depend
 * on them.  A (lda), G (packed Gaussian as for randutv_factor, ldg) are read;
 * Uk (m x k, lduk) and, unless Ak == NULL, Ak (m x n, ldak) are written;
 * `tape` (randutv_approx_tape_size bytes, device) receives the reflectors
 * and R factors of the t steps for randutv_approx_backward.  prec as for
 * randutv_factor (argument 16).  work: randutv_approx_work_size bytes,
 * 256-byte aligned.  Enqueued on `stream`; returns without waiting. */
size_t randutv_approx_tape_size(int64_t m, int64_t n, int64_t b, int64_t k);
size_t randutv_approx_work_size(int64_t m, int64_t n, int64_t b, int q, int64_t k);
int randutv_approx(int64_t m, int64_t n, int64_t b, int q, int64_t k, const double* A,
                   int64_t lda, const double* G, int64_t ldg, double* Ak, int64_t ldak,
                   double* Uk, int64_t lduk, double* tape, size_t tape_bytes, int prec,
                   void* work, size_t work_bytes, void* stream);

/* Reverse-mode derivative of A -> A_k with G held fixed: Abar (m x n, ldab)
 * = J^T Akbar, from A, G, the Uk and tape written by randutv_approx on the
 * same arguments (the trailing matrices of every step are recomputed from A
 * and the tape; no dense U or V is stored).  Defined wherever no Householder
 * sign decision of the t steps flips (where A_k is smooth).  prec is
 * argument 18; work: randutv_approx_backward_work_size bytes, 256-byte
 * aligned.  Enqueued on `stream`. */
size_t randutv_approx_backward_work_size(int64_t m, int64_t n, int64_t b, int q, int64_t k);
int randutv_approx_backward(int64_t m, int64_t n, int64_t b, int q, int64_t k, const double* A,
                            int64_t lda, const double* G, int64_t ldg, const double* Uk,
                            int64_t lduk, const double* tape, size_t tape_bytes,
                            const double* Akbar, int64_t ldakb, double* Abar, int64_t ldab,
                            int prec, void* work, size_t work_bytes, void* stream);

/* Thin-matrix product of the sampling and update stages (Section 1.1 (iii);
 * Section 5.4): C = alpha * op(A) * op(B) + beta * C, all FP64 column-major in
 * memory, op(X) = X^T when tX != 0, inner products in `prec` arithmetic.
 * C is M x N, op(A) is M x K, op(B) is K x N.  work (may be NULL) enables a
 * split of long K: any size, used up to 8*M*N doubles.  Arguments 1..12 are
 * validated (-i on error); prec is RANDUTV_FP64, _FP32 or _BF16X3, or 4 for
 * the BF16x6 arithmetic (three bf16 pieces per operand, six products). */
int randutv_gemm(int prec, int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc, void* work, size_t work_bytes, void* stream);

/* Unpivoted Householder QR of a tall panel (Section 2.4, eq. unpivQR) in
 * place, LAPACK dgeqrf layout (R on and above the diagonal, reflector tails
 * below, unit diagonal implied), reflector scalars tau[nb] (dlarfg
 * convention), and the upper triangular compact-WY factor Tw (nb x nb, ld
 * ldtw, zeros below the diagonal) with H_0 H_1 ... H_{nb-1} = I - V Tw V^T
 * (eq. WYrepresentation).  Requires nb <= Mp <= 32768 and nb <= 256.
 * Computed by CholeskyQR2 with Householder reconstruction when the panel is
 * well conditioned, else by column-by-column Householder; *used_fallback
 * (host pointer, may be NULL) reports which (1 = column-by-column).
 * work: at least randutv_panel_work_size(Mp, nb) bytes, 256-byte aligned
 * (-9 otherwise).  Waits for completion. */
size_t randutv_panel_work_size(int64_t Mp, int64_t nb);
int randutv_panel_qr(int64_t Mp, int64_t nb, double* P, int64_t ldp, double* tau, double* Tw,
                     int64_t ldtw, int* used_fallback, void* work, size_t work_bytes,
                     void* stream);

/* SVD of `count` small square blocks (Figure "The algorithm randUTV": the
 * SVD of each step's diagonal block R): matrix i has size nbs[i] (host array, each
 * 1..ld, ld <= 1024) and is read from R + i*ld*ld (leading dimension ld);
 * outputs Us, Vs (same layout) and D + i*ld, singular values descending,
 * each (u_j, v_j) flipped so the largest-magnitude entry of v_j is positive.
 * work: at least randutv_small_svd_work_size(count, ld) bytes.  Waits for
 * completion; returns 1 if some matrix did not converge. */
size_t randutv_small_svd_work_size(int64_t count, int64_t ld);
int randutv_small_svd(int64_t count, const int* nbs, int64_t ld, const double* R, double* Us,
                      double* Vs, double* D, void* work, size_t work_bytes, void* stream);

/* ---- Kernel timing (measurement support) ----
 * randutv_profile_begin() starts recording HIP events on the launch stream
 * around each thin GEMM, split-K reduction, panel QR and small-SVD launch of
 * later calls; randutv_profile_end() waits for them and fills, per kernel
 * class c < max_classes (names from randutv_profile_class_name(c)), the
 * summed milliseconds, algorithmic flops (2*M*N*K per GEMM), algorithmic
 * bytes (each operand read once and the output written once, 8 bytes per
 * element: 8*(M*K + K*N + M*N) per GEMM, plus 8*M*N when beta != 0; a
 * split-K reduction 8*(splits+1)*M*N, plus 8*M*N when beta != 0; a panel QR
 * 16*Mp*nb; 0 for the small SVDs) and launch counts.  Any of ms, flops,
 * bytes, launches may be NULL.  Returns the number of classes filled, or a
 * negative status.  Not thread-safe; meant for one process-wide measurement
 * at a time.  randutv_profile_begin_class(c) records events around launches
 * of class c only (c < 0: all classes, as randutv_profile_begin), so that
 * a timed run carries the events of the one kernel it measures; returns -1
 * for c beyond the last class. */
int randutv_profile_begin(void);
int randutv_profile_begin_class(int cls);
int randutv_profile_end(int max_classes, double* ms, double* flops, double* bytes,
                        int64_t* launches);
const char* randutv_profile_class_name(int cls);

/* Short text for a status code (static storage). */
const char* randutv_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* RANDUTV_H */
