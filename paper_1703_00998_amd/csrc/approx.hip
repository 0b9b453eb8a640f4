// Truncated approximation A_k = U_k U_k^T A from the first t = k / b steps
// of randUTV (Section 6.2, eq. Ak_randUTV; the Theorem of Section 5.3), and
// its reverse-mode derivative with the Gaussian G held fixed.
//
// Forward.  The steps run with their reflectors kept on a tape; U_k is
// accumulated backwards from [I_k; 0] through the left block reflectors
// (U_k U_k^T does not depend on the b x b rotations of the small SVDs, which
// only mix columns inside a block, so those are skipped).
//
// Backward.  Only A, G, U_k and the tape are kept: the trailing matrices X_i
// of every step are recomputed from A with the taped reflectors, then the
// steps are reversed.  Per step the forward is
//   Y = (X^T X)^q X^T G_i;  (Vy, Ty) = House(Y);  X1 = X (I - Vy Ty Vy^T);
//   (Vu, Tu) = House(X1(:, 0:b));  X2 = (I - Vu Tu Vu^T)^T X1(:, b:);
//   X_{i+1} = X2(b:, :),
// and every product is reversed by the usual GEMM adjoints.  House (the map
// from a tall panel to its Householder vectors V and compact-WY factor T) is
// reversed through the reconstruction that defines it: thin QR P = Q R
// (positive diagonal), the LU Q - [S; 0] = L U, V = L, T = -U S L1^-T.  With
// adjoints Vbar, Tbar:
//   Ubar = -Tbar L1^-1 S,  L1bar += L1^-T Tbar^T U S L1^-T   (strict lower),
//   tall LU: B2bar = L2bar U^-T,  Ubar -= L2^T B2bar,
//            B1bar = L1^-T (stril(L1^T L1bar) + triu(Ubar U^T)) U^-T,
//   thin QR (R unused): M = -Qbar^T Q,  Pbar = (Qbar + Q copyltu(M)) R^-T,
// where Qbar = Bbar, copyltu(M) = tril(M) + tril(M, -1)^T, and S, R, U, Q
// are rebuilt from the taped V, T and Householder R: S = sign(diag R_h),
// R = S R_h, U = -T L1^T S, Q = ([I; 0] - V T L1^T) S.  Valid wherever no
// Householder sign decision flips (the map is smooth there).
#include <algorithm>

#include "../../include/randutv.h"
#include "common.h"

namespace rutv {
namespace {

enum EwOp {
  EW_STRIL = 0,       // Y = strictly lower part of X (trapezoidal), zeros elsewhere
  EW_TRIU = 1,        // Y = upper part of X (with the diagonal)
  EW_COPYLTU = 2,     // Y(i,j) = X(max(i,j), min(i,j))          (square)
  EW_SCALE_COLS = 3,  // Y(:,j) = alpha * s_j * X(:,j)
  EW_SCALE_ROWS_TRIU = 4,  // Y(i,j) = s_i X(i,j) for i <= j, else 0
  EW_ADD_STRIL = 5,   // Y += strictly lower part of X
  EW_ADD_TRIU = 6,    // Y += upper part of X
  EW_ADD_EYE = 7,     // Y(i,i) += 1 for i < min(rows, cols)
  EW_COPY = 8,        // Y = alpha * X
  EW_ADD = 9          // Y += alpha * X
};

__global__ void k_ew(int op, int rows, int cols, const double* __restrict__ X, int64_t ldx,
                     double* __restrict__ Y, int64_t ldy, const double* __restrict__ s,
                     double alpha) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % rows), j = (int)(idx / rows);
    double* y = Y + i + (int64_t)j * ldy;
    switch (op) {
      case EW_STRIL: *y = i > j ? X[i + (int64_t)j * ldx] : 0.0; break;
      case EW_TRIU: *y = i <= j ? X[i + (int64_t)j * ldx] : 0.0; break;
      case EW_COPYLTU:
        *y = i >= j ? X[i + (int64_t)j * ldx] : X[j + (int64_t)i * ldx];
        break;
      case EW_SCALE_COLS: *y = alpha * s[j] * X[i + (int64_t)j * ldx]; break;
      case EW_SCALE_ROWS_TRIU: *y = i <= j ? s[i] * X[i + (int64_t)j * ldx] : 0.0; break;
      case EW_ADD_STRIL:
        if (i > j) *y += X[i + (int64_t)j * ldx];
        break;
      case EW_ADD_TRIU:
        if (i <= j) *y += X[i + (int64_t)j * ldx];
        break;
      case EW_ADD_EYE:
        if (i == j) *y += 1.0;
        break;
      case EW_ADD: *y += alpha * X[i + (int64_t)j * ldx]; break;
      default: *y = alpha * X[i + (int64_t)j * ldx]; break;
    }
  }
}

// s_j = sign(R(j, j)), sign(0) = +1.
__global__ void k_sign_diag(int b, const double* __restrict__ R, int64_t ldr, double* __restrict__ s) {
  for (int j = threadIdx.x; j < b; j += blockDim.x) s[j] = R[j + (int64_t)j * ldr] < 0.0 ? -1.0 : 1.0;
}

hipError_t ew(hipStream_t st, int op, int rows, int cols, const double* X, int64_t ldx, double* Y,
              int64_t ldy, const double* s = nullptr, double alpha = 1.0) {
  const int64_t total = (int64_t)rows * cols;
  if (total <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(k_ew, dim3(blocks), dim3(256), 0, st, op, rows, cols, X, ldx, Y, ldy, s, alpha);
  return hipGetLastError();
}

#define AX_CHK(x)                           \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

// FP64 product with split-K scratch, C = alpha op(A) op(B) + beta C.
struct Mul {
  hipStream_t st;
  Prec prec;
  double* split;
  size_t se;
  hipError_t operator()(bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
                        int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                        int64_t ldc, bool low = false) const {
    return gemm(st, low ? prec : PREC_FP64, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                split, se);
  }
};

// Scratch of one House reversal for panels of up to Mmax rows, b columns.
struct HouseWork {
  double *s, *R, *Uu, *US, *Wt, *L1i, *Ui, *Ri, *Tb, *Ub, *a, *a2, *c1, *c2, *Mm, *cl;  // b x b
  double *Q, *Lb, *Bb, *Pb;  // Mmax x b
};

size_t house_work_doubles(int64_t Mmax, int64_t b) { return 16 * b * b + 4 * Mmax * b; }

void house_work_carve(double* p, int64_t Mmax, int64_t b, HouseWork* w) {
  double** sq[] = {&w->s,  &w->R,  &w->Uu, &w->US, &w->Wt, &w->L1i, &w->Ui, &w->Ri,
                   &w->Tb, &w->Ub, &w->a,  &w->a2, &w->c1, &w->c2,  &w->Mm, &w->cl};
  for (double** q : sq) {
    *q = p;
    p += b * b;
  }
  double** tall[] = {&w->Q, &w->Lb, &w->Bb, &w->Pb};
  for (double** q : tall) {
    *q = p;
    p += Mmax * b;
  }
}

// Pbar (M x b, ld ldp) = adjoint of the panel P given the adjoints of its
// Householder vectors V (M x b, explicit unit lower trapezoidal) and of its
// compact-WY factor T, from the taped V, T and Householder R factor Rh.
hipError_t house_vjp(const Mul& mul, int M, int b, const double* V, int64_t ldv, const double* T,
                     const double* Rh, const double* Vbar, int64_t ldvb, const double* Tbar,
                     double* Pbar, int64_t ldp, const HouseWork& w) {
  hipStream_t st = mul.st;
  const int64_t bb = b, lM = M;
  hipLaunchKernelGGL(k_sign_diag, dim3(1), dim3(256), 0, st, b, Rh, bb, w.s);
  AX_CHK(ew(st, EW_SCALE_ROWS_TRIU, b, b, Rh, bb, w.R, bb, w.s));          // R = S Rh
  AX_CHK(mul(false, true, b, b, b, 1.0, T, bb, V, ldv, 0.0, w.Wt, bb));     // Wt = T L1^T
  AX_CHK(ew(st, EW_SCALE_COLS, b, b, w.Wt, bb, w.Uu, bb, w.s, -1.0));       // U = -Wt S
  AX_CHK(ew(st, EW_SCALE_COLS, b, b, w.Uu, bb, w.US, bb, w.s, 1.0));        // U S
  AX_CHK(mul(false, false, M, b, b, -1.0, V, ldv, w.Wt, bb, 0.0, w.Pb, lM)); // -V Wt
  AX_CHK(ew(st, EW_ADD_EYE, b, b, nullptr, 0, w.Pb, lM));
  AX_CHK(ew(st, EW_SCALE_COLS, M, b, w.Pb, lM, w.Q, lM, w.s, 1.0));         // Q
  AX_CHK(tri_inv(st, b, V, ldv, w.L1i, bb, false));
  AX_CHK(tri_inv(st, b, w.Uu, bb, w.Ui, bb, true));
  AX_CHK(tri_inv(st, b, w.R, bb, w.Ri, bb, true));
  AX_CHK(ew(st, EW_TRIU, b, b, Tbar, bb, w.Tb, bb));
  AX_CHK(ew(st, EW_STRIL, M, b, Vbar, ldvb, w.Lb, lM));
  // Ubar = -Tbar L1^-1 S
  AX_CHK(mul(false, false, b, b, b, 1.0, w.Tb, bb, w.L1i, bb, 0.0, w.a, bb));
  AX_CHK(ew(st, EW_SCALE_COLS, b, b, w.a, bb, w.Ub, bb, w.s, -1.0));
  // L1bar += stril(L1^-T Tbar^T (U S) L1^-T)
  AX_CHK(mul(true, true, b, b, b, 1.0, w.L1i, bb, w.Tb, bb, 0.0, w.a, bb));
  AX_CHK(mul(false, false, b, b, b, 1.0, w.a, bb, w.US, bb, 0.0, w.a2, bb));
  AX_CHK(mul(false, true, b, b, b, 1.0, w.a2, bb, w.L1i, bb, 0.0, w.a, bb));
  AX_CHK(ew(st, EW_ADD_STRIL, b, b, w.a, bb, w.Lb, lM));
  // tall part: B2bar = L2bar U^-T; Ubar -= L2^T B2bar
  if (M > b) {
    AX_CHK(mul(false, true, M - b, b, b, 1.0, w.Lb + b, lM, w.Ui, bb, 0.0, w.Bb + b, lM));
    AX_CHK(mul(true, false, b, b, M - b, -1.0, V + b, ldv, w.Bb + b, lM, 1.0, w.Ub, bb));
  }
  // B1bar = L1^-T (stril(L1^T L1bar) + triu(Ubar U^T)) U^-T
  AX_CHK(mul(true, false, b, b, b, 1.0, V, ldv, w.Lb, lM, 0.0, w.c1, bb));
  AX_CHK(ew(st, EW_STRIL, b, b, w.c1, bb, w.c2, bb));
  AX_CHK(mul(false, true, b, b, b, 1.0, w.Ub, bb, w.Uu, bb, 0.0, w.c1, bb));
  AX_CHK(ew(st, EW_ADD_TRIU, b, b, w.c1, bb, w.c2, bb));
  AX_CHK(mul(true, false, b, b, b, 1.0, w.L1i, bb, w.c2, bb, 0.0, w.c1, bb));
  AX_CHK(mul(false, true, b, b, b, 1.0, w.c1, bb, w.Ui, bb, 0.0, w.Bb, lM));
  // thin QR: M = -Qbar^T Q, Pbar = (Qbar + Q copyltu(M)) R^-T, Qbar = Bbar
  AX_CHK(mul(true, false, b, b, M, -1.0, w.Bb, lM, w.Q, lM, 0.0, w.Mm, bb));
  AX_CHK(ew(st, EW_COPYLTU, b, b, w.Mm, bb, w.cl, bb));
  AX_CHK(mul(false, false, M, b, b, 1.0, w.Q, lM, w.cl, bb, 1.0, w.Bb, lM));
  AX_CHK(mul(false, true, M, b, b, 1.0, w.Bb, lM, w.Ri, bb, 0.0, Pbar, ldp));
  return hipGetLastError();
}

// Y (rows x cols, ld ldy) <- (I - V T V^T) Y, or the transpose when trans.
hipError_t apply_block(const Mul& mul, bool trans, int rows, int cols, int b, const double* V,
                       int64_t ldv, const double* T, double* Y, int64_t ldy, double* w1,
                       double* w2) {
  const int64_t bb = b;
  AX_CHK(mul(true, false, b, cols, rows, 1.0, V, ldv, Y, ldy, 0.0, w1, bb));
  AX_CHK(mul(trans, false, b, cols, b, 1.0, T, bb, w1, bb, 0.0, w2, bb));
  return mul(false, false, rows, cols, b, -1.0, V, ldv, w2, bb, 1.0, Y, ldy);
}

struct ApproxLayout {
  size_t factor, T, tmp, total;
};

ApproxLayout approx_layout(int64_t m, int64_t n, int64_t b, int64_t k) {
  ApproxLayout L{};
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  L.factor = off;
  off = al(off + factor_work_bytes(m, n, b));
  L.T = off;
  off = al(off + (size_t)m * n * sizeof(double));
  L.tmp = off;
  off = al(off + (size_t)std::max(k, b) * std::max(m, n) * 2 * sizeof(double));
  L.total = off;
  return L;
}

struct BackLayout {
  size_t Xs, X1, X1b, Xb, Ys, Zs, W, W2, Wb, W2b, C, C2, Cb, C2b, Vyb, Vub, Tyb, Tub, VubS, TubS,
      F, Fb, Ukb, t1, t2, hw, split, total;
  size_t split_elems;
};

BackLayout back_layout(int64_t m, int64_t n, int64_t b, int q, int64_t k) {
  BackLayout L{};
  const int64_t t = k / b, mx = std::max(m, n);
  const size_t d = sizeof(double);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  L.Xs = take((size_t)std::max<int64_t>(t - 1, 1) * m * n * d);
  L.X1 = take((size_t)m * n * d);
  L.X1b = take((size_t)m * n * d);
  L.Xb = take((size_t)m * n * d);
  L.Ys = take((size_t)(q + 1) * n * b * d);
  L.Zs = take((size_t)std::max(q, 1) * m * b * d);
  L.W = take((size_t)m * b * d);
  L.W2 = take((size_t)m * b * d);
  L.Wb = take((size_t)m * b * d);
  L.W2b = take((size_t)m * b * d);
  L.C = take((size_t)b * n * d);
  L.C2 = take((size_t)b * n * d);
  L.Cb = take((size_t)b * n * d);
  L.C2b = take((size_t)b * n * d);
  L.Vyb = take((size_t)n * b * d);
  L.Vub = take((size_t)m * b * d);
  L.Tyb = take((size_t)b * b * d);
  L.Tub = take((size_t)b * b * d);
  L.VubS = take((size_t)t * m * b * d);
  L.TubS = take((size_t)t * b * b * d);
  L.F = take((size_t)m * k * d);
  L.Fb = take((size_t)m * k * d);
  L.Ukb = take((size_t)m * k * d);
  L.t1 = take((size_t)mx * std::max(k, b) * d);
  L.t2 = take((size_t)mx * std::max(k, b) * d);
  L.hw = take(house_work_doubles(mx, b) * d);
  L.split_elems = (size_t)kMaxSplitK * mx * std::max(k, b);
  L.split = take(L.split_elems * d);
  L.total = off;
  return L;
}

int check_approx_args(int64_t m, int64_t n, int64_t b, int q, int64_t k) {
  if (m < 1 || n < 1) return -1;
  if (m < n || m > ((int64_t)1 << 15)) return RANDUTV_E_UNSUPPORTED;
  if (b < 1 || b > 128) return -3;
  if (q < 0 || q > 16) return -4;
  if (k < b || k % b != 0 || k >= n) return -5;
  return 0;
}

}  // namespace
}  // namespace rutv

using namespace rutv;

#define HIPRET(x)                                                 \
  do {                                                            \
    hipError_t e_ = (x);                                          \
    if (e_ != hipSuccess) return RANDUTV_E_HIP - (int)e_;         \
  } while (0)

extern "C" {

size_t randutv_approx_tape_size(int64_t m, int64_t n, int64_t b, int64_t k) {
  if (m < 1 || n < 1 || b < 1 || k < b || k % b) return 0;
  return ApproxTape::bytes(m, n, b, k / b);
}

size_t randutv_approx_work_size(int64_t m, int64_t n, int64_t b, int q, int64_t k) {
  if (check_approx_args(m, n, b, q, k) != 0) return 0;
  return approx_layout(m, n, b, k).total;
}

size_t randutv_approx_backward_work_size(int64_t m, int64_t n, int64_t b, int q, int64_t k) {
  if (check_approx_args(m, n, b, q, k) != 0) return 0;
  return back_layout(m, n, b, q, k).total;
}

int randutv_approx(int64_t m, int64_t n, int64_t b, int q, int64_t k, const double* A,
                   int64_t lda, const double* G, int64_t ldg, double* Ak, int64_t ldak,
                   double* Uk, int64_t lduk, double* tape, size_t tape_bytes, int prec,
                   void* work, size_t work_bytes, void* stream) {
  const int bad = check_approx_args(m, n, b, q, k);
  if (bad) return bad;
  if (!A || lda < m) return -6;
  if (!G || ldg < m) return -8;
  if (Ak && ldak < m) return -11;
  if (!Uk || lduk < m) return -12;
  if (!tape || tape_bytes < randutv_approx_tape_size(m, n, b, k)) return -14;
  if (prec < 0 || prec > kPrecMax) return -16;
  const ApproxLayout L = approx_layout(m, n, b, k);
  if (!work || ((uintptr_t)work & 255) || work_bytes < L.total) return RANDUTV_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)work;
  double* T = (double*)(base + L.T);
  double* tmp = (double*)(base + L.tmp);
  const int M = (int)m, N = (int)n, B = (int)b, K = (int)k, t = (int)(k / b);
  const ApproxTape tp{tape, m, n, b, t};
  HIPRET(copy_matrix(st, M, N, A, lda, T, M));
  const int r = factor_impl(m, n, b, q, T, m, G, ldg, nullptr, 1, nullptr, 1, k, 0.0, prec, 0,
                            base + L.factor, factor_work_bytes(m, n, b), nullptr, stream, &tp);
  if (r != 0) return r;
  // U_k = H_1 (I + H_2) ... [I_k; 0], accumulated from the last step back.
  const Mul mul{st, PREC_FP64, nullptr, 0};
  HIPRET(set_identity(st, M, K, Uk, lduk));
  double* w1 = tmp;
  double* w2 = tmp + (size_t)b * std::max(k, b);
  for (int i = t - 1; i >= 0; --i) {
    const int r0 = i * B;
    HIPRET(apply_block(mul, false, M - r0, K, B, tp.Vu(i), m, tp.Tu(i), Uk + r0, lduk, w1, w2));
  }
  if (Ak) {  // A_k = U_k (U_k^T A)
    HIPRET(gemm(st, PREC_FP64, true, false, K, N, M, 1.0, Uk, lduk, A, lda, 0.0, tmp, K, nullptr, 0));
    HIPRET(gemm(st, PREC_FP64, false, false, M, N, K, 1.0, Uk, lduk, tmp, K, 0.0, Ak, ldak, nullptr, 0));
  }
  return 0;
}

int randutv_approx_backward(int64_t m, int64_t n, int64_t b, int q, int64_t k, const double* A,
                            int64_t lda, const double* G, int64_t ldg, const double* Uk,
                            int64_t lduk, const double* tape, size_t tape_bytes,
                            const double* Akbar, int64_t ldakb, double* Abar, int64_t ldab,
                            int prec, void* work, size_t work_bytes, void* stream) {
  const int bad = check_approx_args(m, n, b, q, k);
  if (bad) return bad;
  if (!A || lda < m) return -6;
  if (!G || ldg < m) return -8;
  if (!Uk || lduk < m) return -10;
  if (!tape || tape_bytes < randutv_approx_tape_size(m, n, b, k)) return -12;
  if (!Akbar || ldakb < m) return -14;
  if (!Abar || ldab < m) return -16;
  if (prec < 0 || prec > kPrecMax) return -18;
  const BackLayout L = back_layout(m, n, b, q, k);
  if (!work || ((uintptr_t)work & 255) || work_bytes < L.total) return RANDUTV_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)work;
  auto dp = [&](size_t off) { return (double*)(base + off); };
  const int M = (int)m, N = (int)n, B = (int)b, K = (int)k, t = (int)(k / b);
  const int64_t lm = m, ln = n, lb = b;
  const ApproxTape tp{const_cast<double*>(tape), m, n, b, t};
  // Arithmetic of the products with the m x n trailing matrices (as in the
  // forward: sampling in ps, updates in pu); everything else in FP64.
  const Prec ps = sampling_prec(prec);
  const Prec pu = update_prec(prec);
  double* split = dp(L.split);
  const Mul mul{st, pu, split, L.split_elems};
  const Mul mls{st, ps, split, L.split_elems};
  HouseWork hw;
  house_work_carve(dp(L.hw), std::max(m, n), b, &hw);
  double *X1 = dp(L.X1), *X1b = dp(L.X1b), *Xb = dp(L.Xb), *Ys = dp(L.Ys), *Zs = dp(L.Zs),
         *W = dp(L.W), *W2 = dp(L.W2), *Wb = dp(L.Wb), *W2b = dp(L.W2b), *C = dp(L.C),
         *C2 = dp(L.C2), *Cb = dp(L.Cb), *C2b = dp(L.C2b), *Vyb = dp(L.Vyb), *Vub = dp(L.Vub),
         *Tyb = dp(L.Tyb), *Tub = dp(L.Tub), *F = dp(L.F), *Fb = dp(L.Fb), *Ukb = dp(L.Ukb),
         *t1 = dp(L.t1), *t2 = dp(L.t2);
  // X_i for i >= 1 (leading dimension m), recomputed from A and the tape.
  auto Xs = [&](int i) -> const double* { return i == 0 ? A : dp(L.Xs) + (size_t)(i - 1) * m * n; };
  auto ldX = [&](int i) -> int64_t { return i == 0 ? lda : lm; };
  for (int i = 0; i + 1 < t; ++i) {
    const int r0 = i * B, Mi = M - r0, Ni = N - r0;
    const double* X = Xs(i);
    // X1 = X (I - Vy Ty Vy^T); X2 = (I - Vu Tu Vu^T)^T X1(:, b:)
    HIPRET(mul(false, false, Mi, B, Ni, 1.0, X, ldX(i), tp.Vy(i), ln, 0.0, W, lm, true));
    HIPRET(mul(false, false, Mi, B, B, 1.0, W, lm, tp.Ty(i), lb, 0.0, W2, lm));
    HIPRET(copy_matrix(st, Mi, Ni, X, ldX(i), X1, lm));
    HIPRET(mul(false, true, Mi, Ni, B, -1.0, W2, lm, tp.Vy(i), ln, 1.0, X1, lm, true));
    HIPRET(apply_block(mul, true, Mi, Ni - B, B, tp.Vu(i), lm, tp.Tu(i), X1 + (size_t)B * m,
                       lm, C, C2));
    HIPRET(copy_matrix(st, Mi - B, Ni - B, X1 + B + (size_t)B * m, lm, dp(L.Xs) + (size_t)i * m * n, lm));
  }
  // Direct term and the adjoint of U_k: Abar = U_k U_k^T Akbar,
  // Ukbar = Akbar (A^T U_k) + A (Akbar^T U_k).
  HIPRET(gemm(st, PREC_FP64, true, false, K, N, M, 1.0, Uk, lduk, Akbar, ldakb, 0.0, t1, K, split, L.split_elems));
  HIPRET(gemm(st, PREC_FP64, false, false, M, N, K, 1.0, Uk, lduk, t1, K, 0.0, Abar, ldab, nullptr, 0));
  HIPRET(gemm(st, PREC_FP64, true, false, N, K, M, 1.0, A, lda, Uk, lduk, 0.0, t1, ln, split, L.split_elems));
  HIPRET(gemm(st, PREC_FP64, false, false, M, K, N, 1.0, Akbar, ldakb, t1, ln, 0.0, Ukb, lm, nullptr, 0));
  HIPRET(gemm(st, PREC_FP64, true, false, N, K, M, 1.0, Akbar, ldakb, Uk, lduk, 0.0, t1, ln, split, L.split_elems));
  HIPRET(gemm(st, PREC_FP64, false, false, M, K, N, 1.0, A, lda, t1, ln, 1.0, Ukb, lm, nullptr, 0));
  // Reverse of U_k = F_0, F_i = (I + H_i) F_{i+1} (H_i on rows r0:), i = 0..t-1.
  // With X = F_{i+1}(r0:, :) = H_i^T F_i(r0:, :) and Yb = Fbar_i(r0:, :):
  //   Vbar_i = -(Yb (X^T V) T^T + X (Yb^T V) T),  Tbar_i = -(V^T Yb)(X^T V),
  //   Fbar_{i+1}(r0:, :) = H_i^T Yb.
  HIPRET(copy_matrix(st, M, K, Uk, lduk, F, lm));
  HIPRET(copy_matrix(st, M, K, Ukb, lm, Fb, lm));
  const Mul m64{st, PREC_FP64, split, L.split_elems};
  double* VubS = dp(L.VubS);
  double* TubS = dp(L.TubS);
  for (int i = 0; i < t; ++i) {
    const int r0 = i * B, Mi = M - r0;
    const double* Vu = tp.Vu(i);
    const double* Tu = tp.Tu(i);
    double* Xv = F + r0;
    double* Yb = Fb + r0;
    double* vb = VubS + (size_t)i * m * b;
    double* tb = TubS + (size_t)i * b * b;
    HIPRET(apply_block(m64, true, Mi, K, B, Vu, lm, Tu, Xv, lm, t1, t1 + (size_t)b * k));
    double* XtV = C;   // k x b
    double* YtV = C2;  // k x b
    HIPRET(m64(true, false, K, B, Mi, 1.0, Xv, lm, Vu, lm, 0.0, XtV, K));
    HIPRET(m64(true, false, K, B, Mi, 1.0, Yb, lm, Vu, lm, 0.0, YtV, K));
    HIPRET(m64(false, true, K, B, B, 1.0, XtV, K, Tu, lb, 0.0, Cb, K));
    HIPRET(m64(false, false, Mi, B, K, -1.0, Yb, lm, Cb, K, 0.0, vb, lm));
    HIPRET(m64(false, false, K, B, B, 1.0, YtV, K, Tu, lb, 0.0, Cb, K));
    HIPRET(m64(false, false, Mi, B, K, -1.0, Xv, lm, Cb, K, 1.0, vb, lm));
    HIPRET(m64(true, false, B, B, K, -1.0, YtV, K, XtV, K, 0.0, tb, lb));
    HIPRET(apply_block(m64, true, Mi, K, B, Vu, lm, Tu, Yb, lm, t1, t1 + (size_t)b * k));
  }
  // Reverse of the steps, last to first.  Xb carries Xbar_{i+1}.
  for (int i = t - 1; i >= 0; --i) {
    const int r0 = i * B, Mi = M - r0, Ni = N - r0, Nr = Ni - B;
    const double* X = Xs(i);
    const int64_t ldx = ldX(i);
    const double* Gi = G + (int64_t)i * b * ldg;
    const double* Vy = tp.Vy(i);
    const double* Ty = tp.Ty(i);
    const double* Vu = tp.Vu(i);
    const double* Tu = tp.Tu(i);
    // recompute the step's intermediates
    HIPRET(mls(true, false, Ni, B, Mi, 1.0, X, ldx, Gi, ldg, 0.0, Ys, ln, true));
    for (int j = 0; j < q; ++j) {
      HIPRET(mls(false, false, Mi, B, Ni, 1.0, X, ldx, Ys + (size_t)j * n * b, ln, 0.0,
                 Zs + (size_t)j * m * b, lm, true));
      HIPRET(mls(true, false, Ni, B, Mi, 1.0, X, ldx, Zs + (size_t)j * m * b, lm, 0.0,
                 Ys + (size_t)(j + 1) * n * b, ln, true));
    }
    HIPRET(mul(false, false, Mi, B, Ni, 1.0, X, ldx, Vy, ln, 0.0, W, lm, true));
    HIPRET(m64(false, false, Mi, B, B, 1.0, W, lm, Ty, lb, 0.0, W2, lm));
    HIPRET(copy_matrix(st, Mi, Ni, X, ldx, X1, lm));
    HIPRET(mul(false, true, Mi, Ni, B, -1.0, W2, lm, Vy, ln, 1.0, X1, lm, true));
    double* X1r = X1 + (size_t)B * m;  // X1(:, b:)
    HIPRET(mul(true, false, B, Nr, Mi, 1.0, Vu, lm, X1r, lm, 0.0, C, lb, true));
    HIPRET(m64(true, false, B, Nr, B, 1.0, Tu, lb, C, lb, 0.0, C2, lb));
    // X2bar = [0; Xbar_{i+1}] in X1b(:, b:)
    double* X1br = X1b + (size_t)B * m;
    HIPRET(set_zero(st, Mi, Nr, X1br, lm));
    if (i + 1 < t) HIPRET(copy_matrix(st, Mi - B, Nr, Xb, lm, X1br + B, lm));
    HIPRET(copy_matrix(st, Mi, B, VubS + (size_t)i * m * b, lm, Vub, lm));
    HIPRET(copy_matrix(st, B, B, TubS + (size_t)i * b * b, lb, Tub, lb));
    // X2 = X1(:, b:) - Vu C2, C2 = Tu^T C, C = Vu^T X1(:, b:)
    HIPRET(mul(true, false, B, Nr, Mi, -1.0, Vu, lm, X1br, lm, 0.0, C2b, lb, true));
    HIPRET(m64(false, true, Mi, B, Nr, -1.0, X1br, lm, C2, lb, 1.0, Vub, lm));
    HIPRET(m64(false, false, B, Nr, B, 1.0, Tu, lb, C2b, lb, 0.0, Cb, lb));
    HIPRET(m64(false, true, B, B, Nr, 1.0, C, lb, C2b, lb, 1.0, Tub, lb));
    HIPRET(m64(false, true, Mi, B, Nr, 1.0, X1r, lm, Cb, lb, 1.0, Vub, lm));
    HIPRET(mul(false, false, Mi, Nr, B, 1.0, Vu, lm, Cb, lb, 1.0, X1br, lm, true));
    // (Vu, Tu) = House(X1(:, 0:b))
    HIPRET(house_vjp(m64, Mi, B, Vu, lm, Tu, tp.Ru(i), Vub, lm, Tub, X1b, lm, hw));
    // X1 = X - W2 Vy^T, W2 = W Ty, W = X Vy
    HIPRET(copy_matrix(st, Mi, Ni, X1b, lm, Xb, lm));
    HIPRET(mul(false, false, Mi, B, Ni, -1.0, X1b, lm, Vy, ln, 0.0, W2b, lm, true));
    HIPRET(mul(true, false, Ni, B, Mi, -1.0, X1b, lm, W2, lm, 0.0, Vyb, ln, true));
    HIPRET(m64(false, true, Mi, B, B, 1.0, W2b, lm, Ty, lb, 0.0, Wb, lm));
    HIPRET(m64(true, false, B, B, Mi, 1.0, W, lm, W2b, lm, 0.0, Tyb, lb));
    HIPRET(mul(false, true, Mi, Ni, B, 1.0, Wb, lm, Vy, ln, 1.0, Xb, lm, true));
    HIPRET(mul(true, false, Ni, B, Mi, 1.0, X, ldx, Wb, lm, 1.0, Vyb, ln, true));
    // (Vy, Ty) = House(Y)
    double* Yb = t1;  // Ni x b, ld n
    HIPRET(house_vjp(m64, Ni, B, Vy, ln, Ty, tp.Ry(i), Vyb, ln, Tyb, Yb, ln, hw));
    // sampling: Y_{j+1} = X^T Z_j, Z_j = X Y_j, Y_0 = X^T G_i
    double* Zb = t2;  // Mi x b, ld m
    for (int j = q - 1; j >= 0; --j) {
      HIPRET(mls(false, true, Mi, Ni, B, 1.0, Zs + (size_t)j * m * b, lm, Yb, ln, 1.0, Xb, lm, true));
      HIPRET(mls(false, false, Mi, B, Ni, 1.0, X, ldx, Yb, ln, 0.0, Zb, lm, true));
      HIPRET(mls(false, true, Mi, Ni, B, 1.0, Zb, lm, Ys + (size_t)j * n * b, ln, 1.0, Xb, lm, true));
      HIPRET(mls(true, false, Ni, B, Mi, 1.0, X, ldx, Zb, lm, 0.0, Yb, ln, true));
    }
    HIPRET(mls(false, true, Mi, Ni, B, 1.0, Gi, ldg, Yb, ln, 1.0, Xb, lm, true));
  }
  HIPRET(ew(st, EW_ADD, M, N, Xb, lm, Abar, ldab, nullptr, 1.0));  // Abar += Xbar_0
  return 0;
}

}  // extern "C"
