// Randomized SVD (Section 2.5: the range finder and the Remark RSVD, eqs.
// panda1 and panda2; over-sampling as in the Remark on over-sampling) on
// the kernels of randUTV's step:
//   Y = (A^T A)^q A^T G                  (thin MFMA GEMMs, b + p columns)
//   Y = Q_Y R_Y, Householder             (panel QR; Q formed explicitly)
//   B = A Q                              (thin GEMM)
//   B = Q_B R_B, Householder; R_B = U_R D W^T (one-matrix Jacobi SVD)
//   U = Q_B U_R(:, 0:k),  V = Q W(:, 0:k),  D(0:k)
// The SVD of B is taken through its QR: B = (Q_B U_R) D W^T, so W are B's
// right singular vectors and the Jacobi kernel's sign rule (largest |entry|
// of each right vector positive) applies to them.
#include <algorithm>

#include "../../include/randutv.h"
#include "common.h"

using namespace rutv;

namespace {

constexpr int kMaxC = 256;  // k + p: one panel and one Jacobi block
constexpr int kMaxRows = kPanelMaxWGGlobal * kPanelMaxRows;
constexpr int kSweeps = 40;  // Jacobi sweep budget

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct RsvdLayout {
  size_t status, Y, Z, VY, Q, B, VB, TwY, TwB, RB, Cq, UR, VR, Jw, Jv, Dw, C1, C2, tauY, tauB, ints,
      panel, hr, split, total;
  size_t split_elems;
};

RsvdLayout rsvd_layout(int64_t m, int64_t n, int64_t k, int64_t c) {
  RsvdLayout L{};
  const size_t d = sizeof(double), cc = (size_t)c * c;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = al256(off + bytes);
    return o;
  };
  L.status = take(kStatusBytes);  // first: randutv_status reads it at offset 0
  L.Y = take((size_t)n * c * d);
  L.Z = take((size_t)m * c * d);
  L.VY = take((size_t)n * c * d);
  L.Q = take((size_t)n * c * d);
  L.B = take((size_t)m * c * d);
  L.VB = take((size_t)m * c * d);
  L.TwY = take(cc * d);
  L.TwB = take(cc * d);
  L.RB = take(cc * d);
  L.Cq = take(cc * d);
  L.UR = take(cc * d);
  L.VR = take(cc * d);
  L.Jw = take(cc * d);
  L.Jv = take(cc * d);
  L.Dw = take(c * d);
  L.C1 = take((size_t)c * k * d);
  L.C2 = take((size_t)c * k * d);
  L.tauY = take(c * d);
  L.tauB = take(c * d);
  L.ints = take((2 + kSweeps) * sizeof(int));
  L.panel = take(panel_work_bytes((int)c));
  L.hr = take(hr_work_bytes(std::max(m, n), (int)c));
  L.split_elems = (size_t)kMaxSplitK * std::max(m, n) * c;
  L.split = take(L.split_elems * d);
  L.total = off;
  return L;
}

__global__ void k_rsvd_init(int* nbs, int c) {
  if (threadIdx.x == 0) nbs[0] = c;
}

int check_args(int64_t m, int64_t n, int64_t k, int64_t p, int q, int prec) {
  if (m < 1 || n < 1) return -1;
  if (k < 1) return -3;
  if (p < 0 || k + p > kMaxC || k + p > std::min(m, n)) return -4;
  if (q < 0 || q > 16) return -5;
  if (prec < 0 || prec > kPrecMax) return -15;
  if (std::max(m, n) > kMaxRows || m * n > ((int64_t)1 << 40)) return RANDUTV_E_UNSUPPORTED;
  return 0;
}

#define RCHK(x)                                             \
  do {                                                      \
    hipError_t e_ = (x);                                    \
    if (e_ != hipSuccess) return RANDUTV_E_HIP - (int)e_;   \
  } while (0)

}  // namespace

extern "C" {

int randutv_rsvd_workspace_size(int64_t m, int64_t n, int64_t k, int64_t p, int q, int prec,
                                size_t* bytes) {
  const int s = check_args(m, n, k, p, q, prec);
  if (s) return s;
  if (!bytes) return -7;
  *bytes = rsvd_layout(m, n, k, k + p).total;
  return 0;
}

int randutv_rsvd(int64_t m, int64_t n, int64_t k, int64_t p, int q, const double* A, int64_t lda,
                 const double* G, int64_t ldg, double* U, int64_t ldu, double* D, double* V,
                 int64_t ldv, int prec, void* work, size_t work_bytes, int* sweeps_out,
                 void* stream) {
  const int s = check_args(m, n, k, p, q, prec);
  if (s) return s;
  if (!A || lda < m) return -6;
  if (!G || ldg < m) return -8;
  if (!U || ldu < m) return -10;
  if (!D) return -12;
  if (!V || ldv < n) return -13;
  if (!work || ((uintptr_t)work & 255)) return -16;
  const int64_t c64 = k + p;
  const RsvdLayout L = rsvd_layout(m, n, k, c64);
  if (work_bytes < L.total) return RANDUTV_E_WORKSPACE;

  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)work;
  auto dp = [&](size_t off) { return (double*)(base + off); };
  double *Y = dp(L.Y), *Z = dp(L.Z), *VY = dp(L.VY), *Q = dp(L.Q), *Bm = dp(L.B),
         *VB = dp(L.VB), *TwY = dp(L.TwY), *TwB = dp(L.TwB), *RB = dp(L.RB), *Cq = dp(L.Cq),
         *UR = dp(L.UR), *VR = dp(L.VR), *Jw = dp(L.Jw), *Jv = dp(L.Jv), *Dw = dp(L.Dw),
         *C1 = dp(L.C1), *C2 = dp(L.C2), *tauY = dp(L.tauY), *tauB = dp(L.tauB),
         *split = dp(L.split);
  int* ints = (int*)(base + L.ints);  // size word, status word, sweep counters
  PanelWork pw;
  panel_work_carve(base + L.panel, (int)c64, &pw);
  HrWork hw;
  hr_work_carve(base + L.hr, std::max(m, n), (int)c64, &hw);
  StatusBlock* blk = (StatusBlock*)(base + L.status);
  pw.err = &blk->sync_err;
  const size_t se = L.split_elems;
  const Prec ps = sampling_prec(prec);  // sampling products
  const Prec pu = update_prec(prec);    // B = A Q
  const int M = (int)m, N = (int)n, K = (int)k, C = (int)c64;
  const int64_t cc = (int64_t)C * C;

  RCHK(status_init(st, blk));
  hipLaunchKernelGGL(k_rsvd_init, dim3(1), dim3(64), 0, st, ints, C);
  RCHK(hipGetLastError());
  // Range finder: Y = (A^T A)^q A^T G, Q = Householder Q factor of Y.
  RCHK(gemm(st, ps, true, false, N, C, M, 1.0, A, lda, G, ldg, 0.0, Y, N, split, se));
  for (int it = 0; it < q; ++it) {
    RCHK(gemm(st, ps, false, false, M, C, N, 1.0, A, lda, Y, N, 0.0, Z, M, split, se));
    RCHK(gemm(st, ps, true, false, N, C, M, 1.0, A, lda, Z, M, 0.0, Y, N, split, se));
  }
  RCHK(panel_qr_hr(st, N, C, Y, N, VY, N, nullptr, C, tauY, TwY, C, hw, pw, split, se));
  // Q = (I - V_Y Tw_Y V_Y^T) [I; 0] = [I; 0] - V_Y (Tw_Y V_Y(0:C, :)^T)
  RCHK(set_identity(st, N, C, Q, N));
  RCHK(gemm(st, PREC_FP64, false, true, C, C, C, 1.0, TwY, C, VY, N, 0.0, Cq, C, nullptr, 0));
  RCHK(gemm(st, PREC_FP64, false, false, N, C, C, -1.0, VY, N, Cq, C, 1.0, Q, N, split, se));
  // Stage two: B = A Q; B = Q_B R_B; R_B = U_R D W^T.
  RCHK(gemm(st, pu, false, false, M, C, N, 1.0, A, lda, Q, N, 0.0, Bm, M, split, se));
  RCHK(panel_qr_hr(st, M, C, Bm, M, VB, M, RB, C, tauB, TwB, C, hw, pw, split, se));
  RCHK(batched_svd(st, 1, ints, C, RB, cc, UR, VR, cc, Dw, C, Jw, Jv, ints + 1, kSweeps,
                   &blk->svd_fail));
  // U = Q_B [U_R(:, 0:K); 0] = U1 - V_B (Tw_B (V_B(0:C, :)^T U_R(:, 0:K)))
  RCHK(set_zero(st, M, K, U, ldu));
  RCHK(copy_matrix(st, C, K, UR, C, U, ldu));
  RCHK(gemm(st, PREC_FP64, true, false, C, K, C, 1.0, VB, M, UR, C, 0.0, C1, C, nullptr, 0));
  RCHK(gemm(st, PREC_FP64, false, false, C, K, C, 1.0, TwB, C, C1, C, 0.0, C2, C, nullptr, 0));
  RCHK(gemm(st, PREC_FP64, false, false, M, K, C, -1.0, VB, M, C2, C, 1.0, U, ldu, split, se));
  // V = Q W(:, 0:K), D = the K largest singular values.
  RCHK(gemm(st, PREC_FP64, false, false, N, K, C, 1.0, Q, N, VR, C, 0.0, V, ldv, split, se));
  RCHK(hipMemcpyAsync(D, Dw, (size_t)K * sizeof(double), hipMemcpyDeviceToDevice, st));
  RCHK(status_done(st, blk, K));
  if (sweeps_out) {
    const int r = read_status(work, nullptr, st);
    RCHK(hipMemcpy(sweeps_out, ints + 1, sizeof(int), hipMemcpyDeviceToHost));
    return r;
  }
  return 0;
}

}  // extern "C"
