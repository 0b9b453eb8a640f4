// Internal declarations of the gfx950 randUTV library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rutv {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Sub-panel width of the Householder panel kernel (columns factored one at a
// time between block-reflector updates of the rest of the panel).
constexpr int kPanelNB = 16;
// Most workgroups the cooperative panel kernel uses, and most rows one
// workgroup may own (its sub-panel slice lives in LDS).
constexpr int kPanelMaxWG = 256;
constexpr int kPanelMaxWGGlobal = 128;
constexpr int kPanelMaxRows = 256;
// Spin limit of cross-workgroup waits: far above any legitimate wait, so a
// wait that never ends turns into an error instead of a hang.
constexpr unsigned kSpinLimit = 1u << 20;
// Largest split-K factor of the thin GEMMs.
constexpr int kMaxSplitK = 8;
#ifndef MAX_SPLITK_SMALL
#define MAX_SPLITK_SMALL 64
#endif
constexpr int kMaxSplitKSmall = MAX_SPLITK_SMALL;  // for outputs of at most 32 tiles of 64 x 64

// Arithmetic of the thin-matrix products.  FP64, FP32 and BF16X3 have the
// randutv_prec values of the same names; BF16X6 (three bf16 pieces per
// operand, six products) is randutv_prec 4's update arithmetic.
enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2, PREC_BF16X6 = 3 };
// randutv_prec values of the mixed modes: BF16x3 sampling with FP32 updates,
// and BF16x3 sampling with BF16x6 updates.
constexpr int kPrecMixed = 3;
constexpr int kPrecMixed6 = 4;
constexpr int kPrecMax = 4;
// Sampling and update arithmetic of a randutv_prec value.
inline Prec sampling_prec(int prec) {
  return (prec == kPrecMixed || prec == kPrecMixed6) ? PREC_BF16X3 : (Prec)prec;
}
inline Prec update_prec(int prec) {
  return prec == kPrecMixed ? PREC_FP32 : prec == kPrecMixed6 ? PREC_BF16X6 : (Prec)prec;
}

// ---------------------------------------------------------------- timing
// Profiling classes: thin GEMMs per tile shape (0: 64 x 64, 1: 128 x 128),
// arithmetic (FP64, FP32, BF16x3, BF16x6) and transpose case (class =
// 16*shape + 4*prec + 2*tb + ta; one class is one kernel instantiation),
// then the other kernels.
enum ProfClass { PC_GEMM_NN = 0, PC_GEMM_TN = 1, PC_GEMM_NT = 2, PC_GEMM_TT = 3,
                 PC_SPLITK = 32, PC_PANEL, PC_SVD, PC_GEMM_SMALL,
                 PC_UV,  // + op: the U / V stream's FP64 64 x 64 products
                 PC_COUNT = PC_UV + 4 };
bool prof_on();
// Start event of a launch of class `cls`; returns a slot, or -1 when off or
// when timing is restricted to another class.
int prof_mark(hipStream_t st, int cls);
void prof_suppress(int delta);  // +1 / -1 around launches timed by an enclosing mark
// flops and bytes: the launch's algorithmic work and HBM operand traffic.
void prof_done(hipStream_t st, int slot, int cls, double flops, double bytes);

// ---------------------------------------------------------------- GEMM
// C(M x N) = alpha * op(A) * op(B) + beta * C, column-major, op = transpose
// if ta/tb.  `splitws` (>= kMaxSplitK * M * N doubles, or NULL) enables
// split-K for long reductions.  The arithmetic of the inner products is set
// by `prec`; operands and C are FP64 in memory.
// small_tiles marks the U / V stream's products: 64 x 64 tiles (shorter
// workgroups), ROLE 2 of k_gemm in FP64.
// A product operand already split into BF16 pieces (presplit): `rows` rows
// (M for op(A), N for op(B)), `piece` 16-byte chunks per piece.
struct PsOperand {
  const uint4* p;
  int64_t rows, kc, piece;
};
// The kernel's view of the pre-split operands (unused ones NULL).
struct PsOps {
  const uint4* a;
  const uint4* b;
  int64_t rows_a, rows_b, piece_a, piece_b;
};
// Where a product's result is: p with leading dimension ld, as `splits`
// FP64 partials zs apart (to be summed in order) or one matrix (splits 1).
struct SplitKeep {
  const double* p;
  int64_t ld;
  int splits;
  int64_t zs;
};
// psa / psb (may be NULL, BF16x3 and BF16x6 only): op(A) (M x K) / op(B)
// (N x K, as rows) from presplit instead of A / B, which are then unused.
// keep (may be NULL): with alpha 1 and beta 0 a split-K product skips its
// reduction and leaves the partials in splitws for the consumer (presplit
// with S > 1); *keep says where the result is (C itself when not split).
hipError_t gemm(hipStream_t st, Prec prec, bool ta, bool tb, int M, int N, int K,
                double alpha, const double* A, int64_t lda, const double* B,
                int64_t ldb, double beta, double* C, int64_t ldc,
                double* splitws, size_t splitws_elems, bool small_tiles = false,
                const PsOperand* psa = nullptr, const PsOperand* psb = nullptr,
                SplitKeep* keep = nullptr);
// Bytes of the pieces of an R x K operand in `prec` (0 unless BF16x3/BF16x6).
size_t presplit_bytes(Prec prec, int64_t R, int64_t K);
// Split op(X), R x K (element (r, k) = X[r + k ldx] when rcontig, else
// X[k + r ldx]), into BF16 pieces at `out` (presplit_bytes, 16-byte aligned)
// the way the GEMM loaders split FP64 operands, and describe them in *o.
// With S > 1, X holds S split-K partials zs doubles apart (SplitKeep) and
// op(X) is their sum.
hipError_t presplit(hipStream_t st, Prec prec, int R, int K, const double* X, int64_t ldx,
                    bool rcontig, void* out, PsOperand* o, int S = 1, int64_t zs = 0);
// +1 / -1 around the products of a panel factorization: the FP64 products
// in between launch their own kernel instantiation (same code), so traces
// and counters tell them from the method's thin products.  Host-side, one
// enqueuing thread at a time (as the factorization's lock ensures).
void gemm_panel_scope(int delta);

// ---------------------------------------------------------------- panel QR
struct PanelWork {
  double* part;   // 2 * kPanelMaxWG * kPanelNB  (column-step partials)
  double* bcast;  // 2 * kPanelNB                (pivot row broadcast)
  double* bpart;  // kPanelMaxWG * kPanelNB * bmax (block-update partials)
  double* red;    // kPanelNB * bmax            (reduced block products)
  double* gram;   // 2 * kPanelMaxWG * 256      (sub-panel Gram partials)
  double* qtop;   // kPanelNB^2                 (top rows of the sub-panel Q)
  unsigned* bar;  // 2 counters                  (grid barrier)
  int* err;       // 1 flag                      (barrier spin limit hit)
};
size_t panel_work_bytes(int bmax);
void panel_work_carve(void* base, int bmax, PanelWork* w);

// Unpivoted Householder QR of the Mp x nb panel P (in place, LAPACK dgeqrf
// layout: R on and above the diagonal, reflector tails below), tau[nb], and
// the upper-triangular compact-WY factor Tw (nb x nb, ld = ldtw) with
// H_0 ... H_{nb-1} = I - V Tw V^T.
// Launched kernels return at once when `gate` is non-NULL and *gate == 0.
hipError_t panel_qr(hipStream_t st, int Mp, int nb, double* P, int64_t ldp,
                    double* tau, double* Tw, int64_t ldtw, const PanelWork& w,
                    const int* gate = nullptr);

// V (Mp x nb, unit lower trapezoidal, explicit ones and zeros) from the
// dgeqrf layout in P; R (nb x nb upper triangle, zeros below) to Rout.
hipError_t panel_extract(hipStream_t st, int Mp, int nb, const double* P, int64_t ldp,
                         double* V, int64_t ldv, double* Rout, int64_t ldr,
                         const int* gate = nullptr);

// Whole-panel Householder QR by CholeskyQR2 + Householder reconstruction,
// with the column-by-column kernel as a device-gated fallback.
struct HrWork {
  double *G, *R1, *R1i, *R2, *R2i, *RF, *QT, *LU, *Ui, *Li, *US, *Wc, *Cc;  // 128^2 each
  double* Q1;  // Mp_max x 128
  double* P2;  // Mp_max x 128 (second block of a panel wider than 128)
  int* flag;   // 1 when the fallback ran
};
size_t hr_work_bytes(int64_t Mp_max, int nb_max);
void hr_work_carve(void* base, int64_t Mp_max, int nb_max, HrWork* w);
// P (Mp x nb, ld ldp) is read (and only overwritten when the fallback runs);
// V (Mp x nb) receives the unit-lower-trapezoidal reflectors with explicit
// ones and zeros, Rout (nb x nb, may be NULL) the R factor with zeros
// below, tau[nb] and Tw (upper, I - V Tw V^T = H_0 ... H_{nb-1}).
// `split` (split_elems doubles) serves the split-K reductions.
hipError_t panel_qr_hr(hipStream_t st, int Mp, int nb, double* P, int64_t ldp, double* V,
                       int64_t ldv, double* Rout, int64_t ldr, double* tau, double* Tw,
                       int64_t ldtw, const HrWork& hw, const PanelWork& pw, double* split,
                       size_t split_elems);
// Xi = X^-1 for X (n x n, n <= 128) upper triangular, or unit lower
// triangular when !upper (diagonal taken as 1); zeros outside the triangle.
hipError_t tri_inv(hipStream_t st, int n, const double* X, int64_t ldx, double* Xi, int64_t ldxi,
                   bool upper);
// P = [R above and on the diagonal; V below] (LAPACK dgeqrf layout).
hipError_t pack_qr(hipStream_t st, int Mp, int nb, const double* V, int64_t ldv,
                   const double* R, int64_t ldr, double* P, int64_t ldp);

// ---------------------------------------------------------------- small SVD
// Batched one-sided Jacobi SVD of `count` square matrices R_i (size nb_i,
// stored at R + i*strideR with leading dimension ld) -> Us_i, D_i, Vs_i.
// Singular values descending, each (u_j, v_j) sign-normalised so that the
// largest |v_j| entry is positive.  status[i] = sweeps used, or -1 if not
// converged within max_sweeps, and then *fail (device word, may be NULL) is
// or-ed with 1.  Enqueue only: the convergence decision is taken on the
// device.
// nb_dev: device array of sizes; Wk, Vk: scratch of the same shape as Us;
// status: count + count * max_sweeps ints (status words, sweep counters).
hipError_t batched_svd(hipStream_t st, int count, const int* nb_dev, int ld,
                       const double* R, int64_t strideR, double* Us, double* Vs,
                       int64_t strideUV, double* D, int64_t strideD, double* Wk,
                       double* Vk, int* status, int max_sweeps, int* fail);

// ---------------------------------------------------------------- call status
// Status words a factorization (or randomized SVD) leaves at the start of its
// workspace, so that an enqueue-only call can be checked later
// (randutv_status).  sync_err: a bounded cross-workgroup wait hit its spin
// limit; svd_fail: a Jacobi SVD did not converge within its sweep budget;
// k: the number of leading columns reduced; magic: kStatusMagic once the
// call's last kernel has run.
struct StatusBlock {
  int sync_err;
  int svd_fail;
  long long k;
  int magic;
  int pad;
};
constexpr int kStatusMagic = 0x52555456;
constexpr size_t kStatusBytes = 256;  // bytes reserved for it (keeps 256-byte alignment)
// All words cleared (magic 0, k = -1), on the stream.
hipError_t status_init(hipStream_t st, StatusBlock* blk);
// k and the magic word written, on the stream (after the call's other work).
hipError_t status_done(hipStream_t st, StatusBlock* blk, long long k);
// Waits for the stream, then turns the status words at `work` into a status
// code (0, 1 for a non-converged SVD, RANDUTV_E_SYNC, RANDUTV_E_UNSUPPORTED
// when no call has completed there) and *k_out (may be NULL).
int read_status(const void* work, int64_t* k_out, hipStream_t st);

// Raises kernel `fn`'s dynamic-LDS limit to `bytes` on the current device,
// once per device and kernel (thread-safe).
hipError_t ensure_dyn_lds(const void* fn, int bytes);

// ---------------------------------------------------------------- factor core
// Reflectors and R factors of the first t steps, for the truncated
// approximation and its backward: per step i, Vy (n x b, ld n), Ty and Ry
// (b x b), Vu (m x b, ld m), Tu and Ru (b x b).
struct ApproxTape {
  double* p;
  int64_t m, n, b, t;
  int64_t stride() const { return n * b + m * b + 4 * b * b; }
  double* Vy(int64_t i) const { return p + i * stride(); }
  double* Ty(int64_t i) const { return Vy(i) + n * b; }
  double* Ry(int64_t i) const { return Ty(i) + b * b; }
  double* Vu(int64_t i) const { return Ry(i) + b * b; }
  double* Tu(int64_t i) const { return Vu(i) + m * b; }
  double* Ru(int64_t i) const { return Tu(i) + b * b; }
  static size_t bytes(int64_t m, int64_t n, int64_t b, int64_t t) {
    return (size_t)t * (n * b + m * b + 4 * b * b) * sizeof(double);
  }
};
// randutv_factor's body; with a tape, the reflectors of every step are kept
// there and the loop ends without the small SVDs (k_stop must be set).
int factor_impl(int64_t m, int64_t n, int64_t b, int q, double* T, int64_t ldt, const double* G,
                int64_t ldg, double* U, int64_t ldu, double* V, int64_t ldv, int64_t k_stop,
                double tol, int prec, unsigned flags, void* work, size_t work_bytes,
                int64_t* k_out, void* stream, const ApproxTape* tape);
size_t factor_work_bytes(int64_t m, int64_t n, int64_t b);
// factor_impl with over-sampling p; use_side false keeps the U and V updates
// on the caller's stream (no second stream is created or used).
int factor_core(int64_t m, int64_t n, int64_t b, int64_t p, int q, double* T, int64_t ldt,
                const double* G, int64_t ldg, double* U, int64_t ldu, double* V, int64_t ldv,
                int64_t k_stop, double tol, int prec, unsigned flags, void* work,
                size_t work_bytes, int64_t* k_out, void* stream, const ApproxTape* tape,
                bool use_side);

// ---------------------------------------------------------------- misc
hipError_t copy_matrix(hipStream_t st, int M, int N, const double* A, int64_t lda,
                       double* B, int64_t ldb);
hipError_t set_zero(hipStream_t st, int M, int N, double* A, int64_t lda);
hipError_t set_identity(hipStream_t st, int M, int N, double* A, int64_t lda);
// A(0:nb,0:nb) = diag(D) with exact zeros elsewhere in the nb x nb block;
// rows nb..M-1 of those columns are zeroed too.
hipError_t set_diag_block(hipStream_t st, int M, int nb, const double* D, double* A,
                          int64_t lda);
// out[0] = sum of squares of A (M x N).  `scratch` >= 1024 doubles.
hipError_t sumsq(hipStream_t st, int M, int N, const double* A, int64_t lda,
                 double* scratch, double* out);

}  // namespace rutv
