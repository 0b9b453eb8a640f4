// randUTV driver and C ABI (Figure "The algorithm randUTV", Section 5.2).
//
// Per randomized step i (r0 = i*b, X = T(r0:m, r0:n)):
//   Y = X^T G_i; q times: Z = X Y, Y = X^T Z            (thin MFMA GEMMs)
//   [p > 0: Y <- its b dominant left singular vectors]   (over-sampling)
//   Householder QR of Y -> Vh, tau, Tw_V                 (panel_qr_hr)
//   T(:, r0:n) <- T(:, r0:n) (I - Vh Tw_V Vh^T)          (all m rows)
//   V(:, r0:n) likewise                                  (second stream)
//   Householder QR of T(r0:m, r0:r0+b) -> Uh, Tw_U, R    (panel_qr_hr)
//   T(r0:m, r0+b:n) <- (I - Uh Tw_U Uh^T)^T T(...)
//   U(:, r0:m) <- U(:, r0:m) (I - Uh Tw_U Uh^T)          (second stream)
//   T(r0:m, r0:r0+b) <- 0, R stashed
// The last block (I3 or J3 empty) takes the economic path of the Remark on
// tall SVDs: Householder QR, then the SVD of its square R; with fewer rows
// than columns, an LQ of the block row (the Remark on the case m < n).
// The b x b SVDs do not feed later steps: step i's rotations act only on
// block row i (from the left), block column i (from the right) and columns
// of U and V that later steps never touch, and left and right
// multiplications commute.  So all SVDs run batched after the loop (block
// Jacobi, every matrix at once) and their rotations are folded back then.
// The lower-triangular form A = U L V^T runs this on A^T.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/randutv.h"
#include "common.h"

using namespace rutv;

namespace {

constexpr int kMaxB = 256;
constexpr int kMaxPanelRows = kPanelMaxWGGlobal * kPanelMaxRows;
// Sweep budget of the one-sided Jacobi SVDs.  The zero-padded, rank-deficient
// factors of over-sampled steps with fewer than b + p rows left need more
// than 30 sweeps (their near-zero columns keep rotating at rounding level).
constexpr int kJacobiSweeps = 40;

// Reflector slots shared with the U / V stream (step i uses slot i % kSlots).
#ifndef UV_SLOTS
#define UV_SLOTS 3
#endif
constexpr int kSlots = UV_SLOTS;

struct Layout {
  size_t status, Y, Z, W, W2, Ws, W2s, C, C2, tauV, tauU, Rst, TwUst, Ust, Vst, D, Jw, Jv, Ftmp,
      split, nrm, ints, panel, hr, total;
  size_t Vh[kSlots], Uh[kSlots], TwV[kSlots], TwU[kSlots];  // reflector slots
  // Over-sampling (p > 0) only: QR and SVD of the extended sample.
  size_t VY, TwY, RY, UR, VR, JwR, JvR, tauY, DR, Cy, Cy2, intsY;
  size_t split_elems;
};

// Ints per step for the SVD of the extended sample: the size word, the
// status word and one rotation counter per sweep.
constexpr int kIntsY = 2 + kJacobiSweeps;

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// FORM_U, FORM_V, and ECON_U together with FORM_U.
bool valid_flags(unsigned flags) {
  if (flags & ~(unsigned)(RANDUTV_FORM_U | RANDUTV_FORM_V | RANDUTV_ECON_U | RANDUTV_ONE_STREAM))
    return false;
  return !(flags & RANDUTV_ECON_U) || (flags & RANDUTV_FORM_U);
}

int64_t num_steps(int64_t m, int64_t n, int64_t b) {
  return std::min((m + b - 1) / b, (n + b - 1) / b);
}

// Sampling buffers Y and Z are b + p columns wide.
Layout make_layout(int64_t m, int64_t n, int64_t b, int64_t p = 0) {
  Layout L{};
  const int64_t s = num_steps(m, n, b);
  const int64_t bp = b + p;
  const size_t d = sizeof(double);
  const size_t mb = (size_t)m * b, nb = (size_t)n * b, bb = (size_t)b * b;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = al256(off + bytes);
    return o;
  };
  L.status = take(kStatusBytes);  // first: randutv_status reads it at offset 0
  L.Y = take((size_t)n * bp * d);
  for (int k = 0; k < kSlots; ++k) L.Vh[k] = take(nb * d);
  L.Z = take((size_t)m * bp * d);
  for (int k = 0; k < kSlots; ++k) L.Uh[k] = take(mb * d);
  L.W = take(mb * d);
  L.W2 = take(mb * d);
  L.Ws = take(std::max(mb, nb) * d);   // U / V stream products, leading dimension max(m, n)
  L.W2s = take(std::max(mb, nb) * d);
  L.C = take(nb * d);
  L.C2 = take(nb * d);
  for (int k = 0; k < kSlots; ++k) L.TwV[k] = take(bb * d);
  for (int k = 0; k < kSlots; ++k) L.TwU[k] = take(bb * d);
  L.tauV = take(b * d);
  L.tauU = take(b * d);
  L.Rst = take(s * bb * d);
  L.TwUst = take(s * bb * d);  // compact-WY factors of the left transforms (economy U)
  L.Ust = take(s * bb * d);
  L.Vst = take(s * bb * d);
  L.D = take(s * b * d);
  L.Jw = take(s * bb * d);
  L.Jv = take(s * bb * d);
  L.Ftmp = take(std::max(mb, nb) * d);
  L.split_elems = (size_t)kMaxSplitK * std::max(m, n) * bp;
  L.split = take(L.split_elems * d);
  L.nrm = take(1040 * d);
  L.ints = take((2 * s + s * kJacobiSweeps + 8) * sizeof(int));
  L.panel = take(panel_work_bytes((int)bp));
  L.hr = take(hr_work_bytes(std::max(m, n), (int)bp));
  if (p > 0) {
    const size_t bpb = (size_t)bp * bp;
    L.VY = take((size_t)n * bp * d);
    L.TwY = take(bpb * d);
    L.RY = take(bpb * d);
    L.UR = take(bpb * d);
    L.VR = take(bpb * d);
    L.JwR = take(bpb * d);
    L.JvR = take(bpb * d);
    L.tauY = take(bp * d);
    L.DR = take(bp * d);
    L.Cy = take((size_t)bp * b * d);
    L.Cy2 = take((size_t)bp * b * d);
    L.intsY = take((size_t)s * kIntsY * sizeof(int));
  }
  L.total = off;
  return L;
}

// Split-precision factorizations also take two buffers for operands split
// into BF16 pieces once per product (presplit), when the workspace holds
// them: the thin operands of the sampling and update products, which every
// workgroup of a product would otherwise read and split again.
bool uses_bf16(int prec) {
  const Prec ps = sampling_prec(prec), pu = update_prec(prec);
  return ps == PREC_BF16X3 || ps == PREC_BF16X6 || pu == PREC_BF16X3 || pu == PREC_BF16X6;
}
size_t presplit_buf_bytes(int64_t m, int64_t n, int64_t bp) {
  const int64_t r = std::max(m, n);
  return al256(std::max(presplit_bytes(PREC_BF16X6, r, bp), presplit_bytes(PREC_BF16X6, bp, r)));
}
size_t factor_bytes(int64_t m, int64_t n, int64_t b, int64_t p, int prec) {
  return make_layout(m, n, b, p).total + (uses_bf16(prec) ? 2 * presplit_buf_bytes(m, n, b + p) : 0);
}


// U and V accumulation runs on a second stream of the device (default
// priority), ordered against the main stream by events: the panels and
// small products of the main chain are latency-bound and leave most of the
// chip idle, which the FP64 U / V block-reflector products fill.  Step i
// uses reflector slot i % kSlots; the main stream waits for the side stream
// to release a slot before overwriting it (three slots let the side stream
// fall two steps behind without stalling the main one: 126-127 ms per
// 8000 x 8000 factorization against 127.5-128.4 ms with two).
struct SideCtx {
  hipStream_t side = nullptr;
  // V ready, U ready, V done, U done (kSlots each), join.
  hipEvent_t ev[4 * kSlots + 1] = {};
  bool ok = false;
};
constexpr int kMaxDevices = 64;
SideCtx g_side[kMaxDevices];
std::mutex g_mu;  // one factorization enqueues at a time (shared events)

// The side streams and their events are released when the process exits,
// before the HIP runtime's own teardown (this handler is registered after
// the runtime has initialised, so it runs first).
void release_side() {
  for (auto& c : g_side) {
    for (auto& e : c.ev)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
    if (c.side) {
      (void)hipStreamDestroy(c.side);
      c.side = nullptr;
    }
    c.ok = false;
  }
}

SideCtx* side_ctx() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  static bool registered = false;  // g_mu is held
  if (!registered) {
    std::atexit(release_side);
    registered = true;
  }
  SideCtx& c = g_side[dev];
  if (!c.ok) {
    if (!c.side && hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking) != hipSuccess) {
      c.side = nullptr;
      return nullptr;
    }
    for (auto& e : c.ev)
      if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        e = nullptr;
        return nullptr;
      }
    c.ok = true;
  }
  return &c;
}

// FP64 product for the U / V stream on 64 x 64 tiles, cut into launches of
// at most kSideCols output columns and a reduction of at most `chunk`
// (beta = 1 after the first).  A panel kernel on the main stream needs most
// of a CU's LDS, and while a side launch still has workgroups queued, every
// CU that frees up is refilled from it; so the panel starts only when a
// side launch ends.  Short launches (about 130 us for the rank-b updates at
// n = 8000) bound that wait, at some cost in tail effects of the side
// products (measured: 1024 columns, 129.4 ms per factorization against
// 134.6 ms uncut; 512-1536 within 1 ms of that).  The reduction chunk of W =
// X Vh is deeper when the main stream's updates are FP64: their longer
// launches leave the side stream more room (n = 8000: 512 deep, 126.5 ms
// against 128.4 ms at 256; 768 and 1024 deep in between), while with split
// updates 256 and 512 measure the same within noise.
#ifndef SIDE_CHUNK
#define SIDE_CHUNK 256
#endif
#ifndef SIDE_CHUNK_FP64
#define SIDE_CHUNK_FP64 512
#endif
#ifndef SIDE_COLS
#define SIDE_COLS 1024
#endif
constexpr int kSideChunk = SIDE_CHUNK;  // reduction chunk of the thin products W = X Vh
constexpr int kSideChunkFp64 = SIDE_CHUNK_FP64;  // the same with FP64 updates
constexpr int kSideChunkUpd = 256;  // and of the rank-b updates X -= W2 Vh^T
constexpr int kSideCols = SIDE_COLS;  // output columns per launch
hipError_t gemm_side(hipStream_t st, bool ta, bool tb, int M, int N, int K, double alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                     double* C, int64_t ldc, int chunk) {
  for (int n0 = 0; n0 < N; n0 += kSideCols) {
    const int nc = std::min(kSideCols, N - n0);
    const double* Bn = B + (tb ? (int64_t)n0 : (int64_t)n0 * ldb);
    double* Cn = C + (int64_t)n0 * ldc;
    for (int k0 = 0; k0 < K || k0 == 0; k0 += chunk) {
      const int kc = std::min(chunk, K - k0);
      const double* Ak = A + (ta ? (int64_t)k0 : (int64_t)k0 * lda);
      const double* Bk = Bn + (tb ? (int64_t)k0 * ldb : (int64_t)k0);
      const hipError_t e = gemm(st, PREC_FP64, ta, tb, M, nc, kc, alpha, Ak, lda, Bk, ldb,
                                k0 == 0 ? beta : 1.0, Cn, ldc, nullptr, 0, true);
      if (e != hipSuccess) return e;
      if (K <= 0) break;
    }
  }
  return hipSuccess;
}

inline int grid_blocks(int64_t total) { return (int)std::min<int64_t>((total + 255) / 256, 4096); }

// B = A^T for the M x N matrix A (B is N x M).  Used once per factorization
// (the wide last block), so a plain strided copy.
__global__ void k_transpose(int M, int N, const double* __restrict__ A, int64_t lda,
                            double* __restrict__ Bt, int64_t ldb) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M);
    const int64_t j = idx / M;
    Bt[j + (int64_t)i * ldb] = A[i + j * lda];
  }
}

// B = A^T for the M x N matrix A through 32 x 32 LDS tiles (coalesced reads
// and writes); the whole-matrix transposes of the lower-triangular variant.
constexpr int kTT = 32;
__global__ __launch_bounds__(256) void k_transpose_tiled(int M, int N, const double* __restrict__ A,
                                                         int64_t lda, double* __restrict__ Bt,
                                                         int64_t ldb) {
  __shared__ double t[kTT][kTT + 1];
  const int i0 = blockIdx.x * kTT, j0 = blockIdx.y * kTT;
  const int tx = threadIdx.x % kTT, ty = threadIdx.x / kTT;
  for (int jj = ty; jj < kTT; jj += 256 / kTT) {
    const int i = i0 + tx, j = j0 + jj;
    if (i < M && j < N) t[jj][tx] = A[i + (int64_t)j * lda];
  }
  __syncthreads();
  for (int ii = ty; ii < kTT; ii += 256 / kTT) {
    const int j = j0 + tx, i = i0 + ii;
    if (i < M && j < N) Bt[j + (int64_t)i * ldb] = t[tx][ii];
  }
}

hipError_t transpose(hipStream_t st, int M, int N, const double* A, int64_t lda, double* Bt,
                     int64_t ldb) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_tiled, dim3((M + kTT - 1) / kTT, (N + kTT - 1) / kTT),
                     dim3(256), 0, st, M, N, A, lda, Bt, ldb);
  return hipGetLastError();
}

__global__ void k_set_ints(int* p, int count, int v, int last) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = (i == count - 1) ? last : v;
}
__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) p[0] = 0;
}

// Over-sampling (Remark on over-sampling, Section 5.3; Appendix A.2, Figure
// of the over-sampled step): replace the Ni x (b+p) sample Y by its b
// dominant left singular vectors, in the first b columns of Y.  With
// Ni >= b+p: Y = Q_Y R_Y (Householder), R_Y = U_R S W^T, and the vectors
// are Q_Y U_R(:, 0:b) = U1 - V_Y Tw_Y V_Y^T U1 with U1 = [U_R(:, 0:b); 0].
// With Ni < b+p the SVD is taken of Y padded with zero rows to b+p, whose
// leading Ni rows of the left singular vectors are those of Y.  Either way
// the right singular vectors are Y's own, so the batched SVD's sign rule
// (largest entry of each right vector positive) fixes each vector's sign.
// `iy` holds the size word, the status word and the sweep counters.
hipError_t oversample_basis(hipStream_t st, int Ni, int B, int Bp, double* Y, int64_t ldy,
                            const Layout& L, char* base, int* iy, const HrWork& hw,
                            const PanelWork& pw, double* split, size_t se, int* fail) {
  auto dp = [&](size_t off) { return (double*)(base + off); };
  double *VY = dp(L.VY), *TwY = dp(L.TwY), *RY = dp(L.RY), *UR = dp(L.UR), *VR = dp(L.VR),
         *JwR = dp(L.JwR), *JvR = dp(L.JvR), *tauY = dp(L.tauY), *DR = dp(L.DR), *Cy = dp(L.Cy),
         *Cy2 = dp(L.Cy2);
  const int64_t bb = (int64_t)Bp * Bp;
  hipError_t e;
  const bool tall = Ni >= Bp;
  if (tall) {
    e = panel_qr_hr(st, Ni, Bp, Y, ldy, VY, ldy, RY, Bp, tauY, TwY, Bp, hw, pw, split, se);
  } else {
    e = set_zero(st, Bp, Bp, RY, Bp);
    if (e == hipSuccess) e = copy_matrix(st, Ni, Bp, Y, ldy, RY, Bp);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_set_ints, dim3(1), dim3(64), 0, st, iy, 1, Bp, Bp);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = batched_svd(st, 1, iy, Bp, RY, bb, UR, VR, bb, DR, Bp, JwR, JvR, iy + 1, kJacobiSweeps,
                    fail);
  if (e != hipSuccess) return e;
  if (!tall) return copy_matrix(st, Ni, B, UR, Bp, Y, ldy);
  e = set_zero(st, Ni, B, Y, ldy);
  if (e == hipSuccess) e = copy_matrix(st, Bp, B, UR, Bp, Y, ldy);
  if (e == hipSuccess)  // Cy = V_Y(0:Bp, :)^T U1
    e = gemm(st, PREC_FP64, true, false, Bp, B, Bp, 1.0, VY, ldy, UR, Bp, 0.0, Cy, Bp, nullptr, 0);
  if (e == hipSuccess)
    e = gemm(st, PREC_FP64, false, false, Bp, B, Bp, 1.0, TwY, Bp, Cy, Bp, 0.0, Cy2, Bp, nullptr, 0);
  if (e == hipSuccess)
    e = gemm(st, PREC_FP64, false, false, Ni, B, Bp, -1.0, VY, ldy, Cy2, Bp, 1.0, Y, ldy, split, se);
  return e;
}

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return RANDUTV_E_HIP - (int)e_; \
  } while (0)

}  // namespace

extern "C" {

int64_t randutv_random_steps(int64_t m, int64_t n, int64_t b) {
  if (m < 1 || n < 1 || b < 1) return -1;
  const int64_t s = num_steps(m, n, b);
  int64_t c = 0;
  for (int64_t i = 0; i < s; ++i)
    if (i * b + b < m && i * b + b < n) ++c;
  return c;
}

int64_t randutv_g_cols_p(int64_t m, int64_t n, int64_t b, int64_t p) {
  const int64_t r = randutv_random_steps(m, n, b);
  return (r < 0 || p < 0) ? -1 : r * (b + p);
}

int64_t randutv_g_cols(int64_t m, int64_t n, int64_t b) { return randutv_g_cols_p(m, n, b, 0); }

int randutv_workspace_size_p(int64_t m, int64_t n, int64_t b, int64_t p, int q, int prec,
                             unsigned flags, size_t* bytes) {
  if (n < 1 || m < 1) return -1;
  if (b < 1 || b > kMaxB) return -3;
  if (p < 0 || b + p > kMaxB) return -4;
  if (q < 0 || q > 16) return -5;
  if (prec < 0 || prec > kPrecMax) return -6;
  if (!valid_flags(flags)) return -7;
  if (!bytes) return -8;
  *bytes = factor_bytes(m, n, b, p, prec);
  return 0;
}

// flags of the transposed problem: U of A^T is V of A and vice versa.
// (The economy U has no counterpart for V, so the lower form takes neither.)
inline unsigned swap_uv(unsigned flags) {
  return (flags & RANDUTV_FORM_U ? RANDUTV_FORM_V : 0u) | (flags & RANDUTV_FORM_V ? RANDUTV_FORM_U : 0u);
}

int randutv_workspace_size_lower(int64_t m, int64_t n, int64_t b, int q, int prec, unsigned flags,
                                 size_t* bytes) {
  if (n < 1 || m < 1) return -1;
  if (b < 1 || b > kMaxB) return -3;
  if (q < 0 || q > 16) return -4;
  if (prec < 0 || prec > kPrecMax) return -5;
  if (flags & ~(unsigned)(RANDUTV_FORM_U | RANDUTV_FORM_V)) return -6;
  if (!bytes) return -7;
  *bytes = factor_bytes(n, m, b, 0, prec) + al256((size_t)m * n * sizeof(double));
  return 0;
}

int randutv_workspace_size(int64_t m, int64_t n, int64_t b, int q, int prec, unsigned flags,
                           size_t* bytes) {
  if (n < 1 || m < 1) return -1;
  if (b < 1 || b > kMaxB) return -3;
  if (q < 0 || q > 16) return -4;
  if (prec < 0 || prec > kPrecMax) return -5;
  if (!valid_flags(flags)) return -6;
  if (!bytes) return -7;
  *bytes = factor_bytes(m, n, b, 0, prec);
  return 0;
}

const char* randutv_strerror(int status) {
  if (status == 0) return "success";
  if (status == 1) return "a small SVD did not converge within the sweep limit";
  if (status == RANDUTV_E_UNSUPPORTED) return "unsupported case";
  if (status == RANDUTV_E_WORKSPACE) return "workspace too small or misaligned";
  if (status == RANDUTV_E_SYNC) return "cross-workgroup wait exceeded its spin limit";
  if (status <= RANDUTV_E_HIP) return "HIP runtime error";
  if (status < 0) return "invalid argument";
  return "unknown status";
}

int randutv_factor(int64_t m, int64_t n, int64_t b, int q, double* T, int64_t ldt,
                   const double* G, int64_t ldg, double* U, int64_t ldu, double* V,
                   int64_t ldv, int64_t k_stop, double tol, int prec, unsigned flags,
                   void* work, size_t work_bytes, int64_t* k_out, void* stream) {
  return rutv::factor_impl(m, n, b, q, T, ldt, G, ldg, U, ldu, V, ldv, k_stop, tol, prec, flags,
                           work, work_bytes, k_out, stream, nullptr);
}

int randutv_factor_lower(int64_t m, int64_t n, int64_t b, int q, double* T, int64_t ldt,
                         const double* G, int64_t ldg, double* U, int64_t ldu, double* V,
                         int64_t ldv, int64_t k_stop, double tol, int prec, unsigned flags,
                         void* work, size_t work_bytes, int64_t* k_out, void* stream) {
  if (m < 1 || n < 1) return -1;
  if (std::max(m, n) > kMaxPanelRows || m * n > ((int64_t)1 << 40)) return RANDUTV_E_UNSUPPORTED;
  if (b < 1 || b > kMaxB) return -2;
  if (q < 0 || q > 16) return -3;
  if (!T || ldt < m) return -4;
  if (randutv_g_cols(n, m, b) > 0 && (!G || ldg < n)) return -5;
  if ((flags & RANDUTV_FORM_U) && (!U || ldu < m)) return -6;
  if ((flags & RANDUTV_FORM_V) && (!V || ldv < n)) return -7;
  if (prec < 0 || prec > kPrecMax) return -10;
  if (flags & ~(unsigned)(RANDUTV_FORM_U | RANDUTV_FORM_V)) return -11;
  if (!work || ((uintptr_t)work & 255)) return -12;
  size_t need = 0;
  randutv_workspace_size_lower(m, n, b, q, prec, flags, &need);
  if (work_bytes < need) return RANDUTV_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  // The inner factorization's workspace comes first (its status words at
  // offset 0), then A^T (n x m).
  const size_t fb = factor_bytes(n, m, b, 0, prec);
  double* Tt = (double*)((char*)work + fb);
  HIPCHK(transpose(st, (int)m, (int)n, T, ldt, Tt, n));
  // A^T = U' T' V'^T, so A = V' T'^T U'^T: U of A^T goes to V, V of A^T to U.
  // The inner call only enqueues; its status is read after the transpose back.
  const int r = rutv::factor_core(n, m, b, 0, q, Tt, n, G, ldg, V, ldv, U, ldu, k_stop, tol, prec,
                                  swap_uv(flags), work, fb, nullptr, stream, nullptr, true);
  if (r < 0) return r;
  HIPCHK(transpose(st, (int)n, (int)m, Tt, n, T, ldt));
  if (k_out) return read_status(work, k_out, st);
  return 0;
}

int randutv_status(const void* work, size_t work_bytes, int64_t* k_out, void* stream) {
  if (!work || ((uintptr_t)work & 255)) return -1;
  if (work_bytes < kStatusBytes) return -2;
  return read_status(work, k_out, (hipStream_t)stream);
}

int randutv_factor_p(int64_t m, int64_t n, int64_t b, int64_t p, int q, double* T, int64_t ldt,
                     const double* G, int64_t ldg, double* U, int64_t ldu, double* V,
                     int64_t ldv, int64_t k_stop, double tol, int prec, unsigned flags,
                     void* work, size_t work_bytes, int64_t* k_out, void* stream) {
  return rutv::factor_core(m, n, b, p, q, T, ldt, G, ldg, U, ldu, V, ldv, k_stop, tol, prec, flags,
                     work, work_bytes, k_out, stream, nullptr, true);
}
}  // extern "C"

namespace rutv {

size_t factor_work_bytes(int64_t m, int64_t n, int64_t b) { return make_layout(m, n, b).total; }

int factor_impl(int64_t m, int64_t n, int64_t b, int q, double* T, int64_t ldt, const double* G,
                int64_t ldg, double* U, int64_t ldu, double* V, int64_t ldv, int64_t k_stop,
                double tol, int prec, unsigned flags, void* work, size_t work_bytes,
                int64_t* k_out, void* stream, const ApproxTape* tape) {
  return factor_core(m, n, b, 0, q, T, ldt, G, ldg, U, ldu, V, ldv, k_stop, tol, prec, flags, work,
                     work_bytes, k_out, stream, tape, true);
}

int factor_core(int64_t m, int64_t n, int64_t b, int64_t p, int q, double* T, int64_t ldt,
                const double* G, int64_t ldg, double* U, int64_t ldu, double* V, int64_t ldv,
                int64_t k_stop, double tol, int prec, unsigned flags, void* work,
                size_t work_bytes, int64_t* k_out, void* stream, const ApproxTape* tape,
                bool use_side) {
  if (m < 1 || n < 1) return -1;
  if (m < n && tape) return RANDUTV_E_UNSUPPORTED;  // the approximation takes m >= n
  if (p > 0 && tape) return RANDUTV_E_UNSUPPORTED;
  if (std::max(m, n) > kMaxPanelRows || m * n > ((int64_t)1 << 40)) return RANDUTV_E_UNSUPPORTED;
  if (b < 1 || b > kMaxB) return -2;
  if (p < 0 || b + p > kMaxB) return -13;
  if (q < 0 || q > 16) return -3;
  if (!T || ldt < m) return -4;
  const int64_t gcols = randutv_g_cols_p(m, n, b, p);
  if (gcols > 0 && (!G || ldg < m)) return -5;
  const bool formU = flags & RANDUTV_FORM_U, formV = flags & RANDUTV_FORM_V;
  if (formU && (!U || ldu < m)) return -6;
  if (formV && (!V || ldv < n)) return -7;
  if (prec < 0 || prec > kPrecMax) return -10;
  if (!valid_flags(flags)) return -11;
  if (!work || ((uintptr_t)work & 255)) return -12;
  const Layout L = make_layout(m, n, b, p);
  if (work_bytes < L.total) return RANDUTV_E_WORKSPACE;
  const size_t psb = presplit_buf_bytes(m, n, b + p);
  const bool use_ps = uses_bf16(prec) && work_bytes >= L.total + 2 * psb;

  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  char* base = (char*)work;
  auto dp = [&](size_t off) { return (double*)(base + off); };
  double *Y = dp(L.Y), *Z = dp(L.Z), *W = dp(L.W), *W2 = dp(L.W2), *Ws = dp(L.Ws),
         *W2s = dp(L.W2s), *C = dp(L.C), *C2 = dp(L.C2),
         *tauV = dp(L.tauV), *tauU = dp(L.tauU), *Rst = dp(L.Rst), *Ust = dp(L.Ust),
         *Vst = dp(L.Vst), *Dd = dp(L.D), *Jw = dp(L.Jw), *Jv = dp(L.Jv), *Ftmp = dp(L.Ftmp),
         *split = dp(L.split), *nrm = dp(L.nrm);
  const int64_t s = num_steps(m, n, b);
  int* ints = (int*)(base + L.ints);
  int* nbs = ints;
  int* jstatus = ints + s;
  PanelWork pw;
  panel_work_carve(base + L.panel, (int)(b + p), &pw);
  HrWork hw;
  hr_work_carve(base + L.hr, std::max(m, n), (int)(b + p), &hw);
  // The status words live at the start of the workspace; the panel kernels'
  // spin-limit flag is one of them.
  StatusBlock* blk = (StatusBlock*)(base + L.status);
  pw.err = &blk->sync_err;
  // Arithmetic of the sampling products (ps) and of the trailing updates (pu).
  const Prec ps = sampling_prec(prec);
  const Prec pu = update_prec(prec);
  const size_t se = L.split_elems;
  const int M = (int)m, N = (int)n, B = (int)b;
  const int Bp = (int)(b + p);    // samples per randomized step
  const int MN = std::max(M, N);  // leading dimension of the U / V stream products
  const int side_chunk = pu == PREC_FP64 ? kSideChunkFp64 : kSideChunk;
  int* intsY = p > 0 ? (int*)(base + L.intsY) : nullptr;
  // Buffers of the pre-split operands (use_ps), and the product through them:
  // op(A) from A (rows M, rcontig when A is not transposed) if sa, op(B)
  // from B (rows N, rcontig when B is transposed) if sb; plain gemm when
  // the product's arithmetic is not BF16 or the buffers are absent.
  void* psA = use_ps ? (void*)(base + L.total) : nullptr;
  void* psB = use_ps ? (void*)(base + L.total + psb) : nullptr;
  // With pre-split operands, inB (a SplitKeep, B not transposed) takes op(B)
  // from the previous product's unreduced partials, and out keeps this
  // product's partials for the next one (alpha 1, beta 0).
  auto gemm_ps = [&](Prec pr, bool ta, bool tb, int Mq, int Nq, int Kq, double al,
                     const double* Aq, int64_t lda, const double* Bq, int64_t ldb, double be,
                     double* Cq, int64_t ldc, double* sp, size_t spe, bool sa, bool sb,
                     const SplitKeep* inB = nullptr, SplitKeep* out = nullptr) -> hipError_t {
    if (!use_ps || !(pr == PREC_BF16X3 || pr == PREC_BF16X6) || Mq <= 0 || Nq <= 0 || Kq <= 0)
      return gemm(st, pr, ta, tb, Mq, Nq, Kq, al, Aq, lda, Bq, ldb, be, Cq, ldc, sp, spe);
    PsOperand oa{}, ob{};
    hipError_t e = hipSuccess;
    if (sa && (e = presplit(st, pr, Mq, Kq, Aq, lda, !ta, psA, &oa)) != hipSuccess) return e;
    if (sb) {
      e = inB ? presplit(st, pr, Nq, Kq, inB->p, inB->ld, false, psB, &ob, inB->splits, inB->zs)
              : presplit(st, pr, Nq, Kq, Bq, ldb, tb, psB, &ob);
      if (e != hipSuccess) return e;
    }
    return gemm(st, pr, ta, tb, Mq, Nq, Kq, al, Aq, lda, Bq, ldb, be, Cq, ldc, sp, spe, false,
                sa ? &oa : nullptr, sb ? &ob : nullptr, out);
  };

  double *VhS[kSlots], *UhS[kSlots], *TwVS[kSlots], *TwUS[kSlots];
  for (int k = 0; k < kSlots; ++k)
    VhS[k] = dp(L.Vh[k]), UhS[k] = dp(L.Uh[k]), TwVS[k] = dp(L.TwV[k]), TwUS[k] = dp(L.TwU[k]);
  constexpr int kVR = 0, kUR = kSlots, kVD = 2 * kSlots, kUD = 3 * kSlots, kJoin = 4 * kSlots;

  // Economy U (m x min(m, n)): each step's left reflectors are stored in U's
  // own block column (rows r0..m, LAPACK's dgeqrf layout with explicit ones
  // and zeros) and their compact-WY factors in a stash; U is formed after the
  // loop by backward accumulation (Q [I; 0], last block first).
  const bool econU = formU && (flags & RANDUTV_ECON_U);
  const int cU = econU ? (int)std::min(m, n) : M;  // columns of U
  double* TwUst = dp(L.TwUst);
  int nrefl = 0;  // leading blocks whose left reflectors are stored in U

  HIPCHK(status_init(st, blk));
  if (formU) HIPCHK(set_identity(st, M, cU, U, ldu));
  if (formV) HIPCHK(set_identity(st, N, N, V, ldv));
  // Without the second stream (use_side false) U and V are updated on the
  // caller's stream, in the same launches.
  if (flags & RANDUTV_ONE_STREAM) use_side = false;
  SideCtx* sc = (use_side && ((formU && !econU) || formV)) ? side_ctx() : nullptr;
  const hipStream_t ss = sc ? sc->side : st;  // U / V stream (the main one if none)
  bool vpend[kSlots] = {}, upend[kSlots] = {};
  if (sc) {
    HIPCHK(hipEventRecord(sc->ev[kJoin], st));
    HIPCHK(hipStreamWaitEvent(ss, sc->ev[kJoin], 0));
  }
  // Hand the reflectors of one side to the U / V stream and back.
  auto to_side = [&](int ready) -> hipError_t {
    if (!sc) return hipSuccess;
    hipError_t e = hipEventRecord(sc->ev[ready], st);
    return e == hipSuccess ? hipStreamWaitEvent(ss, sc->ev[ready], 0) : e;
  };
  auto side_done = [&](int done, bool* pend) -> hipError_t {
    if (!sc) return hipSuccess;
    *pend = true;
    return hipEventRecord(sc->ev[done], ss);
  };
  auto reclaim = [&](int done, bool pend) -> hipError_t {
    return sc && pend ? hipStreamWaitEvent(st, sc->ev[done], 0) : hipSuccess;
  };

  double normA = 0.0;
  if (tol > 0.0) {
    HIPCHK(sumsq(st, M, N, T, ldt, nrm + 16, nrm));
    double h = 0.0;
    HIPCHK(hipMemcpyAsync(&h, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    normA = std::sqrt(h);
  }

  // Blocks whose R goes to the batched SVD: all b wide except possibly the last.
  int nsvd = 0, last_w = B;
  int64_t k_done = std::min(m, n);
  for (int64_t i = 0; i < s; ++i) {
    const int r0 = (int)(i * b);
    const int Mi = M - r0, Ni = N - r0;
    double* X = T + r0 + (int64_t)r0 * ldt;
    const int sl = (int)(i % kSlots);
    double *Vh = VhS[sl], *Uh = UhS[sl], *TwV = TwVS[sl], *TwU = TwUS[sl];
    double *RV = nullptr, *RU = Rst + (size_t)i * B * B;
    int64_t ldUh = M;
    if (econU) {  // left reflectors into U's block column, their factor to the stash
      Uh = U + r0 + (int64_t)r0 * ldu;
      ldUh = ldu;
      TwU = TwUst + (size_t)i * B * B;
    }
    if (tape) {  // reflectors and R factors of this step go to the tape
      Vh = tape->Vy(i);
      TwV = tape->Ty(i);
      RV = tape->Ry(i);
      Uh = tape->Vu(i);
      TwU = tape->Tu(i);
      RU = tape->Ru(i);
    }
    if (r0 + B < M && r0 + B < N) {
      const double* Gi = G + (int64_t)i * Bp * ldg;
      // Sampling matrix Y = (X^T X)^q X^T G_i (b + p columns).
      // With pre-split operands the intermediate samples stay unreduced: each
      // next product's pre-split sums their partials (fuse); the last Y is
      // reduced into Y for the panel.
      const bool fuse = use_ps && (ps == PREC_BF16X3 || ps == PREC_BF16X6);
      SplitKeep kY{}, kZ{};
      HIPCHK(gemm_ps(ps, true, false, Ni, Bp, Mi, 1.0, X, ldt, Gi, ldg, 0.0, Y, N, split, se,
                     false, true, nullptr, fuse && q > 0 ? &kY : nullptr));
      for (int it = 0; it < q; ++it) {
        HIPCHK(gemm_ps(ps, false, false, Mi, Bp, Ni, 1.0, X, ldt, Y, N, 0.0, Z, M, split, se,
                       false, true, fuse ? &kY : nullptr, fuse ? &kZ : nullptr));
        HIPCHK(gemm_ps(ps, true, false, Ni, Bp, Mi, 1.0, X, ldt, Z, M, 0.0, Y, N, split, se,
                       false, true, fuse ? &kZ : nullptr, fuse && it + 1 < q ? &kY : nullptr));
      }
      if (p > 0) HIPCHK(oversample_basis(st, Ni, B, Bp, Y, N, L, base, intsY + (size_t)i * kIntsY,
                                         hw, pw, split, se, &blk->svd_fail));
      // Householder QR of Y: the right transform's reflectors.
      HIPCHK(reclaim(kVD + sl, vpend[sl]));
      HIPCHK(panel_qr_hr(st, Ni, B, Y, N, Vh, N, RV, B, tauV, TwV, B, hw, pw, split, se));
      // Right transform of T's trailing columns, all m rows.
      double* TJ = T + (int64_t)r0 * ldt;
      HIPCHK(gemm_ps(pu, false, false, M, B, Ni, 1.0, TJ, ldt, Vh, N, 0.0, W, M, split, se, false, true));
      HIPCHK(gemm(st, PREC_FP64, false, false, M, B, B, 1.0, W, M, TwV, B, 0.0, W2, M, nullptr, 0));
      HIPCHK(gemm_ps(pu, false, true, M, Ni, B, -1.0, W2, M, Vh, N, 1.0, TJ, ldt, nullptr, 0, true, true));
      if (formV) {  // V(:, J) = V(:, J) Vq, on the U / V stream
        double* VJ = V + (int64_t)r0 * ldv;
        HIPCHK(to_side(kVR + sl));
        HIPCHK(gemm_side(ss, false, false, N, B, Ni, 1.0, VJ, ldv, Vh, N, 0.0, Ws, MN, side_chunk));
        HIPCHK(gemm(ss, PREC_FP64, false, false, N, B, B, 1.0, Ws, MN, TwV, B, 0.0, W2s, MN, nullptr, 0));
        HIPCHK(gemm_side(ss, false, true, N, Ni, B, -1.0, W2s, MN, Vh, N, 1.0, VJ, ldv, kSideChunkUpd));
        HIPCHK(side_done(kVD + sl, &vpend[sl]));
      }
      // Householder QR of the new block column (rows I2, I3): the left
      // transform's reflectors and the diagonal block's R.
      // (The panel is read in place; T([I2,I3], J2) is overwritten below.)
      HIPCHK(reclaim(kUD + sl, upend[sl]));
      HIPCHK(panel_qr_hr(st, Mi, B, X, ldt, Uh, ldUh, RU, B, tauU, TwU, B, hw, pw, split, se));
      if (econU) ++nrefl;
      // Left transform of the trailing rows right of the block.
      const int Nr = Ni - B;
      double* XJ3 = X + (int64_t)B * ldt;
      HIPCHK(gemm_ps(pu, true, false, B, Nr, Mi, 1.0, Uh, ldUh, XJ3, ldt, 0.0, C, B, split, se, true, false));
      HIPCHK(gemm(st, PREC_FP64, true, false, B, Nr, B, 1.0, TwU, B, C, B, 0.0, C2, B, nullptr, 0));
      HIPCHK(gemm_ps(pu, false, false, Mi, Nr, B, -1.0, Uh, ldUh, C2, B, 1.0, XJ3, ldt, nullptr, 0, true, true));
      // U's trailing columns times the left transform (forward accumulation)
      if (formU && !econU) {  // on the U / V stream
        double* UI = U + (int64_t)r0 * ldu;
        HIPCHK(to_side(kUR + sl));
        HIPCHK(gemm_side(ss, false, false, M, B, Mi, 1.0, UI, ldu, Uh, M, 0.0, Ws, MN, side_chunk));
        HIPCHK(gemm(ss, PREC_FP64, false, false, M, B, B, 1.0, Ws, MN, TwU, B, 0.0, W2s, MN, nullptr, 0));
        HIPCHK(gemm_side(ss, false, true, M, Mi, B, -1.0, W2s, MN, Uh, M, 1.0, UI, ldu, kSideChunkUpd));
        HIPCHK(side_done(kUD + sl, &upend[sl]));
      }
      // T([I2,I3], J2) = [R; 0]; R moves to the stash, the diagonal block is
      // written from the SVD after the loop.
      HIPCHK(set_zero(st, Mi, B, X, ldt));
      ++nsvd;
      bool stop = k_stop > 0 && r0 + B >= k_stop;
      if (!stop && tol > 0.0) {
        HIPCHK(sumsq(st, Mi - B, Ni - B, X + B + (int64_t)B * ldt, ldt, nrm + 16, nrm + 1));
        double h = 0.0;
        HIPCHK(hipMemcpyAsync(&h, nrm + 1, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        stop = std::sqrt(h) <= tol * normA;
      }
      if (stop) {
        k_done = r0 + B;
        break;
      }
    } else if (Mi < Ni) {
      // Last block with fewer rows than columns (the paper's remark on the
      // case m < n): an LQ of the block row T(I2, [J2,J3]) as the Householder
      // QR of its transpose (copied into Y), so T(I2, J) = [L, 0] H^T with
      // L = R^T.  H acts from the right on the rows above the block and on V;
      // L goes to the stash for the batched SVD, whose right singular vectors
      // fold into the first Mi columns of J as for any other block.
      const int c = Mi;
      double* TJ = T + (int64_t)r0 * ldt;
      hipLaunchKernelGGL(k_transpose, dim3(grid_blocks((int64_t)Mi * Ni)), dim3(256), 0, st, Mi,
                         Ni, X, ldt, Y, (int64_t)N);
      HIPCHK(hipGetLastError());
      HIPCHK(reclaim(kVD + sl, vpend[sl]));
      HIPCHK(panel_qr_hr(st, Ni, c, Y, N, Vh, N, Ftmp, c, tauV, TwV, B, hw, pw, split, se));
      hipLaunchKernelGGL(k_transpose, dim3(grid_blocks((int64_t)c * c)), dim3(256), 0, st, c, c,
                         Ftmp, (int64_t)c, RU, (int64_t)B);
      HIPCHK(hipGetLastError());
      if (r0 > 0) {  // the rows above the block, times H
        HIPCHK(gemm(st, PREC_FP64, false, false, r0, c, Ni, 1.0, TJ, ldt, Vh, N, 0.0, W, M, split, se));
        HIPCHK(gemm(st, PREC_FP64, false, false, r0, c, c, 1.0, W, M, TwV, B, 0.0, W2, M, nullptr, 0));
        HIPCHK(gemm(st, PREC_FP64, false, true, r0, Ni, c, -1.0, W2, M, Vh, N, 1.0, TJ, ldt, nullptr, 0));
      }
      if (formV) {  // V(:, J) = V(:, J) H, on the U / V stream
        double* VJ = V + (int64_t)r0 * ldv;
        HIPCHK(to_side(kVR + sl));
        HIPCHK(gemm(ss, PREC_FP64, false, false, N, c, Ni, 1.0, VJ, ldv, Vh, N, 0.0, Ws, MN, nullptr, 0));
        HIPCHK(gemm(ss, PREC_FP64, false, false, N, c, c, 1.0, Ws, MN, TwV, B, 0.0, W2s, MN, nullptr, 0));
        HIPCHK(gemm(ss, PREC_FP64, false, true, N, Ni, c, -1.0, W2s, MN, Vh, N, 1.0, VJ, ldv, nullptr, 0));
        HIPCHK(side_done(kVD + sl, &vpend[sl]));
      }
      HIPCHK(set_zero(st, Mi, Ni, X, ldt));
      ++nsvd;
      last_w = c;
      k_done = M;
    } else {
      // Last block: economic SVD via Householder QR of T([I2,I3],[J2,J3]).
      const int c = Ni;
      HIPCHK(reclaim(kUD + sl, upend[sl]));
      HIPCHK(panel_qr_hr(st, Mi, c, X, ldt, Uh, ldUh, Rst + (size_t)i * B * B, B, tauU, TwU, B, hw,
                         pw, split, se));
      if (econU) ++nrefl;
      if (formU && !econU) {
        double* UI = U + (int64_t)r0 * ldu;
        HIPCHK(to_side(kUR + sl));
        HIPCHK(gemm(ss, PREC_FP64, false, false, M, c, Mi, 1.0, UI, ldu, Uh, M, 0.0, Ws, MN, nullptr, 0));
        HIPCHK(gemm(ss, PREC_FP64, false, false, M, c, c, 1.0, Ws, MN, TwU, B, 0.0, W2s, MN, nullptr, 0));
        HIPCHK(gemm(ss, PREC_FP64, false, true, M, Mi, c, -1.0, W2s, MN, Uh, M, 1.0, UI, ldu, nullptr, 0));
        HIPCHK(side_done(kUD + sl, &upend[sl]));
      }
      HIPCHK(set_zero(st, Mi, c, X, ldt));
      ++nsvd;
      last_w = c;
      k_done = n;
    }
  }

  auto join_side = [&]() -> hipError_t {
    if (!sc) return hipSuccess;
    hipError_t e = hipEventRecord(sc->ev[kJoin], ss);
    return e == hipSuccess ? hipStreamWaitEvent(st, sc->ev[kJoin], 0) : e;
  };
  if (tape) {  // truncated approximation: no small SVDs (U_k U_k^T does not see them)
    HIPCHK(join_side());
    HIPCHK(status_done(st, blk, k_done));
    if (k_out) *k_out = k_done;
    return 0;
  }
  // Batched SVDs of the stashed R blocks, then fold the rotations back:
  // T(I2,J2) = Ds, T(I2,J3) = Us^T T(I2,J3), T(I1,J2) = T(I1,J2) Vs,
  // U(:,I2) = U(:,I2) Us, V(:,J2) = V(:,J2) Vs.  The SVDs run while the
  // U / V stream finishes its last products; then T's part runs on the main
  // stream and U and V's part on the U / V stream.
  auto width = [&](int i) { return i == nsvd - 1 ? last_w : B; };
  // Economy U by backward accumulation: for block i (last first), the
  // columns right of it (already formed) times H_i = I - Uh_i Tw_i Uh_i^T,
  // then the block's own columns H_i [I_w; 0] in place of its reflectors.
  for (int i = nrefl - 1; i >= 0 && econU; --i) {
    const int r0 = i * B, w = width(i), mi = M - r0, rest = cU - r0 - w;
    const double* Uhi = U + r0 + (int64_t)r0 * ldu;
    const double* Twi = TwUst + (size_t)i * B * B;
    if (rest > 0) {
      double* Xr = U + r0 + (int64_t)(r0 + w) * ldu;
      HIPCHK(gemm(st, PREC_FP64, true, false, w, rest, mi, 1.0, Uhi, ldu, Xr, ldu, 0.0, C, w, split, se));
      HIPCHK(gemm(st, PREC_FP64, false, false, w, rest, w, 1.0, Twi, B, C, w, 0.0, C2, w, nullptr, 0));
      HIPCHK(gemm(st, PREC_FP64, false, false, mi, rest, w, -1.0, Uhi, ldu, C2, w, 1.0, Xr, ldu, nullptr, 0));
    }
    HIPCHK(gemm(st, PREC_FP64, false, true, w, w, w, 1.0, Twi, B, Uhi, ldu, 0.0, C2, w, nullptr, 0));
    HIPCHK(set_identity(st, mi, w, Ftmp, mi));
    HIPCHK(gemm(st, PREC_FP64, false, false, mi, w, w, -1.0, Uhi, ldu, C2, w, 1.0, Ftmp, mi, nullptr, 0));
    HIPCHK(copy_matrix(st, mi, w, Ftmp, mi, U + r0 + (int64_t)r0 * ldu, ldu));
  }
  hipLaunchKernelGGL(k_set_ints, dim3(1), dim3(256), 0, st, nbs, nsvd, B, last_w);
  HIPCHK(batched_svd(st, nsvd, nbs, B, Rst, (int64_t)B * B, Ust, Vst, (int64_t)B * B, Dd, B, Jw, Jv,
                     jstatus, kJacobiSweeps, &blk->svd_fail));
  // U and V's part of the fold-back on the U / V stream (once it has formed
  // them), beside T's part on the main stream; its products go through Ws.
  HIPCHK(to_side(kVR));
  for (int i = 0; i < nsvd && (formU || formV); ++i) {
    const int r0 = i * B, w = width(i);
    const double* Us = Ust + (size_t)i * B * B;
    const double* Vs = Vst + (size_t)i * B * B;
    if (formU) {
      double* blk = U + (int64_t)r0 * ldu;
      HIPCHK(gemm(ss, PREC_FP64, false, false, M, w, w, 1.0, blk, ldu, Us, B, 0.0, Ws, MN, nullptr, 0));
      HIPCHK(copy_matrix(ss, M, w, Ws, MN, blk, ldu));
    }
    if (formV) {
      double* blk = V + (int64_t)r0 * ldv;
      HIPCHK(gemm(ss, PREC_FP64, false, false, N, w, w, 1.0, blk, ldv, Vs, B, 0.0, Ws, MN, nullptr, 0));
      HIPCHK(copy_matrix(ss, N, w, Ws, MN, blk, ldv));
    }
  }
  for (int i = 0; i < nsvd; ++i) {
    const int r0 = i * B, w = width(i);
    const double* Us = Ust + (size_t)i * B * B;
    const double* Vs = Vst + (size_t)i * B * B;
    double* X = T + r0 + (int64_t)r0 * ldt;
    HIPCHK(set_diag_block(st, w, w, Dd + (size_t)i * B, X, ldt));
    const int nr = N - r0 - w;
    if (nr > 0) {
      double* blk = X + (int64_t)w * ldt;
      HIPCHK(gemm(st, PREC_FP64, true, false, w, nr, w, 1.0, Us, B, blk, ldt, 0.0, Ftmp, w, nullptr, 0));
      HIPCHK(copy_matrix(st, w, nr, Ftmp, w, blk, ldt));
    }
    if (r0 > 0) {
      double* blk = T + (int64_t)r0 * ldt;
      HIPCHK(gemm(st, PREC_FP64, false, false, r0, w, w, 1.0, blk, ldt, Vs, B, 0.0, Ftmp, r0, nullptr, 0));
      HIPCHK(copy_matrix(st, r0, w, Ftmp, r0, blk, ldt));
    }
  }
  HIPCHK(join_side());
  HIPCHK(status_done(st, blk, k_done));
  if (k_out) {
    *k_out = k_done;
    return read_status(base, nullptr, st);
  }
  return 0;
}

}  // namespace rutv

extern "C" {

int randutv_gemm(int prec, int ta, int tb, int64_t M, int64_t N, int64_t K, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc, void* work, size_t work_bytes, void* stream) {
  // Arithmetic: RANDUTV_FP64, _FP32, _BF16X3, or 4 for BF16x6.
  if (prec < 0 || prec > 4 || prec == 3) return -1;
  const Prec gp = prec == 4 ? PREC_BF16X6 : (Prec)prec;
  if (M < 0 || M > INT32_MAX) return -4;
  if (N < 0 || N > INT32_MAX) return -5;
  if (K < 0 || K > INT32_MAX) return -6;
  const int64_t arows = ta ? K : M, brows = tb ? N : K;
  if (M > 0 && N > 0 && K > 0) {
    if (!A || lda < std::max<int64_t>(1, arows)) return -8;
    if (!B || ldb < std::max<int64_t>(1, brows)) return -10;
  }
  if (M > 0 && N > 0 && (!C || ldc < M)) return -13;
  hipError_t e = gemm((hipStream_t)stream, gp, ta != 0, tb != 0, (int)M, (int)N, (int)K,
                      alpha, A, lda, B, ldb, beta, C, ldc, (double*)work,
                      work ? work_bytes / sizeof(double) : 0);
  return e == hipSuccess ? 0 : RANDUTV_E_HIP - (int)e;
}

size_t randutv_panel_work_size(int64_t Mp, int64_t nb) {
  if (nb < 1 || nb > kMaxB || Mp < nb || Mp > kMaxPanelRows) return 0;
  return al256(panel_work_bytes((int)nb)) + al256(hr_work_bytes(Mp, (int)nb)) +
         al256((size_t)Mp * nb * sizeof(double)) + al256((size_t)nb * nb * sizeof(double)) +
         al256((size_t)kMaxSplitKSmall * nb * nb * sizeof(double));
}

int randutv_panel_qr(int64_t Mp, int64_t nb, double* P, int64_t ldp, double* tau, double* Tw,
                     int64_t ldtw, int* used_fallback, void* work, size_t work_bytes,
                     void* stream) {
  if (Mp < 1 || Mp > kMaxPanelRows) return -1;
  if (nb < 1 || nb > kMaxB || nb > Mp) return -2;
  if (!P || ldp < Mp) return -3;
  if (!tau) return -5;
  if (!Tw || ldtw < nb) return -6;
  if (!work || ((uintptr_t)work & 255) || work_bytes < randutv_panel_work_size(Mp, nb))
    return -9;
  char* base = (char*)work;
  PanelWork pw;
  panel_work_carve(base, (int)nb, &pw);
  base += al256(panel_work_bytes((int)nb));
  HrWork hw;
  hr_work_carve(base, Mp, (int)nb, &hw);
  base += al256(hr_work_bytes(Mp, (int)nb));
  double* V = (double*)base;
  base += al256((size_t)Mp * nb * sizeof(double));
  double* R = (double*)base;
  base += al256((size_t)nb * nb * sizeof(double));
  double* split = (double*)base;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, pw.err);
  hipError_t e = panel_qr_hr(st, (int)Mp, (int)nb, P, ldp, V, Mp, R, nb, tau, Tw, ldtw, hw, pw,
                             split, (size_t)kMaxSplitKSmall * nb * nb);
  if (e == hipSuccess) e = pack_qr(st, (int)Mp, (int)nb, V, Mp, R, nb, P, ldp);
  if (e != hipSuccess) return RANDUTV_E_HIP - (int)e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return RANDUTV_E_HIP - (int)e;
  int err = 0, fb = 0;
  e = hipMemcpy(&err, pw.err, sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&fb, hw.flag, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return RANDUTV_E_HIP - (int)e;
  if (used_fallback) *used_fallback = fb;
  return err ? RANDUTV_E_SYNC : 0;
}

size_t randutv_small_svd_work_size(int64_t count, int64_t ld) {
  if (count < 1 || ld < 1 || ld > 1024) return 0;
  return al256((size_t)2 * count * ld * ld * sizeof(double)) +
         al256((size_t)(2 + kJacobiSweeps) * count * sizeof(int));
}

int randutv_small_svd(int64_t count, const int* nbs, int64_t ld, const double* R, double* Us,
                      double* Vs, double* D, void* work, size_t work_bytes, void* stream) {
  if (count < 1) return -1;
  if (!nbs) return -2;
  if (ld < 1 || ld > 1024) return -3;
  for (int64_t i = 0; i < count; ++i)
    if (nbs[i] < 1 || nbs[i] > ld) return -2;
  if (!R) return -4;
  if (!Us) return -5;
  if (!Vs) return -6;
  if (!D) return -7;
  const size_t need = randutv_small_svd_work_size(count, ld);
  if (!work || ((uintptr_t)work & 255) || work_bytes < need) return -8;
  hipStream_t st = (hipStream_t)stream;
  double* Jw = (double*)work;
  double* Jv = Jw + (size_t)count * ld * ld;
  int* ints = (int*)((char*)work + al256((size_t)2 * count * ld * ld * sizeof(double)));
  hipError_t e = hipMemcpyAsync(ints, nbs, count * sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = batched_svd(st, (int)count, ints, (int)ld, R, ld * ld, Us, Vs, ld * ld, D, ld, Jw, Jv,
                    ints + count, kJacobiSweeps, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return RANDUTV_E_HIP - (int)e;
  std::vector<int> js(count);
  e = hipMemcpy(js.data(), ints + count, count * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return RANDUTV_E_HIP - (int)e;
  for (int v : js)
    if (v < 0) return 1;
  return 0;
}

}  // extern "C"
