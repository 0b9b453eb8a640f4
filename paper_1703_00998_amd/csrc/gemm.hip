// Thin-matrix GEMMs of randUTV on CDNA4 matrix cores.
//
// The paper puts almost all of randUTV's flops in products of the m x n
// working matrix with thin b-column matrices (Section 1.1 (iii), Section
// 5.4): the sampling products X^T G, X Y, X^T Z and the two block-reflector
// updates.  They are compute-bound in FP64 (b/4 flop per byte against a
// ridge near 10 at b = 256), so they run on v_mfma_f64_16x16x4_f64.
//
// Kernel shape: a 256-thread workgroup computes a 64 x 64 tile of C; each
// of its four waves owns a 32 x 32 quarter as 2 x 2 MFMA 16 x 16 blocks.
// K is walked in 16-deep slabs staged through double-buffered LDS with the
// next slab prefetched into registers while the current one is multiplied.
// The MFMA is issued as C^T = op(B)^T op(A)^T so that the 16 lanes sharing
// an output column hold 16 consecutive rows of the column-major C (128-byte
// coalesced stores).  Long reductions are split over blockIdx.z into FP64
// partials that a second kernel sums in a fixed order (bit-reproducible).
#include <algorithm>

#include "common.h"

namespace rutv {
namespace {

constexpr int BK = 16, PAD = 2;

__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// BM x BN output tile per 256-thread workgroup; 2 x 2 waves, each owning a
// (BM/2) x (BN/2) quarter as (BM/32) x (BN/32) MFMA 16 x 16 blocks.  The
// occupancy hint keeps registers low enough for two workgroups per CU, so
// one workgroup's loads overlap the other's MFMAs (measured: 128 x 128 tiles
// at 51-55 TFLOP/s on the n = 8000 shapes vs 20-26 without the hint).
template <bool TA, bool TB, int BM, int BN>
__global__ __launch_bounds__(256, 2) void k_dgemm(int M, int N, int K, int kper,
                                               const double* __restrict__ A, int64_t lda,
                                               const double* __restrict__ B, int64_t ldb,
                                               double* __restrict__ C, int64_t ldc,
                                               int64_t zstride, double alpha, double beta) {
  constexpr int FM = BM / 32, FN = BN / 32;       // MFMA blocks per wave
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;  // elements per thread
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * kper;
  const int kend = min(K, kbeg + kper);
  if (gridDim.z > 1) C += (int64_t)blockIdx.z * zstride;

  // Element r of this thread's share of the A (BM x BK) and B (BK x BN)
  // slabs, chosen so that consecutive threads read consecutive addresses.
  auto a_idx = [&](int r, int& i, int& k) {
    if (!TA) { i = tid % BM; k = tid / BM + (256 / BM) * r; }
    else     { k = tid % BK; i = tid / BK + (256 / BK) * r; }
  };
  auto b_idx = [&](int r, int& k, int& j) {
    if (!TB) { k = tid % BK; j = tid / BK + (256 / BK) * r; }
    else     { j = tid % BN; k = tid / BN + (256 / BN) * r; }
  };
  double ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      int i, k;
      a_idx(r, i, k);
      const int gi = m0 + i, gk = k0 + k;
      ra[r] = (gi < M && gk < kend) ? (TA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      int k, j;
      b_idx(r, k, j);
      const int gj = n0 + j, gk = k0 + k;
      rb[r] = (gj < N && gk < kend) ? (TB ? B[gj + (int64_t)gk * ldb] : B[gk + (int64_t)gj * ldb]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      int i, k;
      a_idx(r, i, k);
      As[buf][k][i] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      int k, j;
      b_idx(r, k, j);
      Bs[buf][k][j] = rb[r];
    }
  };

  v4d acc[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  const int kr = lane >> 4, cr = lane & 15;
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) load(kbeg + (t + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a[FM], b[FN];
#pragma unroll
      for (int x = 0; x < FM; ++x) a[x] = As[cur][kk + kr][wm * (BM / 2) + x * 16 + cr];
#pragma unroll
      for (int y = 0; y < FN; ++y) b[y] = Bs[cur][kk + kr][wn * (BN / 2) + y * 16 + cr];
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfma64(b[y], a[x], acc[x][y]);
    }
    if (t + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
  // v_mfma_f64_16x16x4f64 leaves D(row = (lane>>4) + 4r, col = lane&15) in
  // register r of each lane; D is C^T here, so
  // acc[x][y][r] = C(row = m0 + wm*BM/2 + x*16 + (lane&15),
  //                  col = n0 + wn*BN/2 + y*16 + (lane>>4) + 4r)
#pragma unroll
  for (int x = 0; x < FM; ++x) {
    const int row = m0 + wm * (BM / 2) + x * 16 + cr;
    if (row >= M) continue;
#pragma unroll
    for (int y = 0; y < FN; ++y) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = n0 + wn * (BN / 2) + y * 16 + kr + 4 * r;
        if (col < N) {
          double* p = C + row + (int64_t)col * ldc;
          double v = alpha * acc[x][y][r];
          if (beta != 0.0) v += beta * *p;
          *p = v;
        }
      }
    }
  }
}

__global__ void k_splitk_reduce(int M, int N, int S, const double* __restrict__ P,
                                int64_t zstride, double* __restrict__ C, int64_t ldc,
                                double alpha, double beta) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M);
    const int64_t j = idx / M;
    double s = 0.0;
    for (int z = 0; z < S; ++z) s += P[z * zstride + idx];
    double* p = C + i + j * ldc;
    double v = alpha * s;
    if (beta != 0.0) v += beta * *p;
    *p = v;
  }
}

template <bool TA, bool TB, int BM, int BN>
void launch(hipStream_t st, dim3 grid, int M, int N, int K, int kper, const double* A,
            int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
            int64_t zstride, double alpha, double beta) {
  hipLaunchKernelGGL((k_dgemm<TA, TB, BM, BN>), grid, dim3(256), 0, st, M, N, K, kper, A, lda,
                     B, ldb, C, ldc, zstride, alpha, beta);
}

template <int BM, int BN>
void launch_t(hipStream_t st, bool ta, bool tb, dim3 grid, int M, int N, int K, int kper,
              const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
              int64_t ldc, int64_t zs, double al, double be) {
  if (!ta && !tb) launch<false, false, BM, BN>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be);
  else if (ta && !tb) launch<true, false, BM, BN>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be);
  else if (!ta && tb) launch<false, true, BM, BN>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be);
  else launch<true, true, BM, BN>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be);
}

}  // namespace

hipError_t gemm(hipStream_t st, Prec prec, bool ta, bool tb, int M, int N, int K,
                double alpha, const double* A, int64_t lda, const double* B,
                int64_t ldb, double beta, double* C, int64_t ldc, double* splitws,
                size_t splitws_elems) {
  (void)prec;
  if (M <= 0 || N <= 0) return hipSuccess;
  // 128 x 128 tiles when the output, or the output times a split of K,
  // gives enough workgroups; else 64 x 64.  Long reductions are split over
  // blockIdx.z until about two workgroups per CU are in flight.
  const int64_t t128 = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
  const bool big = t128 >= 384 || (splitws && K >= 2048 && t128 * std::min(8, K / 512) >= 384);
  const int BMs = big ? 128 : 64, BNs = big ? 128 : 64;
  const int tm = (M + BMs - 1) / BMs, tn = (N + BNs - 1) / BNs;
  const int tiles = tm * tn;
  int splits = 1;
  if (splitws && tiles < 512 && K >= 1024) {
    splits = (512 + tiles - 1) / tiles;
    splits = std::min(splits, K / 512);
    splits = std::min(splits, kMaxSplitK);
    while (splits > 1 && (size_t)splits * M * N > splitws_elems) --splits;
    if (splits < 1) splits = 1;
  }
  int kper = (K + splits - 1) / splits;
  kper = (kper + BK - 1) / BK * BK;
  if (kper <= 0) kper = BK;
  splits = K > 0 ? (K + kper - 1) / kper : 1;
  dim3 grid(tm, tn, splits);
  double* Cout = C;
  int64_t ldo = ldc, zs = 0;
  double al = alpha, be = beta;
  if (splits > 1) {
    Cout = splitws;
    ldo = M;
    zs = (int64_t)M * N;
    al = 1.0;
    be = 0.0;
  }
  const int slot = prof_mark(st);
  if (big) launch_t<128, 128>(st, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else launch_t<64, 64>(st, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  prof_done(st, slot, ta ? (tb ? PC_GEMM_TT : PC_GEMM_TN) : (tb ? PC_GEMM_NT : PC_GEMM_NN),
            2.0 * M * N * (double)K);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  const int64_t total = (int64_t)M * N;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  const int slot2 = prof_mark(st);
  hipLaunchKernelGGL(k_splitk_reduce, dim3(blocks), dim3(256), 0, st, M, N, splits, splitws,
                     zs, C, ldc, alpha, beta);
  prof_done(st, slot2, PC_SPLITK, (double)splits * M * N);
  return hipGetLastError();
}

}  // namespace rutv
