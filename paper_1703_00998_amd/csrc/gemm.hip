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

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;

__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm(int M, int N, int K, int kper,
                                               const double* __restrict__ A, int64_t lda,
                                               const double* __restrict__ B, int64_t ldb,
                                               double* __restrict__ C, int64_t ldc,
                                               int64_t zstride, double alpha, double beta) {
  __shared__ double As[2][BK][BM + PAD];
  __shared__ double Bs[2][BK][BN + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * kper;
  const int kend = min(K, kbeg + kper);
  if (gridDim.z > 1) C += (int64_t)blockIdx.z * zstride;

  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i, k;
      if (!TA) { i = tid & 63; k = (tid >> 6) + 4 * r; }
      else     { k = tid & 15; i = (tid >> 4) + 16 * r; }
      const int gi = m0 + i, gk = k0 + k;
      ra[r] = (gi < M && gk < kend) ? (TA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : 0.0;
      int j;
      if (!TB) { k = tid & 15; j = (tid >> 4) + 16 * r; }
      else     { j = tid & 63; k = (tid >> 6) + 4 * r; }
      const int gj = n0 + j, gk2 = k0 + k;
      rb[r] = (gj < N && gk2 < kend) ? (TB ? B[gj + (int64_t)gk2 * ldb] : B[gk2 + (int64_t)gj * ldb]) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i, k;
      if (!TA) { i = tid & 63; k = (tid >> 6) + 4 * r; }
      else     { k = tid & 15; i = (tid >> 4) + 16 * r; }
      As[buf][k][i] = ra[r];
      int j;
      if (!TB) { k = tid & 15; j = (tid >> 4) + 16 * r; }
      else     { j = tid & 63; k = (tid >> 6) + 4 * r; }
      Bs[buf][k][j] = rb[r];
    }
  };

  v4d acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = v4d{0.0, 0.0, 0.0, 0.0};

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
      const double a0 = As[cur][kk + kr][wm * 32 + cr];
      const double a1 = As[cur][kk + kr][wm * 32 + 16 + cr];
      const double b0 = Bs[cur][kk + kr][wn * 32 + cr];
      const double b1 = Bs[cur][kk + kr][wn * 32 + 16 + cr];
      acc[0][0] = mfma64(b0, a0, acc[0][0]);
      acc[0][1] = mfma64(b1, a0, acc[0][1]);
      acc[1][0] = mfma64(b0, a1, acc[1][0]);
      acc[1][1] = mfma64(b1, a1, acc[1][1]);
    }
    if (t + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
  // v_mfma_f64_16x16x4f64 leaves D(row = (lane>>4) + 4r, col = lane&15) in
  // register r of each lane; D is C^T here, so
  // acc[x][y][r] = C(row = m0 + wm*32 + x*16 + (lane&15),
  //                  col = n0 + wn*32 + y*16 + (lane>>4) + 4r)
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int row = m0 + wm * 32 + x * 16 + cr;
    if (row >= M) continue;
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = n0 + wn * 32 + y * 16 + kr + 4 * r;
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

template <bool TA, bool TB>
void launch(hipStream_t st, dim3 grid, int M, int N, int K, int kper, const double* A,
            int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
            int64_t zstride, double alpha, double beta) {
  hipLaunchKernelGGL((k_dgemm<TA, TB>), grid, dim3(256), 0, st, M, N, K, kper, A, lda, B,
                     ldb, C, ldc, zstride, alpha, beta);
}

}  // namespace

hipError_t gemm(hipStream_t st, Prec prec, bool ta, bool tb, int M, int N, int K,
                double alpha, const double* A, int64_t lda, const double* B,
                int64_t ldb, double beta, double* C, int64_t ldc, double* splitws,
                size_t splitws_elems) {
  (void)prec;
  if (M <= 0 || N <= 0) return hipSuccess;
  const int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  const int tiles = tm * tn;
  int splits = 1;
  if (splitws && tiles < 512 && K >= 1024) {
    splits = (1024 + tiles - 1) / tiles;
    splits = min(splits, K / 512);
    splits = min(splits, kMaxSplitK);
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
  if (!ta && !tb) launch<false, false>(st, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else if (ta && !tb) launch<true, false>(st, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else if (!ta && tb) launch<false, true>(st, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else launch<true, true>(st, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
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
