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
#include <type_traits>

#include "common.h"

namespace rutv {
namespace {

constexpr int PAD = 2;
#ifndef K64_SLAB
#define K64_SLAB 16
#endif
constexpr int kSmallMN = 128;  // products at most this size in M and N
constexpr int kSmallK = 512;   // and this deep go to k_gemm_small (FP64)

__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline v4f mfma32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfmabf(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// K depth of one LDS slab: 16 for the FP64 and FP32 MFMAs (16x16x4), 32 for
// the BF16 ones (16x16x32).  32-deep slabs on the 64 x 64 FP64 tiles (67 KB
// of LDS per workgroup) made the 8000 x 8000 factorization 8-10 ms slower.
template <int P, int BM>
constexpr int slab_k() {
  return (P == PREC_BF16X3 || P == PREC_BF16X6) ? 32 : (BM <= 64 ? K64_SLAB : 16);
}

// LDS slabs of one K step, per arithmetic.  FP64/FP32: [k][i] with i
// contiguous (MFMA 16x16x4 takes one element per lane).  BF16 pieces:
// [k/8][i][k%8] so that each lane reads its 8 consecutive k values of row i
// (the bf16 MFMA operand) as one 16-byte load.  NB buffers: two (the next
// slab is stored while the current one is multiplied) except for the
// three-piece BF16x6 slabs of 128 x 128 tiles, whose single buffer (48 KB)
// keeps two workgroups per CU.  (A single buffer for the U / V stream's FP64
// products, 17 KB, so that a panel kernel's 142 KB fit on a CU beside one of
// them, made the panels' Cholesky kernels 2 ms faster per factorization but
// the whole 3 ms slower.)
template <int P, int BM, int BN, int NB>
struct Slabs;
template <int BM, int BN, int NB>
struct Slabs<PREC_FP64, BM, BN, NB> {
  double A[NB][slab_k<PREC_FP64, BM>()][BM + PAD];
  double B[NB][slab_k<PREC_FP64, BM>()][BN + PAD];
};
template <int BM, int BN, int NB>
struct Slabs<PREC_FP32, BM, BN, NB> {
  float A[NB][slab_k<PREC_FP32, BM>()][BM + PAD];
  float B[NB][slab_k<PREC_FP32, BM>()][BN + PAD];
};
template <int BM, int BN, int NB>
struct Slabs<PREC_BF16X3, BM, BN, NB> {
  alignas(16) __bf16 Ah[NB][4][BM][8];
  alignas(16) __bf16 Al[NB][4][BM][8];
  alignas(16) __bf16 Bh[NB][4][BN][8];
  alignas(16) __bf16 Bl[NB][4][BN][8];
};
template <int BM>
constexpr int bf6_bufs() { return BM >= 128 ? 1 : 2; }
template <int BM, int BN, int NB>
struct Slabs<PREC_BF16X6, BM, BN, NB> {
  alignas(16) __bf16 Ah[NB][4][BM][8];
  alignas(16) __bf16 Am[NB][4][BM][8];
  alignas(16) __bf16 Al[NB][4][BM][8];
  alignas(16) __bf16 Bh[NB][4][BN][8];
  alignas(16) __bf16 Bm[NB][4][BN][8];
  alignas(16) __bf16 Bl[NB][4][BN][8];
};

// fl32(x): x rounded to FP32 (to nearest), held as a float.  The empty asm
// keeps the compiler from merging this rounding with a following rounding
// to BF16 into one direct FP64 -> BF16 rounding (through a round-to-odd
// FP32, a handful of extra instructions per value), which it does in some
// contexts and not in others: with it every loader and k_presplit take the
// BF16 pieces of the same FP32 value, as written.
__device__ inline float fl32(double x) {
  float r = (float)x;
  asm volatile("" : "+v"(r));
  return r;
}

// x ~ h + m + l in bf16, from x32 = fl32(x): each piece is the bf16 rounding
// of what the earlier ones leave (the remainders are exact in FP32), so the
// three carry about 24 significant bits.
struct Bf3 {
  __bf16 h, m, l;
};
__device__ inline Bf3 split3(float x32) {
  const __bf16 h = (__bf16)x32;
  const float r1 = x32 - (float)h;
  const __bf16 m = (__bf16)r1;
  const float r2 = r1 - (float)m;
  return Bf3{h, m, (__bf16)r2};
}

// BM x BN output tile per workgroup of WM x WN waves, each owning a
// (BM/WM) x (BN/WN) part as MFMA 16 x 16 blocks.  The 128 x 128 and 64 x 64
// tiles use 2 x 2 waves with an occupancy hint for two workgroups per CU,
// so one workgroup's loads overlap the other's MFMAs (measured in FP64:
// 128 x 128 tiles at 51-55 TFLOP/s on the n = 8000 shapes vs 20-26 without
// it).  Operands are FP64 in memory for every arithmetic; the loader
// converts.
// ROLE tells apart instantiations of the same code, so that kernel traces
// and counters attribute them separately: 0 for the method's thin products
// on the main stream (sampling, trailing updates, fold-back of T), 1 for the
// products inside the Householder panel factorizations, 2 for the U / V
// stream's products.
template <int P, bool TA, bool TB, int BM, int BN, int WM, int WN, int ROLE>
__global__ __launch_bounds__(64 * WM * WN, WM * WN <= 8 ? 2 : 1) void k_gemm(
    int M, int N, int K, int kper, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ B, int64_t ldb, double* __restrict__ C, int64_t ldc,
    int64_t zstride, double alpha, double beta, PsOps ps) {
  constexpr int NT = 64 * WM * WN;                     // threads
  constexpr int BK = slab_k<P, BM>();
  constexpr int PM = BM / WM, PN = BN / WN;            // per-wave part
  constexpr int FM = PM / 16, FN = PN / 16;            // MFMA blocks per wave
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;  // elements per thread
  static_assert(LA * NT == BM * BK && LB * NT == BN * BK, "loader shape");
  static_assert(NT % BM == 0 && NT % BN == 0 && NT % BK == 0, "loader shape");
  constexpr int NBUF = P == PREC_BF16X6 ? bf6_bufs<BM>() : 2;
  __shared__ Slabs<P, BM, BN, NBUF> sl;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  // Tile order.  Workgroups go to the 8 XCDs round-robin by linear id, and
  // each XCD has its own L2.  Linear id L runs on XCD L % 8 as that XCD's
  // (L / 8)-th workgroup; giving every XCD one contiguous range of the tile
  // sequence, walked down groups of 8 tile rows, keeps the workgroups that
  // one XCD holds at once on a compact patch of C, so the A row-tiles and B
  // column-tiles they read are shared in that XCD's L2.
  const int tm = gridDim.x, tn = gridDim.y;
  const int tiles = tm * tn, total = tiles * (int)gridDim.z;
  const int lin = blockIdx.x + tm * (blockIdx.y + tn * (int)blockIdx.z);
  const int xcd = lin & 7, per = total >> 3, extra = total & 7;
  const int seq = xcd * per + min(xcd, extra) + (lin >> 3);
  const int bz = seq / tiles, rem = seq - bz * tiles;
  constexpr int kGroup = 8;
  const int g0 = rem / (kGroup * tn) * kGroup;
  const int gsz = min(kGroup, tm - g0);
  const int gi = rem - g0 * tn;
  const int m0 = (g0 + gi % gsz) * BM, n0 = (gi / gsz) * BN;
  const int kbeg = bz * kper;
  const int kend = min(K, kbeg + kper);
  if (gridDim.z > 1) C += (int64_t)bz * zstride;

  // Element r of this thread's share of the A (BM x BK) and B (BK x BN)
  // slabs, chosen so that consecutive threads read consecutive addresses.
  auto a_idx = [&](int r, int& i, int& k) {
    if (!TA) { i = tid % BM; k = tid / BM + (NT / BM) * r; }
    else     { k = tid % BK; i = tid / BK + (NT / BK) * r; }
  };
  auto b_idx = [&](int r, int& k, int& j) {
    if (!TB) { k = tid % BK; j = tid / BK + (NT / BK) * r; }
    else     { j = tid % BN; k = tid / BN + (NT / BN) * r; }
  };
  // The prefetch registers hold the FP64 operands as loaded; the conversion
  // waits until the slab is stored to LDS, after the current slab's MFMAs,
  // so the loads stay in flight under them (converting at load time exposed
  // their latency: the 128 x 128 split-precision products ran 1.3-2.8x
  // slower).
  using LoadT = double;
  LoadT ra[LA], rb[LB];
  // Operands given as BF16 pieces (ROLE bit 2: A, bit 3: B): 16-byte chunks
  // of 8 consecutive k of one row, already in the LDS layout; CA (CB)
  // chunks per thread and piece per slab.
  constexpr bool PSA = (ROLE & 4) != 0, PSB = (ROLE & 8) != 0;
  static_assert(!(PSA || PSB) || P == PREC_BF16X3 || P == PREC_BF16X6, "pre-split operands are BF16");
  constexpr int NPC = P == PREC_BF16X6 ? 3 : 2;
  constexpr int CA = PSA ? 4 * BM / NT : 1, CB = PSB ? 4 * BN / NT : 1;
  static_assert(!PSA || CA * NT == 4 * BM, "pre-split A chunks");
  static_assert(!PSB || CB * NT == 4 * BN, "pre-split B chunks");
  uint4 pa[PSA ? NPC : 1][CA], pb[PSB ? NPC : 1][CB];
  // Slabs that lie wholly inside A (or B) take a path without per-element
  // guards: element r sits at a fixed offset from the thread's first one
  // (r * rsA, resp. r * rsB), and a slab moves by k0 * ksA (ksB).  The guards
  // compile to exec-mask branches around every load and keep the compiler
  // from interleaving the loads with the MFMAs.
  int a_i0, a_k0, b_k0, b_j0;
  a_idx(0, a_i0, a_k0);
  b_idx(0, b_k0, b_j0);
  const int64_t offA = TA ? a_k0 + (int64_t)(m0 + a_i0) * lda : (m0 + a_i0) + (int64_t)a_k0 * lda;
  const int64_t rsA = TA ? (int64_t)(NT / BK) * lda : (int64_t)(NT / BM) * lda;
  const int64_t ksA = TA ? 1 : lda;
  const int64_t offB = TB ? (n0 + b_j0) + (int64_t)b_k0 * ldb : b_k0 + (int64_t)(n0 + b_j0) * ldb;
  const int64_t rsB = TB ? (int64_t)(NT / BN) * ldb : (int64_t)(NT / BK) * ldb;
  const int64_t ksB = TB ? ldb : 1;
  const bool rowsA = m0 + BM <= M, colsB = n0 + BN <= N;
  auto load = [&](int k0) {
    const bool kin = k0 + BK <= kend;
    if constexpr (PSA) {
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        const int c = tid + NT * u, kc = c / BM, r = c % BM;
        const bool in = m0 + r < M;
        const uint4* src = ps.a + ((int64_t)((k0 >> 3) + kc) * ps.rows_a + (m0 + r));
#pragma unroll
        for (int q = 0; q < NPC; ++q) pa[q][u] = in ? src[q * ps.piece_a] : uint4{0, 0, 0, 0};
      }
    } else if (rowsA && kin) {
      const double* pa = A + offA + (int64_t)k0 * ksA;
#pragma unroll
      for (int r = 0; r < LA; ++r) ra[r] = pa[r * rsA];
    } else {
#pragma unroll
      for (int r = 0; r < LA; ++r) {
        int i, k;
        a_idx(r, i, k);
        const int gi = m0 + i, gk = k0 + k;
        ra[r] = (gi < M && gk < kend) ? (TA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : 0.0;
      }
    }
    if constexpr (PSB) {
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = tid + NT * u, kc = c / BN, r = c % BN;
        const bool in = n0 + r < N;
        const uint4* src = ps.b + ((int64_t)((k0 >> 3) + kc) * ps.rows_b + (n0 + r));
#pragma unroll
        for (int q = 0; q < NPC; ++q) pb[q][u] = in ? src[q * ps.piece_b] : uint4{0, 0, 0, 0};
      }
    } else if (colsB && kin) {
      const double* pbb = B + offB + (int64_t)k0 * ksB;
#pragma unroll
      for (int r = 0; r < LB; ++r) rb[r] = pbb[r * rsB];
    } else {
#pragma unroll
      for (int r = 0; r < LB; ++r) {
        int k, j;
        b_idx(r, k, j);
        const int gj = n0 + j, gk = k0 + k;
        rb[r] = (gj < N && gk < kend) ? (TB ? B[gj + (int64_t)gk * ldb] : B[gk + (int64_t)gj * ldb]) : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
    if constexpr (PSA) {
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        const int c = tid + NT * u, kc = c / BM, r = c % BM;
        *(uint4*)&sl.Ah[buf][kc][r][0] = pa[0][u];
        if constexpr (P == PREC_BF16X6) {
          *(uint4*)&sl.Am[buf][kc][r][0] = pa[1][u];
          *(uint4*)&sl.Al[buf][kc][r][0] = pa[2][u];
        } else {
          *(uint4*)&sl.Al[buf][kc][r][0] = pa[1][u];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < LA; ++r) {
        int i, k;
        a_idx(r, i, k);
        if constexpr (P == PREC_FP64) sl.A[buf][k][i] = ra[r];
        else if constexpr (P == PREC_FP32) sl.A[buf][k][i] = (float)ra[r];
        else if constexpr (P == PREC_BF16X6) {
          const Bf3 x = split3(fl32(ra[r]));
          sl.Ah[buf][k >> 3][i][k & 7] = x.h;
          sl.Am[buf][k >> 3][i][k & 7] = x.m;
          sl.Al[buf][k >> 3][i][k & 7] = x.l;
        } else {
          const float x = fl32(ra[r]);
          const __bf16 h = (__bf16)x;
          sl.Ah[buf][k >> 3][i][k & 7] = h;
          sl.Al[buf][k >> 3][i][k & 7] = (__bf16)(x - (float)h);
        }
      }
    }
    if constexpr (PSB) {
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = tid + NT * u, kc = c / BN, r = c % BN;
        *(uint4*)&sl.Bh[buf][kc][r][0] = pb[0][u];
        if constexpr (P == PREC_BF16X6) {
          *(uint4*)&sl.Bm[buf][kc][r][0] = pb[1][u];
          *(uint4*)&sl.Bl[buf][kc][r][0] = pb[2][u];
        } else {
          *(uint4*)&sl.Bl[buf][kc][r][0] = pb[1][u];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < LB; ++r) {
        int k, j;
        b_idx(r, k, j);
        if constexpr (P == PREC_FP64) sl.B[buf][k][j] = rb[r];
        else if constexpr (P == PREC_FP32) sl.B[buf][k][j] = (float)rb[r];
        else if constexpr (P == PREC_BF16X6) {
          const Bf3 x = split3(fl32(rb[r]));
          sl.Bh[buf][k >> 3][j][k & 7] = x.h;
          sl.Bm[buf][k >> 3][j][k & 7] = x.m;
          sl.Bl[buf][k >> 3][j][k & 7] = x.l;
        } else {
          const float x = fl32(rb[r]);
          const __bf16 h = (__bf16)x;
          sl.Bh[buf][k >> 3][j][k & 7] = h;
          sl.Bl[buf][k >> 3][j][k & 7] = (__bf16)(x - (float)h);
        }
      }
    }
  };

  using AccT = typename std::conditional<P == PREC_FP64, v4d, v4f>::type;
  AccT acc[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y) acc[x][y] = AccT{0, 0, 0, 0};

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  const int kr = lane >> 4, cr = lane & 15;
  for (int t = 0; t < nk; ++t) {
    const int cur = NBUF == 2 ? (t & 1) : 0;
    if (t + 1 < nk) load(kbeg + (t + 1) * BK);
    if constexpr (P == PREC_BF16X6) {
      // Six products per block pair, small terms first: h m, m h, h l, l h,
      // m m, then h h (m l, l m, l l are below FP32's rounding and dropped).
      // B's three pieces are read once per slab, A's per 16-row block (the
      // register budget of two workgroups per CU holds no more).
      v8bf bh[FN], bm[FN], bl[FN];
#pragma unroll
      for (int y = 0; y < FN; ++y) {
        bh[y] = *(const v8bf*)&sl.Bh[cur][kr][wn * PN + y * 16 + cr][0];
        bm[y] = *(const v8bf*)&sl.Bm[cur][kr][wn * PN + y * 16 + cr][0];
        bl[y] = *(const v8bf*)&sl.Bl[cur][kr][wn * PN + y * 16 + cr][0];
      }
#pragma unroll
      for (int x = 0; x < FM; ++x) {
        const v8bf ah = *(const v8bf*)&sl.Ah[cur][kr][wm * PM + x * 16 + cr][0];
        const v8bf am = *(const v8bf*)&sl.Am[cur][kr][wm * PM + x * 16 + cr][0];
        const v8bf al = *(const v8bf*)&sl.Al[cur][kr][wm * PM + x * 16 + cr][0];
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bm[y], ah, acc[x][y]);
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bh[y], am, acc[x][y]);
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bl[y], ah, acc[x][y]);
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bh[y], al, acc[x][y]);
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bm[y], am, acc[x][y]);
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bh[y], ah, acc[x][y]);
      }
    } else if constexpr (P == PREC_BF16X3) {
      v8bf ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
      for (int x = 0; x < FM; ++x) {
        ah[x] = *(const v8bf*)&sl.Ah[cur][kr][wm * PM + x * 16 + cr][0];
        al[x] = *(const v8bf*)&sl.Al[cur][kr][wm * PM + x * 16 + cr][0];
      }
#pragma unroll
      for (int y = 0; y < FN; ++y) {
        bh[y] = *(const v8bf*)&sl.Bh[cur][kr][wn * PN + y * 16 + cr][0];
        bl[y] = *(const v8bf*)&sl.Bl[cur][kr][wn * PN + y * 16 + cr][0];
      }
      // One FP32 accumulator takes the two cross terms, then hi*hi; the
      // passes run over all blocks so consecutive MFMAs are independent.
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bh[y], al[x], acc[x][y]);
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bl[y], ah[x], acc[x][y]);
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = mfmabf(bh[y], ah[x], acc[x][y]);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        typename std::conditional<P == PREC_FP64, double, float>::type a[FM], b[FN];
#pragma unroll
        for (int x = 0; x < FM; ++x) a[x] = sl.A[cur][kk + kr][wm * PM + x * 16 + cr];
#pragma unroll
        for (int y = 0; y < FN; ++y) b[y] = sl.B[cur][kk + kr][wn * PN + y * 16 + cr];
#pragma unroll
        for (int x = 0; x < FM; ++x)
#pragma unroll
          for (int y = 0; y < FN; ++y) {
            if constexpr (P == PREC_FP64) acc[x][y] = mfma64(b[y], a[x], acc[x][y]);
            else acc[x][y] = mfma32(b[y], a[x], acc[x][y]);
          }
      }
    }
    if constexpr (NBUF == 2) {
      if (t + 1 < nk) store(cur ^ 1);
    } else {
      __syncthreads();  // every wave is done with the single buffer
      if (t + 1 < nk) store(0);
    }
    __syncthreads();
  }
  // The MFMA computes D = C^T.  v_mfma_f64_16x16x4f64 leaves D(row =
  // (lane>>4) + 4r, col = lane&15) in register r; the f32 and bf16 MFMAs
  // leave D(row = 4(lane>>4) + r, col = lane&15).  So C(row, col) with
  // row = m0 + wm*BM/2 + x*16 + (lane&15) and col = n0 + wn*BN/2 + y*16 +
  // ((lane>>4) + 4r) for FP64, (4(lane>>4) + r) otherwise.
  // With beta != 0 the old values of one 16-row block (FN * 4 per lane) are
  // all loaded before any of them is written: loads and stores of C may
  // alias as far as the compiler knows, so element-by-element code waits for
  // each load in turn (64 round trips per lane on a 128 x 128 tile).  Tiles
  // inside C take a path without per-element guards, whose stores then need
  // no waits between them.
  auto colof = [&](int y, int r) {
    return n0 + wn * PN + y * 16 + (P == PREC_FP64 ? kr + 4 * r : 4 * kr + r);
  };
  if (m0 + BM <= M && n0 + BN <= N) {
#pragma unroll
    for (int x = 0; x < FM; ++x) {
      double* Cr = C + (m0 + wm * PM + x * 16 + cr);
      double old[FN][4];
      if (beta != 0.0) {
#pragma unroll
        for (int y = 0; y < FN; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) old[y][r] = Cr[(int64_t)colof(y, r) * ldc];
      }
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double v = alpha * (double)acc[x][y][r];
          Cr[(int64_t)colof(y, r) * ldc] = beta != 0.0 ? v + beta * old[y][r] : v;
        }
    }
    return;
  }
#pragma unroll
  for (int x = 0; x < FM; ++x) {
    const int row = m0 + wm * PM + x * 16 + cr;
    const bool rok = row < M;
    double old[FN][4];
    if (beta != 0.0) {
#pragma unroll
      for (int y = 0; y < FN; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = colof(y, r);
          old[y][r] = (rok && col < N) ? C[row + (int64_t)col * ldc] : 0.0;
        }
    }
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = colof(y, r);
        if (rok && col < N) {
          double v = alpha * (double)acc[x][y][r];
          if (beta != 0.0) v += beta * old[y][r];
          C[row + (int64_t)col * ldc] = v;
        }
      }
  }
}

// op(X) (R x K: element (r, k) = X[r + k ldx] when rcontig, else X[k + r ldx])
// split into NPC BF16 pieces exactly as k_gemm's loaders split it, in the
// LDS slab layout: chunk (kc, r) holds k = 8 kc .. 8 kc + 7 of row r (zeros
// from K on) at out[q * Kc * R + kc * R + r], piece q.
// With S > 1, X holds S split-K partials zs apart and op(X) is their sum,
// taken as k_splitk_reduce takes it (alpha 1, beta 0), so the pieces are
// those of the reduced matrix and the reduction launch is saved.
// Thread w takes chunk (kc, r): with rcontig, r = w mod R (consecutive lanes
// read consecutive rows at each k); otherwise lanes go in 8 x 8 tiles, lane
// l on kc = 8 kt + l mod 8, r = 8 rt + l / 8, so that eight lanes read 512
// contiguous bytes of one column and eight lanes write 128 contiguous bytes.
// NS = S known at compile time (1..8; 0: S taken at run time).  A chunk
// inside X issues the loads of four partials (32 values) before summing
// them, in the same order; with NS the partial loop unrolls completely.
// (Summing element by element, each partial's load waited for the one
// before it: about 50 us per launch for the four partials of an 8000 x 256
// sample.)
template <int NPC, int NS>
__global__ void k_presplit(int R, int K, int Kc, const double* __restrict__ X, int64_t ldx,
                           int rcontig, int S, int64_t zs, uint4* __restrict__ out) {
  const int64_t total = (int64_t)Kc * R;
  const int rt8 = (R + 7) / 8;
  const int64_t span = rcontig ? total : (int64_t)((Kc + 7) / 8) * rt8 * 64;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < span;
       w += (int64_t)gridDim.x * blockDim.x) {
    int r, kc;
    if (rcontig) {
      r = (int)(w % R);
      kc = (int)(w / R);
    } else {
      const int64_t tile = w >> 6;
      const int l = (int)(w & 63);
      kc = (int)(tile / rt8) * 8 + (l & 7);
      r = (int)(tile % rt8) * 8 + (l >> 3);
      if (kc >= Kc || r >= R) continue;
    }
    const int64_t idx = (int64_t)kc * R + r;
    double v[8];
    if (8 * kc + 8 <= K) {
      // Whole chunk inside X: every load first (four partials at a time),
      // then the sums in order z = 0, 1, ... as below.
      const int64_t o0 = rcontig ? r + (int64_t)(8 * kc) * ldx : 8 * kc + (int64_t)r * ldx;
      const int64_t ke = rcontig ? ldx : 1;  // step between consecutive k
      if constexpr (NS == 1) {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = X[o0 + e * ke];
      } else {
        const int ns = NS > 0 ? NS : S;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.0;
        int z0 = 0;
#pragma unroll
        for (; z0 + 4 <= ns; z0 += 4) {
          double p[4][8];
#pragma unroll
          for (int zz = 0; zz < 4; ++zz)
#pragma unroll
            for (int e = 0; e < 8; ++e) p[zz][e] = X[(z0 + zz) * zs + o0 + e * ke];
#pragma unroll
          for (int zz = 0; zz < 4; ++zz)
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] += p[zz][e];
        }
#pragma unroll
        for (; z0 < ns; ++z0) {
          double p[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) p[e] = X[z0 * zs + o0 + e * ke];
#pragma unroll
          for (int e = 0; e < 8; ++e) v[e] += p[e];
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 8 * kc + e;
        v[e] = 0.0;
        if (k < K) {
          const int64_t o = rcontig ? r + (int64_t)k * ldx : k + (int64_t)r * ldx;
          if (S == 1) {
            v[e] = X[o];
          } else {  // split-K partials, summed in k_splitk_reduce's order
            for (int z = 0; z < S; ++z) v[e] += X[z * zs + o];
          }
        }
      }
    }
    unsigned short h[8], m[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float x = fl32(v[e]);
      if constexpr (NPC == 3) {
        const Bf3 p = split3(x);
        h[e] = __builtin_bit_cast(unsigned short, p.h);
        m[e] = __builtin_bit_cast(unsigned short, p.m);
        l[e] = __builtin_bit_cast(unsigned short, p.l);
      } else {
        const __bf16 hb = (__bf16)x;
        h[e] = __builtin_bit_cast(unsigned short, hb);
        l[e] = __builtin_bit_cast(unsigned short, (__bf16)(x - (float)hb));
        m[e] = 0;
      }
    }
    auto pack = [](const unsigned short (&a)[8]) {
      return uint4{a[0] | ((unsigned)a[1] << 16), a[2] | ((unsigned)a[3] << 16),
                   a[4] | ((unsigned)a[5] << 16), a[6] | ((unsigned)a[7] << 16)};
    };
    out[idx] = pack(h);
    if constexpr (NPC == 3) {
      out[total + idx] = pack(m);
      out[2 * total + idx] = pack(l);
    } else {
      out[total + idx] = pack(l);
    }
  }
}

// Small FP64 products (M, N <= kSmallMN, short K: the 128 x 128 blocks of
// the panel factorizations).  Four waves per 16 x 16 tile of C, wave w
// taking the w-th quarter of K (a multiple of 4 deep), with its operands
// read straight from memory (L2) into the MFMA operand registers, eight K
// steps of loads in flight at a time and two accumulators; the four partial
// tiles are summed in wave order through LDS.  A 128-deep product then waits
// for one round trip of loads instead of four.  Spreads a 128 x 128 product
// over 64 CUs, where the LDS-tiled kernel puts it on four.
// Same transposed MFMA orientation as k_gemm: register r of lane l holds
// C(m0 + (l & 15), n0 + (l >> 4) + 4 r).
constexpr int kSmallWaves = 4;
template <bool TA, bool TB>
__global__ __launch_bounds__(64 * kSmallWaves) void k_gemm_small(
    int M, int N, int K, const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
    int64_t ldb, double* __restrict__ C, int64_t ldc, double alpha, double beta) {
  __shared__ v4d part[kSmallWaves - 1][64];  // the partial tiles of waves 1, 2, 3
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 16, n0 = blockIdx.y * 16;
  const int li = lane & 15, lk = lane >> 4;
  const int ia = m0 + li, jb = n0 + li;  // row of op(A), column of op(B) this lane reads
  const int kq = (K + 4 * kSmallWaves - 1) / (4 * kSmallWaves) * 4;
  const int kb = wave * kq, ke = min(K, kb + kq);  // this wave's part of K
  auto opA = [&](int k) -> double {
    if (ia >= M || k >= ke) return 0.0;
    return TA ? A[k + (int64_t)ia * lda] : A[ia + (int64_t)k * lda];
  };
  auto opB = [&](int k) -> double {
    if (jb >= N || k >= ke) return 0.0;
    return TB ? B[jb + (int64_t)k * ldb] : B[k + (int64_t)jb * ldb];
  };
  v4d acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  constexpr int kSteps = 8;  // K steps of 4 per batch of loads
  for (int k0 = kb; k0 < ke; k0 += 4 * kSteps) {
    double a[kSteps], b[kSteps];
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
      a[u] = opA(k0 + 4 * u + lk);
      b[u] = opB(k0 + 4 * u + lk);
    }
#pragma unroll
    for (int u = 0; u < kSteps; u += 2) {
      acc0 = mfma64(b[u], a[u], acc0);
      acc1 = mfma64(b[u + 1], a[u + 1], acc1);
    }
  }
  v4d acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = acc0[r] + acc1[r];
  if (wave > 0) part[wave - 1][lane] = acc;
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int w = 0; w < kSmallWaves - 1; ++w) {
    const v4d p = part[w][lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += p[r];
  }
  const int row = m0 + li;
  if (row >= M) return;
  double old[4] = {0.0, 0.0, 0.0, 0.0};  // loaded together, before any store
  if (beta != 0.0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = n0 + lk + 4 * r;
      if (col < N) old[r] = C[row + (int64_t)col * ldc];
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int col = n0 + lk + 4 * r;
    if (col < N) C[row + (int64_t)col * ldc] = alpha * acc[r] + beta * old[r];
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
    // Partials summed in order z = 0, 1, ...; loaded 32 (then eight) at a
    // time so the loads are in flight together (the deep splits of the
    // Gram matrices, 64 partials, wait for two round trips).
    double s = 0.0;
    int z = 0;
    for (; z + 32 <= S; z += 32) {
      double p[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) p[u] = P[(z + u) * zstride + idx];
#pragma unroll
      for (int u = 0; u < 32; ++u) s += p[u];
    }
    for (; z + 8 <= S; z += 8) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = P[(z + u) * zstride + idx];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += p[u];
    }
    for (; z < S; ++z) s += P[z * zstride + idx];
    double* p = C + i + j * ldc;
    double v = alpha * s;
    if (beta != 0.0) v += beta * *p;
    *p = v;
  }
}

template <int P, bool TA, bool TB, int BM, int BN, int WM, int WN, int ROLE>
void launch(hipStream_t st, dim3 grid, int M, int N, int K, int kper, const double* A,
            int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
            int64_t zstride, double alpha, double beta, const PsOps& ps) {
  hipLaunchKernelGGL((k_gemm<P, TA, TB, BM, BN, WM, WN, ROLE>), grid, dim3(64 * WM * WN), 0, st, M, N, K,
                     kper, A, lda, B, ldb, C, ldc, zstride, alpha, beta, ps);
}

template <int P, int BM, int BN, int WM, int WN, int ROLE>
void launch_t(hipStream_t st, bool ta, bool tb, dim3 grid, int M, int N, int K, int kper,
              const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
              int64_t ldc, int64_t zs, double al, double be, const PsOps& ps) {
  if (!ta && !tb) launch<P, false, false, BM, BN, WM, WN, ROLE>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
  else if (ta && !tb) launch<P, true, false, BM, BN, WM, WN, ROLE>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
  else if (!ta && tb) launch<P, false, true, BM, BN, WM, WN, ROLE>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
  else launch<P, true, true, BM, BN, WM, WN, ROLE>(st, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
}

// Tile shapes: 0 = 64 x 64 on 2 x 2 waves; 1 = 128 x 128 on 2 x 2 waves, in
// FP64 on 2 x 4 waves of 64 x 32 (two workgroups of eight waves per CU, four
// waves per SIMD to cover each other's LDS and barrier waits: 50-61 against
// 47-58 TFLOP/s on the 8000 x 8000 thin products alone; 4 x 2 waves of
// 32 x 64 need 140 registers, one workgroup per CU, and were slower).
template <int P, int ROLE = 0>
void launch_p(hipStream_t st, int shape, bool ta, bool tb, dim3 grid, int M, int N, int K,
              int kper, const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
              int64_t ldc, int64_t zs, double al, double be, const PsOps& ps = PsOps{}) {
  if constexpr (P == PREC_FP64) {
    if (shape == 1) launch_t<P, 128, 128, 2, 4, ROLE>(st, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
    else launch_t<P, 64, 64, 2, 2, ROLE>(st, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
  } else {
    if (shape == 1) launch_t<P, 128, 128, 2, 2, ROLE>(st, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
    else launch_t<P, 64, 64, 2, 2, ROLE>(st, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
  }
}

// The BF16 products with pre-split operands: ROLE 4 (A), 8 (B) or 12 (both).
template <int P>
void launch_ps(hipStream_t st, int role, int shape, bool ta, bool tb, dim3 grid, int M, int N,
               int K, int kper, const double* A, int64_t lda, const double* B, int64_t ldb,
               double* C, int64_t ldc, int64_t zs, double al, double be, const PsOps& ps) {
  if (role == 4) launch_p<P, 4>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
  else if (role == 8) launch_p<P, 8>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
  else launch_p<P, 12>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, C, ldc, zs, al, be, ps);
}

int g_panel_scope = 0;  // > 0 while a panel factorization enqueues its products

}  // namespace

void gemm_panel_scope(int delta) { g_panel_scope += delta; }

#ifndef SMALL_SPLIT_MIN_K
#define SMALL_SPLIT_MIN_K 64
#endif
// Least reduction depth per split of a small output (a Gram matrix of a tall
// panel): its workgroups are latency-bound, so shorter splits finish sooner.
constexpr int kSmallSplitMinK = SMALL_SPLIT_MIN_K;

hipError_t gemm(hipStream_t st, Prec prec, bool ta, bool tb, int M, int N, int K,
                double alpha, const double* A, int64_t lda, const double* B,
                int64_t ldb, double beta, double* C, int64_t ldc, double* splitws,
                size_t splitws_elems, bool small_tiles, const PsOperand* psa,
                const PsOperand* psb, SplitKeep* keep) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int role_ps = (psa ? 4 : 0) | (psb ? 8 : 0);
  if (role_ps) {
    if (prec != PREC_BF16X3 && prec != PREC_BF16X6) return hipErrorInvalidValue;
    const int64_t kc = (K + 31) / 32 * 4;
    if ((psa && (psa->rows != M || psa->kc < kc)) || (psb && (psb->rows != N || psb->kc < kc)))
      return hipErrorInvalidValue;
  }
  const PsOps ops{psa ? psa->p : nullptr, psb ? psb->p : nullptr, psa ? psa->rows : 0,
                  psb ? psb->rows : 0, psa ? psa->piece : 0, psb ? psb->piece : 0};
  if (prec == PREC_FP64 && M <= kSmallMN && N <= kSmallMN && K <= kSmallK) {
    const dim3 grid((M + 15) / 16, (N + 15) / 16);
    const int slot = prof_mark(st, PC_GEMM_SMALL);
    if (!ta && !tb) hipLaunchKernelGGL((k_gemm_small<false, false>), grid, dim3(64 * kSmallWaves), 0, st, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta);
    else if (ta && !tb) hipLaunchKernelGGL((k_gemm_small<true, false>), grid, dim3(64 * kSmallWaves), 0, st, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta);
    else if (!ta && tb) hipLaunchKernelGGL((k_gemm_small<false, true>), grid, dim3(64 * kSmallWaves), 0, st, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta);
    else hipLaunchKernelGGL((k_gemm_small<true, true>), grid, dim3(64 * kSmallWaves), 0, st, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta);
    prof_done(st, slot, PC_GEMM_SMALL, 2.0 * M * N * (double)K,
              8.0 * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1)));
    return hipGetLastError();
  }
  // 128 x 128 tiles when the output, or the output times a split of K,
  // gives enough workgroups; else 64 x 64.  Long reductions are split over
  // blockIdx.z until about two workgroups per CU are in flight.
  const int64_t t128 = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
  const bool big = !small_tiles &&
                   (t128 >= 384 || (splitws && K >= 2048 && t128 * std::min(8, K / 512) >= 384));
  // (Tiles spanning the thin b = 256 side with one workgroup per CU were
  // measured slower than two 128 x 128 workgroups per CU on every thin
  // product of the step, in all three arithmetics.)
  const int shape = big ? 1 : 0;
  // Slab depth of the chosen tile (split-K boundaries are multiples of it).
  const int BK = (prec == PREC_BF16X3 || prec == PREC_BF16X6) ? 32 : (shape ? 16 : K64_SLAB);
  const int BMs = shape ? 128 : 64, BNs = shape ? 128 : 64;
  const int tm = (M + BMs - 1) / BMs, tn = (N + BNs - 1) / BNs;
  const int tiles = tm * tn;
  int splits = 1;
  if (splitws && tiles < 512 && K >= 1024) {
    // Small outputs (Gram matrices of tall panels) split deeper.
    const bool small = tiles <= 32;
    // 128 x 128 tiles in BF16x3 or FP64 fit two workgroups per CU (LDS):
    // at most 512 workgroups, rounded down, so that all of them run in one
    // wave instead of a full wave and a short second one (126 tiles of the
    // thin sampling products: 4 splits, not 5).  Otherwise about 512,
    // rounded up (FP32 128 x 128 and 64 x 64 tiles fit more per CU, and the
    // FP32 products keep their shorter FP32 accumulation chains).
    const bool two_per_cu =
        shape == 1 && (prec == PREC_BF16X3 || prec == PREC_BF16X6 || prec == PREC_FP64);
    splits = small ? (1024 + tiles - 1) / tiles
                   : (two_per_cu ? std::max(1, 512 / tiles) : (512 + tiles - 1) / tiles);
    splits = std::min(splits, K / (small ? kSmallSplitMinK : 512));
    splits = std::min(splits, small ? kMaxSplitKSmall : kMaxSplitK);
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
  const int op = ta ? (tb ? PC_GEMM_TT : PC_GEMM_TN) : (tb ? PC_GEMM_NT : PC_GEMM_NN);
  const bool uv = small_tiles && prec == PREC_FP64;  // the U / V stream's products
  const int cls = uv ? PC_UV + op : 16 * shape + 4 * (int)prec + op;
  const int slot = prof_mark(st, cls);
  if (prec == PREC_FP32)
    launch_p<PREC_FP32>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else if (prec == PREC_BF16X6 && role_ps)
    launch_ps<PREC_BF16X6>(st, role_ps, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be, ops);
  else if (prec == PREC_BF16X6)
    launch_p<PREC_BF16X6>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else if (prec == PREC_BF16X3 && role_ps)
    launch_ps<PREC_BF16X3>(st, role_ps, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be, ops);
  else if (prec == PREC_BF16X3)
    launch_p<PREC_BF16X3>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else if (uv)
    launch_p<PREC_FP64, 2>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else if (g_panel_scope > 0)
    launch_p<PREC_FP64, 1>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  else
    launch_p<PREC_FP64>(st, shape, ta, tb, grid, M, N, K, kper, A, lda, B, ldb, Cout, ldo, zs, al, be);
  prof_done(st, slot, cls, 2.0 * M * N * (double)K,
            8.0 * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1)));
  hipError_t e = hipGetLastError();
  if (keep) *keep = SplitKeep{C, ldc, 1, 0};
  if (e != hipSuccess || splits == 1) return e;
  if (keep && alpha == 1.0 && beta == 0.0) {  // the consumer sums the partials
    *keep = SplitKeep{splitws, M, splits, zs};
    return e;
  }
  const int64_t total = (int64_t)M * N;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  const int slot2 = prof_mark(st, PC_SPLITK);
  hipLaunchKernelGGL(k_splitk_reduce, dim3(blocks), dim3(256), 0, st, M, N, splits, splitws,
                     zs, C, ldc, alpha, beta);
  prof_done(st, slot2, PC_SPLITK, (double)splits * M * N,
            8.0 * (double)M * N * (splits + (beta != 0.0 ? 2 : 1)));
  return hipGetLastError();
}

size_t presplit_bytes(Prec prec, int64_t R, int64_t K) {
  if (prec != PREC_BF16X3 && prec != PREC_BF16X6) return 0;
  const int64_t kc = (K + 31) / 32 * 4;  // 8-deep chunks, K padded to the 32-deep slab
  return (size_t)(prec == PREC_BF16X6 ? 3 : 2) * kc * R * sizeof(uint4);
}

hipError_t presplit(hipStream_t st, Prec prec, int R, int K, const double* X, int64_t ldx,
                    bool rcontig, void* out, PsOperand* o, int S, int64_t zs) {
  if (prec != PREC_BF16X3 && prec != PREC_BF16X6) return hipErrorInvalidValue;
  if (R < 0 || K < 0 || S < 1 || ((uintptr_t)out & 15)) return hipErrorInvalidValue;
  const int kc = (K + 31) / 32 * 4;
  *o = PsOperand{(const uint4*)out, R, kc, (int64_t)kc * R};
  if (R == 0 || kc == 0) return hipSuccess;
  const int64_t total = rcontig ? (int64_t)kc * R : (int64_t)((kc + 7) / 8) * ((R + 7) / 8) * 64;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  const int rc = rcontig ? 1 : 0;
  auto go = [&](auto npc, auto ns) {
    hipLaunchKernelGGL((k_presplit<decltype(npc)::value, decltype(ns)::value>), dim3(blocks),
                       dim3(256), 0, st, R, K, kc, X, ldx, rc, S, zs, (uint4*)out);
  };
  auto by_s = [&](auto npc) {
    using std::integral_constant;
    switch (S) {
      case 1: go(npc, integral_constant<int, 1>{}); break;
      case 2: go(npc, integral_constant<int, 2>{}); break;
      case 3: go(npc, integral_constant<int, 3>{}); break;
      case 4: go(npc, integral_constant<int, 4>{}); break;
      case 5: go(npc, integral_constant<int, 5>{}); break;
      case 6: go(npc, integral_constant<int, 6>{}); break;
      case 7: go(npc, integral_constant<int, 7>{}); break;
      case 8: go(npc, integral_constant<int, 8>{}); break;
      default: go(npc, integral_constant<int, 0>{}); break;
    }
  };
  if (prec == PREC_BF16X6) by_s(std::integral_constant<int, 3>{});
  else by_s(std::integral_constant<int, 2>{});
  return hipGetLastError();
}

}  // namespace rutv
