// Householder QR of a whole tall panel by CholeskyQR2 and Householder
// reconstruction (Section 2.4, eqs. unpivQR and WYrepresentation).
//
// The reflectors of an unpivoted Householder QR are fixed by the orthonormal
// factor Q alone: with S = diag(s_k), s_k = -sign of the k-th pivot, the LU
// factorization Q - [S; 0] = L U (no pivoting needed: every |u_kk| >= 1)
// gives V = L (unit lower trapezoidal), Tw = -U S L1^-T (L1 = top nb x nb
// block of L) and R_householder = S R, so that (I - V Tw V^T)(:, 1:nb) = Q S.
// The signs follow LAPACK dlarfg (beta = -sign(alpha) ||x||, sign(0) = +1),
// so the result is the dgeqrf factorization up to rounding.
//
// Q comes from CholeskyQR2 (Gram, Cholesky, Q1 = P R1^-1, repeated once), so
// the whole panel costs four tall MFMA products over its Mp rows plus three
// nb x nb factorizations, instead of nb dependent column steps.  CholeskyQR2
// needs kappa(P) well below eps^-1/2: the Cholesky kernels and the LU raise
// a device flag when a pivot says otherwise (or when a column tail is
// exactly zero, where dlarfg takes tau = 0), and then the column-by-column
// cooperative kernel refactors the panel, gated on that flag, so no host
// round trip is needed.
//
// The nb x nb work runs in one workgroup of 8 waves on 16 x 16 FP64 MFMA
// tiles (matrix padded to a multiple of 16 with an identity block): right-
// looking blocked factorizations whose 16 x 16 diagonal blocks are factored
// by one wave in LDS, with the triangular inverses built alongside, block
// column by block column.
#include <algorithm>
#include <utility>

#include "common.h"

namespace rutv {
namespace {

constexpr int TS = 16;         // tile size
constexpr int kWaves = 8;      // waves of the single-workgroup kernels
constexpr int kThreads = 64 * kWaves;
constexpr int kBlk = 128;      // widest block factored in LDS (wider panels: two blocks)
constexpr int LDA = kBlk + 1;  // LDS leading dimension (odd: spreads the banks)
constexpr int kLoadCols = kThreads / kBlk;  // columns per pass when loading a block
// Largest max |G - I| for which the second CholeskyQR pass takes its factors
// from the first-order expansion (see k_hr_chol): 128 (2^-30)^2 = 2^-53.
constexpr double kNearIdentity = 0x1p-30;

__device__ inline v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc += op(A) op(B) for 16 x 16 tiles (K = 16).  Tiles are column-major with
// leading dimensions lda / ldb; TA / TB take the transpose.  MFMA operand
// layout: A(i, k) from lane i + 16k, B(k, j) from lane j + 16k; result
// D((lane>>4) + 4r, lane & 15) in register r.
template <bool TA, bool TB>
__device__ inline v4d tile_mma(v4d acc, const double* A, int lda, const double* B, int ldb) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, kq = l >> 4;
#pragma unroll
  for (int kk = 0; kk < TS; kk += 4) {
    const int k = kk + kq;
    const double a = TA ? A[k + i * lda] : A[i + k * lda];
    const double b = TB ? B[i + k * ldb] : B[k + i * ldb];
    acc = mfma(a, b, acc);
  }
  return acc;
}

// As tile_mma<false, false>, reading A and / or B as a triangle of a
// packed diagonal tile: mask 1 keeps the upper part (with the diagonal), 2
// the strictly lower part with a unit diagonal; 0 reads the whole tile.
__device__ inline double tri_mask(double v, int r, int c, int mask) {
  if (mask == 1) return r <= c ? v : 0.0;
  if (mask == 2) return r > c ? v : (r == c ? 1.0 : 0.0);
  return v;
}

__device__ inline v4d tile_mma_m(v4d acc, const double* A, int lda, int ma, const double* B,
                                 int ldb, int mb) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, kq = l >> 4;
#pragma unroll
  for (int kk = 0; kk < TS; kk += 4) {
    const int k = kk + kq;
    const double a = tri_mask(A[i + k * lda], i, k, ma);
    const double b = tri_mask(B[k + i * ldb], k, i, mb);
    acc = mfma(a, b, acc);
  }
  return acc;
}

__device__ inline v4d tile_load(const double* X, int ld) {
  const int l = threadIdx.x & 63;
  v4d v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = X[((l >> 4) + 4 * r) + (l & 15) * ld];
  return v;
}

__device__ inline void tile_store(double* X, int ld, v4d v) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) X[((l >> 4) + 4 * r) + (l & 15) * ld] = v[r];
}

__device__ inline v4d vzero() { return v4d{0.0, 0.0, 0.0, 0.0}; }

// acc += A * b, where b is a register tile in the result layout (register r
// of lane l holds b((l>>4) + 4r, l & 15)), which is exactly the MFMA B-operand
// layout for k = 4r + (l>>4); A is a 16 x 16 tile (ld lda).
__device__ inline v4d mma_reg_b(v4d acc, const double* A, int lda, v4d b) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, kq = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc = mfma(A[i + (4 * r + kq) * lda], b[r], acc);
  return acc;
}

// ---- 16 x 16 tiles in registers, one wave: lane j < 16 holds column j
// (a[i] = X(i, j)); lanes 16..63 carry copies that are never stored.  Values
// of other columns are read with readlane at compile-time lane indices.

__device__ inline double rl(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Orders register values in program order: an empty volatile statement
// taking the value as a read-write operand, so that the compiler neither
// hoists the broadcasts that read it above the statement nor sinks the
// arithmetic that writes it below the next one.  Without it all broadcasts
// of a step are issued at once and the scalar registers spill.
__device__ inline void pin(double& v) { asm volatile("" : "+v"(v)); }

// Value of v in lane C of each row of 16 lanes (DPP row_newbcast; one
// v_mov_b64 per double).  The four rows of a wave hold copies of the same
// 16 columns, so every lane receives column C's value.
template <int C>
__device__ inline double bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + C, 0xF, 0xF, true);
}

// 1/x and 1/sqrt(x) from the hardware estimates (relative error below
// 2^-22, denormals supported) and two Newton steps each: a few ulp, in
// five or six dependent FMAs instead of the IEEE division sequence.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double rsq_nr(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

__device__ inline void col_load(const double* T, int ld, double (&a)[TS]) {
  const int j = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < TS; ++i) a[i] = T[i + j * ld];
}

__device__ inline void col_store(double* T, int ld, const double (&a)[TS]) {
  const int j = threadIdx.x & 63;
  if (j < TS) {
#pragma unroll
    for (int i = 0; i < TS; ++i) T[i + j * ld] = a[i];
  }
}

constexpr int kPipe = 4;  // broadcasts in flight per group in the tile routines

// The 15 rank-1 updates of step C of a 16-column elimination, as a pipeline:
// job e < 15 - C updates row C+1+e of the eliminated matrix, a later job
// row e-(15-C) of the inverse being accumulated; broadcasts are read kPipe
// at a time, one group ahead of the FMAs that use them, and pin() bounds
// how many are live.  upd(e, b) applies job e with broadcast value b.
template <int C, typename Src, typename Upd>
__device__ inline void step_updates(Src src, Upd upd) {
  double bp[kPipe], bn[kPipe];
#pragma unroll
  for (int e0 = 0; e0 < TS - 1 + kPipe; e0 += kPipe) {
#pragma unroll
    for (int q = 0; q < kPipe; ++q) {
      const int e = e0 + q;
      if (e < TS - 1) {
        double& z = src(e);
        pin(z);
        bn[q] = bcast<C>(z);
      }
    }
#pragma unroll
    for (int q = 0; q < kPipe; ++q) {
      const int e = e0 - kPipe + q;
      if (e >= 0 && e < TS - 1) upd(e, bp[q]);
    }
#pragma unroll
    for (int q = 0; q < kPipe; ++q) bp[q] = bn[q];
  }
}

// Upper Cholesky R of the symmetric tile in a (both triangles present) and
// x = R^-1, in one sweep: the elimination runs without square roots (A =
// U^T diag(d) U, U unit upper) so the pivot chain holds one reciprocal per
// column, and the columns of U^-1 are accumulated right-looking from the
// same broadcasts (column c of U^-1 is final once step c starts).  Then R =
// diag(d)^1/2 U and R^-1 = U^-1 diag(d)^-1/2, the square roots taken once
// per lane at the end.  On return a holds R and x
// holds R^-1 (zeros below the diagonal).  A pivot at or below thr in a real
// column (k0 + c < n) is replaced by 1 and reported through bad.
template <int C>
__device__ inline void chol_step(double (&a)[TS], double (&x)[TS], int k0, int n, double thr,
                                 bool& bad, double& my_d) {
  const int j = threadIdx.x & 15;
  double d = bcast<C>(a[C]);
  if (k0 + C < n && !(d > thr)) {
    bad = true;
    d = 1.0;
  }
  const double t = j > C ? a[C] * rcp_nr(d) : 0.0;  // U(C, j)
  auto src = [&](int e) -> double& { return e < TS - 1 - C ? a[C + 1 + e] : x[e - (TS - 1 - C)]; };
  step_updates<C>(src, [&](int e, double b) {
    double& z = src(e);
    z = fma(-b, t, z);
    pin(z);
  });
  x[C] -= t;
  if (j == C) my_d = d;
}

template <int... Cs>
__device__ inline void chol_steps(std::integer_sequence<int, Cs...>, double (&a)[TS],
                                  double (&x)[TS], int k0, int n, double thr, bool& bad,
                                  double& my_d) {
  (chol_step<Cs>(a, x, k0, n, thr, bad, my_d), ...);
}

// R(i, j) = d_i^-1/2 A(i, j) above the diagonal (row i's scale broadcast
// from lane i), d_j^1/2 on it, zero below.  The broadcast is taken by every
// lane before the selection (a DPP read from a lane switched off by a branch
// returns zero).
template <int I>
__device__ inline void chol_scale_row(double (&a)[TS], double my_d, double my_s) {
  const int j = threadIdx.x & 15;
  const double si = bcast<I>(my_s);
  a[I] = I < j ? a[I] * si : (I == j ? my_d * my_s : 0.0);
}
template <int... Is>
__device__ inline void chol_scale(std::integer_sequence<int, Is...>, double (&a)[TS],
                                  double my_d, double my_s) {
  (chol_scale_row<Is>(a, my_d, my_s), ...);
}

__device__ inline void chol_inv16(double (&a)[TS], double (&x)[TS], int k0, int n, double thr,
                                  bool& bad) {
  const int j = threadIdx.x & 15;
  double my_d = 1.0;
#pragma unroll
  for (int i = 0; i < TS; ++i) x[i] = i == j ? 1.0 : 0.0;
  chol_steps(std::make_integer_sequence<int, TS>(), a, x, k0, n, thr, bad, my_d);
  const double my_s = rsq_nr(my_d);  // d_j^-1/2
  chol_scale(std::make_integer_sequence<int, TS>(), a, my_d, my_s);
#pragma unroll
  for (int i = 0; i < TS; ++i) x[i] *= my_s;
}

// LU of the tile in a minus S, S = diag(s_c) with s_c = -sign(pivot) chosen
// as each pivot is reached (sign(0) = +1; the last column of a square panel,
// last_col, takes s = sign(p) and u = 0 instead), with L^-1 and U^-1 built in
// the same sweep: at step c every lane reads column c (pivot and L(:, c)) and,
// for U^-1, column c of W = U^-1 diag(u) (final once step c starts); lanes
// right of c update their part of A and of W with t = U(c, j) / u_cc, and
// every lane updates its column of Y = L^-1 with Y(c, j) / u_cc (zero right
// of c).  On return a holds L \ U packed (unit diagonal of L implied), xl =
// L^-1 (unit lower), xu = U^-1 (zero column for u = 0).  sg_out[c] and
// tau_out[c] (c < n) receive s_c and -u_cc s_c; bad is set for a
// pivot with |p| >= 1 - 2^-50 in a real column other than last_col.
struct LuState {
  double my_ui, my_sg;
};

template <int C>
__device__ inline void lu_step(double (&a)[TS], double (&xl)[TS], double (&xu)[TS], int k0,
                               int n, int last_col, bool& bad, LuState& st) {
  const int j = threadIdx.x & 15;
  const double p = bcast<C>(a[C]);
  const bool last = k0 + C == last_col;
  double sg = p >= 0.0 ? -1.0 : 1.0;  // s = -sign(p), sign(0) = +1
  if (last) sg = -sg;
  if (!last && k0 + C < n && !(fabs(p) < 1.0 - 0x1p-50)) bad = true;
  const double u = last ? 0.0 : p - sg;
  const double ui = last ? 0.0 : rcp_nr(u);
  const double t = j > C ? a[C] * ui : 0.0;  // U(C, j) / u_CC
  const double ty = xl[C] * ui;              // Y(C, j) / u_CC
  auto src = [&](int e) -> double& { return e < TS - 1 - C ? a[C + 1 + e] : xu[e - (TS - 1 - C)]; };
  step_updates<C>(src, [&](int e, double b) {
    if (e < TS - 1 - C) {  // row below C: used for A and for Y
      const int i = C + 1 + e;
      a[i] = fma(-b, t, a[i]);
      xl[i] = fma(-b, ty, xl[i]);
      pin(a[i]);
      pin(xl[i]);
    } else {
      double& z = xu[e - (TS - 1 - C)];
      z = fma(-b, t, z);
      pin(z);
    }
  });
  xu[C] -= t;
  if (j == C) {
    a[C] = u;
    st.my_ui = ui;
    st.my_sg = sg;
  }
}

template <int... Cs>
__device__ inline void lu_steps(std::integer_sequence<int, Cs...>, double (&a)[TS],
                                double (&xl)[TS], double (&xu)[TS], int k0, int n, int last_col,
                                bool& bad, LuState& st) {
  (lu_step<Cs>(a, xl, xu, k0, n, last_col, bad, st), ...);
}

__device__ inline void lu_inv16(double (&a)[TS], double (&xl)[TS], double (&xu)[TS], int k0,
                                int n, int last_col, double* sg_out, double* tau_out,
                                bool& bad) {
  const int lane = threadIdx.x & 63, j = lane & 15;
  LuState st{0.0, 0.0};
#pragma unroll
  for (int i = 0; i < TS; ++i) xl[i] = xu[i] = i == j ? 1.0 : 0.0;
  lu_steps(std::make_integer_sequence<int, TS>(), a, xl, xu, k0, n, last_col, bad, st);
#pragma unroll
  for (int i = 0; i < TS; ++i) {
    if (i > j) a[i] *= st.my_ui;  // L(i, j)
    xu[i] *= st.my_ui;
  }
  if (lane < TS) {
    sg_out[k0 + lane] = st.my_sg;
    if (k0 + lane < n) tau_out[k0 + lane] = -a[lane] * st.my_sg;
  }
}

// x = inverse of the upper-triangular tile in a (x zero below the diagonal).
__device__ inline void inv_upper16(const double (&a)[TS], double (&x)[TS]) {
  const int lane = threadIdx.x & 63;
  double myd = 1.0;
#pragma unroll
  for (int i = 0; i < TS; ++i)
    if (lane == i) myd = a[i];
  const double myinv = 1.0 / myd;
#pragma unroll
  for (int i = TS - 1; i >= 0; --i) {
    double s = (lane == i) ? 1.0 : 0.0;
#pragma unroll
    for (int k = i + 1; k < TS; ++k) s -= rl(a[i], k) * x[k];
    x[i] = s * rl(myinv, i);
  }
}

// x = inverse of the unit-lower-triangular tile in a (strict lower part
// used, diagonal taken as 1; x zero above the diagonal).
__device__ inline void inv_unit_lower16(const double (&a)[TS], double (&x)[TS]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < TS; ++i) {
    double s = (lane == i) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) s -= rl(a[i], k) * x[k];
    x[i] = s;
  }
}

// The whole (padded) matrix of a single-workgroup kernel lives in LDS.
struct Smem {
  double A[kBlk * LDA];  // column-major, leading dimension LDA
  double D[2][TS * 17];  // inverses of the diagonal tiles of steps kt, kt + 1 (ld 17)
  double D2[2][TS * 17];
  double red[kWaves];
  double sgn[kBlk];
  int fail;
};

__device__ inline double* tile(Smem& sm, int it, int jt) { return sm.A + it * TS + jt * TS * LDA; }

__device__ inline double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < kWaves; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

// Element loops over an nbp x nbp matrix: thread t takes row t % nbp and
// every (kThreads / nbp)-th column from t / nbp (consecutive threads on
// consecutive rows; threads beyond a whole number of columns sit out).
__device__ inline int elem_j0(int nbp) {
  const int js = kThreads / nbp;
  return (int)threadIdx.x < js * nbp ? (int)threadIdx.x / nbp : nbp;
}

// (a, b) with 0 <= a <= b < n from a linear index over the upper triangle.
__device__ inline void upper_pair(int t, int n, int& a, int& b) {
  a = 0;
  while (t >= n - a) {
    t -= n - a;
    ++a;
  }
  b = a + t;
}

// Right-looking blocked upper Cholesky A = R^T R (nt tiles) with R^-1 built
// in the same loop: at step kt, after R_kk and R(kt, kt+1:) are formed, block
// column kt of R is final; it is written to Rg (global, ld nbp) and then
// replaced in LDS by block column kt of X = R^-1:
//   X(i, kt) = -sum_{k=i}^{kt-1} X(i, k) (R(k, kt) R_kk^-1),  X(kt, kt) = R_kk^-1.
// On return sm.A holds X (upper, zeros below); Rg holds R (upper part only;
// the caller zeroes below).  A pivot at or below thr in a real column
// (index < n) marks failure and is replaced by 1 so that all stays finite.
__device__ void chol_inv_lds(Smem& sm, int n, int nt, double thr, double* __restrict__ Rg) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nbp = nt * TS;
  // Diagonal tile kt, by wave 0: R_kk into the tile, R_kk^-1 into D[kt & 1].
  auto diag = [&](int kt) {
    bool bad = false;
    double a[TS], x[TS];
    double* Akk = tile(sm, kt, kt);
    col_load(Akk, LDA, a);
    chol_inv16(a, x, kt * TS, n, thr, bad);
    col_store(Akk, LDA, a);
    col_store(sm.D[kt & 1], 17, x);
    if (bad && lane == 0) sm.fail = 1;
  };
  if (wave == 0) diag(0);
  __syncthreads();
  for (int kt = 0; kt < nt; ++kt) {
    const double* D = sm.D[kt & 1];
    double* Akk = tile(sm, kt, kt);
    // row panel R(kt, jt) = R_kk^-T A(kt, jt); block column kt of R to Rg,
    // then R(k, kt) <- R(k, kt) R_kk^-1 for k < kt
    const int nrow = nt - 1 - kt;
    for (int t = wave; t < nrow + kt + 1; t += kWaves) {
      if (t < nrow) {
        double* At = tile(sm, kt, kt + 1 + t);
        tile_store(At, LDA, tile_mma<true, false>(vzero(), D, 17, At, LDA));
      } else {
        const int k = t - nrow;
        double* Ak = tile(sm, k, kt);
        const v4d r = tile_load(Ak, LDA);
        tile_store(Rg + k * TS + (int64_t)kt * TS * nbp, nbp, r);
        if (k < kt) tile_store(Ak, LDA, tile_mma<false, false>(vzero(), Ak, LDA, D, 17));
      }
    }
    __syncthreads();
    // trailing A(it, jt) -= R(kt, it)^T R(kt, jt) (kt < it <= jt) and block
    // column kt of the inverse (into registers until every reader is done).
    // Look-ahead: wave 0 updates tile (kt+1, kt+1) first and factors it while
    // the other waves do the rest.
    const int ntr = nrow * (nrow + 1) / 2;
    v4d xi = vzero();
    int myi = -1;
    if (wave == 0) {
      if (nrow > 0) {
        double* At = tile(sm, kt + 1, kt + 1);
        v4d acc = tile_load(At, LDA);
        const double* Rk = tile(sm, kt, kt + 1);
        const v4d p = tile_mma<true, false>(vzero(), Rk, LDA, Rk, LDA);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] -= p[r];
        tile_store(At, LDA, acc);
        diag(kt + 1);
      }
    } else {
      const int ntask = kt + (ntr > 0 ? ntr - 1 : 0);
      for (int t = wave - 1; t < ntask; t += kWaves - 1) {
        if (t < kt) {
          const int i = t;
          v4d z = vzero();
          for (int k = i; k < kt; ++k)
            z = tile_mma_m(z, tile(sm, i, k), LDA, k == i ? 1 : 0, tile(sm, k, kt), LDA, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) xi[r] = -z[r];
          myi = i;
        } else {
          int a, b;
          upper_pair(t - kt + 1, nrow, a, b);  // pair (0, 0) is wave 0's
          const int it = kt + 1 + a, jt = kt + 1 + b;
          double* At = tile(sm, it, jt);
          v4d acc = tile_load(At, LDA);
          const v4d p = tile_mma<true, false>(vzero(), tile(sm, kt, it), LDA, tile(sm, kt, jt), LDA);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r] -= p[r];
          tile_store(At, LDA, acc);
        }
      }
    }
    __syncthreads();
    if (myi >= 0) tile_store(tile(sm, myi, kt), LDA, xi);
    if (wave == kWaves - 1) tile_store(Akk, LDA, tile_load(D, 17));
    __syncthreads();
  }
  for (int j = elem_j0(nbp), i = (threadIdx.x) % nbp; j < nbp; j += kThreads / nbp) {
    if (i > j) sm.A[i + j * LDA] = 0.0;
  }
  __syncthreads();
}

// In-place inverse of the upper-triangular matrix in sm.A, block row by block
// row from the bottom: X(it, jt) = -R_ii^-1 sum_{k=it+1}^{jt} R(it,k) X(k,jt).
__device__ void inv_upper_lds(Smem& sm, int nt) {
  const int wave = threadIdx.x >> 6;
  for (int it = nt - 1; it >= 0; --it) {
    if (wave == 0) {
      double a[TS], x[TS];
      col_load(tile(sm, it, it), LDA, a);
      inv_upper16(a, x);
      col_store(sm.D[0], 17, x);
    }
    __syncthreads();
    v4d x = vzero();
    const int jt = it + 1 + wave;  // at most nt - 1 - it <= 7 tiles: one per wave
    if (jt < nt) {
      v4d z = vzero();
      for (int k = it + 1; k <= jt; ++k)
        z = tile_mma<false, false>(z, tile(sm, it, k), LDA, tile(sm, k, jt), LDA);
      x = mma_reg_b(vzero(), sm.D[0], 17, z);
    }
    __syncthreads();
    if (jt < nt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = -x[r];
      tile_store(tile(sm, it, jt), LDA, x);
    }
    if (wave == 0) tile_store(tile(sm, it, it), LDA, tile_load(sm.D[0], 17));
    __syncthreads();
  }
}

// In-place inverse of the unit-lower-triangular matrix in sm.A (diagonal
// taken as 1), block row by block row from the top:
// X(it, jt) = -L_ii^-1 sum_{k=jt}^{it-1} L(it,k) X(k,jt), jt < it.
__device__ void inv_unit_lower_lds(Smem& sm, int nt) {
  const int wave = threadIdx.x >> 6;
  for (int it = 0; it < nt; ++it) {
    if (wave == 0) {
      double a[TS], x[TS];
      col_load(tile(sm, it, it), LDA, a);
      inv_unit_lower16(a, x);
      col_store(sm.D[0], 17, x);
    }
    __syncthreads();
    v4d x = vzero();
    const int jt = wave;  // jt < it <= 7: one per wave
    if (jt < it) {
      v4d z = vzero();
      for (int k = jt; k < it; ++k)
        z = tile_mma<false, false>(z, tile(sm, it, k), LDA, tile(sm, k, jt), LDA);
      x = mma_reg_b(vzero(), sm.D[0], 17, z);
    }
    __syncthreads();
    if (jt < it) {
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = -x[r];
      tile_store(tile(sm, it, jt), LDA, x);
    }
    if (wave == 0) tile_store(tile(sm, it, it), LDA, tile_load(sm.D[0], 17));
    __syncthreads();
  }
}

// Upper Cholesky G = R^T R of an n x n Gram matrix (n <= 128, padded to
// nbp = 16 nt with an identity block) and R^-1, both written nbp x nbp with
// leading dimension nbp and exact zeros below the diagonal.
//   pass 1: fail if a pivot falls below 1e-13 * max diag(G) (kappa(P)
//           beyond about 3e6, where CholeskyQR2 loses orthogonality);
//   pass 2: fail unless max |G - I| < 0.1 (the first pass was accurate
//           enough for the second to reach orthogonality to rounding).
//           When max |G - I| <= 2^-30 (any panel with kappa up to about
//           1e4), G = I + E and the factors are taken from the expansion
//           R = I + N + D/2, R^-1 = I - N - D/2 (N the strictly upper part
//           of E, D its diagonal), whose neglected terms are at most
//           n max|E|^2 <= 2^-53 in each entry: rounding level, without the
//           sequential factorization.
// flag: stores the verdict if `overwrite`, else ORs into it.
__global__ __launch_bounds__(kThreads) void k_hr_chol(int n, int nt, const double* __restrict__ G,
                                                      int ldg, double* __restrict__ R,
                                                      double* __restrict__ Ri, int pass,
                                                      int overwrite, int* flag) {
  __shared__ Smem sm;
  const int tid = threadIdx.x;
  const int nbp = nt * TS;
  if (tid == 0) sm.fail = 0;
  double m = 0.0;
  {
    // All loads first (clamped indices keep them in bounds), then the stores:
    // one memory round trip instead of one per column group.
    const int i = tid % kBlk, j0 = tid / kBlk;
    double g[kBlk / kLoadCols];
#pragma unroll
    for (int r = 0; r < kBlk / kLoadCols; ++r) {
      const int j = j0 + kLoadCols * r;
      g[r] = G[min(i, n - 1) + (int64_t)min(j, n - 1) * ldg];
    }
#pragma unroll
    for (int r = 0; r < kBlk / kLoadCols; ++r) {
      const int j = j0 + kLoadCols * r;
      const bool in = i < n && j < n;
      const double v = in ? g[r] : (i == j ? 1.0 : 0.0);
      if (i < nbp && j < nbp) sm.A[i + j * LDA] = v;
      if (in) {
        if (pass == 1) {
          if (i == j) m = fmax(m, v);
        } else {
          m = fmax(m, fabs(v - (i == j ? 1.0 : 0.0)));
        }
        if (!(v == v)) m = __builtin_inf();  // NaN input: fail below
      }
    }
  }
  __syncthreads();
  const double gm = block_max(m, sm.red);
  double thr;
  if (pass == 1) {
    if (tid == 0 && (!(gm > 0.0) || !(gm < __builtin_inf()))) sm.fail = 1;
    thr = 1e-13 * gm;
  } else {
    if (tid == 0 && !(gm < 0.1)) sm.fail = 1;
    thr = 0.5;
  }
  __syncthreads();
  if (pass == 2 && gm <= kNearIdentity) {
    for (int j = elem_j0(nbp), i = (tid) % nbp; j < nbp; j += kThreads / nbp) {
      const int idx = i + j * nbp;
      const double e = sm.A[i + j * LDA] - (i == j ? 1.0 : 0.0);
      R[idx] = i < j ? e : (i == j ? 1.0 + 0.5 * e : 0.0);
      Ri[idx] = i < j ? -e : (i == j ? 1.0 - 0.5 * e : 0.0);
    }
    if (tid == 0) {
      if (overwrite) *flag = sm.fail;
      else if (sm.fail) *flag = 1;
    }
    return;
  }
  chol_inv_lds(sm, n, nt, thr, R);
  for (int j = elem_j0(nbp), i = (tid) % nbp; j < nbp; j += kThreads / nbp) {
    const int idx = i + j * nbp;
    Ri[idx] = sm.A[i + j * LDA];
    if (i > j) R[idx] = 0.0;
  }
  if (tid == 0) {
    if (overwrite) *flag = sm.fail;
    else if (sm.fail) *flag = 1;
  }
}

// LU of B = QT - S (QT = top n x n block of the orthonormal factor, padded
// with an identity block), with s_k = -sign(pivot) chosen as the pivot is
// reached (sign(0) = +1), so |u_kk| = |pivot| + 1 >= 1.  Outputs:
//   V(0:n, 0:n) = L1 (unit lower, explicit ones and zeros), ld ldv;
//   Ui = U^-1, Li = L1^-1, US = U S (nbp x nbp, ld nbp), the inverses built
//   in the factorization loop (block column kt of U^-1 and block row kt of
//   L1^-1 once U(:, kt) and L1(kt, :) are final);
//   tau_k = -u_kk s_k;  Rout = S * RF (upper, zeros below) if Rout != NULL.
// Flags a column whose pivot has |p| >= 1 - 2^-50: its tail below the
// diagonal is zero, where dlarfg takes tau = 0 instead.  The one exception
// is the last column of a square panel (square != 0), whose tail is empty:
// there dlarfg keeps alpha (tau = 0, R(n,n) = alpha), which is s = sign(p)
// and u = 0 here.
__global__ __launch_bounds__(kThreads) void k_hr_lu(
    int n, int nt, int square, const double* __restrict__ QT, int ldq,
    double* __restrict__ Ui, double* __restrict__ Li, double* __restrict__ US,
    const double* __restrict__ RF, int ldrf, double* __restrict__ V, int64_t ldv,
    double* __restrict__ Rout, int64_t ldr, double* __restrict__ tau, int* flag) {
  __shared__ Smem sm;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nbp = nt * TS;
  if (tid == 0) sm.fail = 0;
  {
    const int i = tid % kBlk, j0 = tid / kBlk;
    double g[kBlk / kLoadCols];
#pragma unroll
    for (int r = 0; r < kBlk / kLoadCols; ++r) {
      const int j = j0 + kLoadCols * r;
      g[r] = QT[min(i, n - 1) + min(j, n - 1) * ldq];
    }
#pragma unroll
    for (int r = 0; r < kBlk / kLoadCols; ++r) {
      const int j = j0 + kLoadCols * r;
      if (i < nbp && j < nbp) sm.A[i + j * LDA] = (i < n && j < n) ? g[r] : (i == j ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  // Diagonal tile kt, by wave 0: packed L \ U into the tile, L_kk^-1 and
  // U_kk^-1 (unused for the last tile of a square panel) into D[kt & 1] and
  // D2[kt & 1].
  auto diag = [&](int kt) {
    bool bad = false;
    double a[TS], xl[TS], xu[TS];
    double* Akk = tile(sm, kt, kt);
    col_load(Akk, LDA, a);
    lu_inv16(a, xl, xu, kt * TS, n, square ? n - 1 : -1, sm.sgn, tau, bad);
    col_store(Akk, LDA, a);
    col_store(sm.D[kt & 1], 17, xl);
    col_store(sm.D2[kt & 1], 17, xu);
    if (bad && lane == 0) sm.fail = 1;
  };
  if (wave == 0) diag(0);
  __syncthreads();
  for (int kt = 0; kt < nt; ++kt) {
    const int k0 = kt * TS;
    double* Akk = tile(sm, kt, kt);
    const double* D = sm.D[kt & 1];
    const double* D2 = sm.D2[kt & 1];
    // U(kt, jt) = L_kk^-1 A(kt, jt), L(it, kt) = A(it, kt) U_kk^-1 (it, jt > kt).
    // Block column kt of U and block row kt of L are then final: US = U S and
    // the top of V go out, and they are replaced by U(k, kt) U_kk^-1 and
    // L_kk^-1 L(kt, k) (k < kt) for the inverses.
    const int nr = nt - 1 - kt;
    for (int t = wave; t < 2 * nr + 2 * kt + 1; t += kWaves) {
      if (t < nr) {
        double* At = tile(sm, kt, kt + 1 + t);
        tile_store(At, LDA, tile_mma<false, false>(vzero(), D, 17, At, LDA));
      } else if (t < 2 * nr) {
        double* At = tile(sm, kt + 1 + (t - nr), kt);
        tile_store(At, LDA, tile_mma<false, false>(vzero(), At, LDA, D2, 17));
      } else if (t < 2 * nr + kt + 1) {  // U(k, kt), k <= kt
        const int k = t - 2 * nr;
        double* At = tile(sm, k, kt);
        const int l = lane;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = (l >> 4) + 4 * r, j = l & 15;
          const int gi = k * TS + i, gj = kt * TS + j;
          const double u = (k < kt || i <= j) ? At[i + j * LDA] : 0.0;
          US[gi + (int64_t)gj * nbp] = u * sm.sgn[gj];
        }
        if (k < kt) tile_store(At, LDA, tile_mma<false, false>(vzero(), At, LDA, D2, 17));
      } else {  // L(kt, k), k < kt, and the diagonal block's unit lower part
        const int k = t - 2 * nr - kt - 1;
        double* At = tile(sm, kt, k);
        const int l = lane;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = (l >> 4) + 4 * r, j = l & 15;
          const int gi = kt * TS + i, gj = k * TS + j;
          if (gi < n && gj < n) V[gi + (int64_t)gj * ldv] = At[i + j * LDA];
        }
        tile_store(At, LDA, tile_mma<false, false>(vzero(), D, 17, At, LDA));
      }
    }
    if (wave == 0) {  // diagonal block of V (unit lower; its zeros above come at the end)
      const int l = lane;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = (l >> 4) + 4 * r, j = l & 15;
        const int gi = k0 + i, gj = k0 + j;
        if (gi < n && gj < n) V[gi + (int64_t)gj * ldv] = i > j ? Akk[i + j * LDA] : (i == j ? 1.0 : 0.0);
      }
    }
    __syncthreads();
    // trailing A(it, jt) -= L(it, kt) U(kt, jt), and block column kt of U^-1
    // and block row kt of L^-1 (packed diagonal tiles read through masks):
    //   X(i, kt) = -sum_{k=i}^{kt-1} X(i, k) U'(k, kt),
    //   Y(kt, j) = -sum_{k=j}^{kt-1} L'(kt, k) Y(k, j).
    // Look-ahead: wave 0 updates tile (kt+1, kt+1) first and factors it while
    // the other waves do the rest.
    v4d xi = vzero(), yj = vzero();
    int myi = -1, myj = -1;
    if (wave == 0) {
      if (nr > 0) {
        double* At = tile(sm, kt + 1, kt + 1);
        v4d acc = tile_load(At, LDA);
        const v4d p = tile_mma<false, false>(vzero(), tile(sm, kt + 1, kt), LDA,
                                             tile(sm, kt, kt + 1), LDA);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] -= p[r];
        tile_store(At, LDA, acc);
        diag(kt + 1);
      }
    } else {
      const int ntask = 2 * kt + (nr > 0 ? nr * nr - 1 : 0);
      for (int t = wave - 1; t < ntask; t += kWaves - 1) {
        if (t < kt) {
          const int i = t;
          v4d z = vzero();
          for (int k = i; k < kt; ++k)
            z = tile_mma_m(z, tile(sm, i, k), LDA, k == i ? 1 : 0, tile(sm, k, kt), LDA, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) xi[r] = -z[r];
          myi = i;
        } else if (t < 2 * kt) {
          const int j = t - kt;
          v4d z = vzero();
          for (int k = j; k < kt; ++k)
            z = tile_mma_m(z, tile(sm, kt, k), LDA, 0, tile(sm, k, j), LDA, k == j ? 2 : 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) yj[r] = -z[r];
          myj = j;
        } else {
          const int u = t - 2 * kt + 1;  // u = 0, tile (kt+1, kt+1), is wave 0's
          const int it = kt + 1 + u % nr, jt = kt + 1 + u / nr;
          double* At = tile(sm, it, jt);
          v4d acc = tile_load(At, LDA);
          const v4d p = tile_mma<false, false>(vzero(), tile(sm, it, kt), LDA, tile(sm, kt, jt), LDA);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r] -= p[r];
          tile_store(At, LDA, acc);
        }
      }
    }
    __syncthreads();
    if (myi >= 0) tile_store(tile(sm, myi, kt), LDA, xi);
    if (myj >= 0) tile_store(tile(sm, kt, myj), LDA, yj);
    if (wave == kWaves - 1) {  // packed inverse of the diagonal block
      const int l = lane;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = (l >> 4) + 4 * r, j = l & 15;
        Akk[i + j * LDA] = i <= j ? D2[i + j * 17] : D[i + j * 17];
      }
    }
    __syncthreads();
  }
  // Outputs: U^-1 and L1^-1 from the packed inverses, the zeros of V above
  // its diagonal, then S R with the RF loads issued eight at a time.
  {
    const int i = tid % kBlk, j0 = tid / kBlk;
#pragma unroll 4
    for (int r = 0; r < kBlk / kLoadCols; ++r) {
      const int j = j0 + kLoadCols * r;
      if (i < nbp && j < nbp) {
        const int idx = i + j * nbp;
        const double a = sm.A[i + j * LDA];
        Ui[idx] = i <= j ? a : 0.0;
        Li[idx] = i > j ? a : (i == j ? 1.0 : 0.0);
        if (i > j) US[idx] = 0.0;
        if (i < j && j < n) V[i + (int64_t)j * ldv] = 0.0;
      }
    }
    if (Rout) {
      constexpr int kBatch = 8;
#pragma unroll 1
      for (int r0 = 0; r0 < kBlk / kLoadCols; r0 += kBatch) {
        double rf[kBatch];
#pragma unroll
        for (int r = 0; r < kBatch; ++r) {
          const int j = j0 + kLoadCols * (r0 + r);
          rf[r] = RF[min(i, n - 1) + (int64_t)min(j, n - 1) * ldrf];
        }
#pragma unroll
        for (int r = 0; r < kBatch; ++r) {
          const int j = j0 + kLoadCols * (r0 + r);
          if (i < n && j < n) Rout[i + (int64_t)j * ldr] = i <= j ? sm.sgn[i] * rf[r] : 0.0;
        }
      }
    }
  }
  if (tid == 0 && sm.fail) *flag = 1;
}

// Inverse of an n x n (n <= 128) upper-triangular (upper != 0) or
// unit-lower-triangular (diagonal taken as 1) matrix; entries outside the
// triangle are ignored and written as zeros.
__global__ __launch_bounds__(kThreads) void k_tri_inv(int n, int nt, const double* __restrict__ X,
                                                      int64_t ldx, double* __restrict__ Xi,
                                                      int64_t ldxi, int upper) {
  __shared__ Smem sm;
  const int nbp = nt * TS;
  for (int j = elem_j0(nbp), i = (threadIdx.x) % nbp; j < nbp; j += kThreads / nbp) {
    double v = i == j ? 1.0 : 0.0;
    if (i < n && j < n && (upper ? i <= j : i > j)) v = X[i + (int64_t)j * ldx];
    sm.A[i + j * LDA] = v;
  }
  __syncthreads();
  if (upper) inv_upper_lds(sm, nt);
  else inv_unit_lower_lds(sm, nt);
  for (int idx = threadIdx.x; idx < n * n; idx += kThreads) {
    const int i = idx % n, j = idx / n;
    Xi[i + (int64_t)j * ldxi] = sm.A[i + j * LDA];
  }
}

// Writes R (upper) and the reflector tails (below) back into the dgeqrf
// layout of P, for callers that want LAPACK's packed form.
__global__ void k_pack_qr(int Mp, int nb, const double* __restrict__ V, int64_t ldv,
                          const double* __restrict__ R, int64_t ldr, double* __restrict__ P,
                          int64_t ldp) {
  const int64_t total = (int64_t)Mp * nb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % Mp);
    const int j = (int)(idx / Mp);
    P[i + (int64_t)j * ldp] = i <= j ? R[i + (int64_t)j * ldr] : V[i + (int64_t)j * ldv];
  }
}

}  // namespace

size_t hr_work_bytes(int64_t Mp_max, int nb_max) {
  (void)nb_max;
  return (size_t)(13 * kBlk * kBlk + 2 * Mp_max * (int64_t)kBlk) * sizeof(double) + 256;
}

void hr_work_carve(void* base, int64_t Mp_max, int nb_max, HrWork* w) {
  (void)nb_max;
  double* p = (double*)base;
  double** slots[] = {&w->G,  &w->R1, &w->R1i, &w->R2, &w->R2i, &w->RF, &w->QT,
                      &w->LU, &w->Ui, &w->Li,  &w->US, &w->Wc,  &w->Cc};
  for (double** s : slots) {
    *s = p;
    p += kBlk * kBlk;
  }
  w->Q1 = p;
  p += Mp_max * (int64_t)kBlk;
  w->P2 = p;
  p += Mp_max * (int64_t)kBlk;
  w->flag = (int*)p;
}

namespace {

// One block of n <= 128 columns: CholeskyQR2, then Householder
// reconstruction.  P is only read.  The flag is reset when `first`.
hipError_t hr_block(hipStream_t st, int Mp, int n, const double* P, int64_t ldp, double* V,
                    int64_t ldv, double* Rout, int64_t ldr, double* tau, double* Tw, int64_t ldtw,
                    const HrWork& hw, double* split, size_t se, bool first) {
  const int nt = (n + TS - 1) / TS, nbp = nt * TS;
  hipError_t e;
#define HR_CHK(x)                           \
  do {                                      \
    if ((e = (x)) != hipSuccess) return e;  \
  } while (0)
  // pass 1: G = P^T P, R1 = chol(G), Q1 = P R1^-1
  HR_CHK(gemm(st, PREC_FP64, true, false, n, n, Mp, 1.0, P, ldp, P, ldp, 0.0, hw.G, nbp, split, se));
  hipLaunchKernelGGL(k_hr_chol, dim3(1), dim3(kThreads), 0, st, n, nt, hw.G, nbp, hw.R1, hw.R1i, 1,
                     first ? 1 : 0, hw.flag);
  HR_CHK(gemm(st, PREC_FP64, false, false, Mp, n, n, 1.0, P, ldp, hw.R1i, nbp, 0.0, hw.Q1, Mp,
              split, se));
  // pass 2: G = Q1^T Q1, R2 = chol(G); R = R2 R1; top block of Q = Q1 R2^-1
  HR_CHK(gemm(st, PREC_FP64, true, false, n, n, Mp, 1.0, hw.Q1, Mp, hw.Q1, Mp, 0.0, hw.G, nbp,
              split, se));
  hipLaunchKernelGGL(k_hr_chol, dim3(1), dim3(kThreads), 0, st, n, nt, hw.G, nbp, hw.R2, hw.R2i, 2,
                     0, hw.flag);
  HR_CHK(gemm(st, PREC_FP64, false, false, n, n, n, 1.0, hw.R2, nbp, hw.R1, nbp, 0.0, hw.RF, nbp,
              nullptr, 0));
  HR_CHK(gemm(st, PREC_FP64, false, false, n, n, n, 1.0, hw.Q1, Mp, hw.R2i, nbp, 0.0, hw.QT, nbp,
              nullptr, 0));
  // Householder reconstruction: LU of Q(0:n,:) - S; V top block, tau, S R.
  hipLaunchKernelGGL(k_hr_lu, dim3(1), dim3(kThreads), 0, st, n, nt, Mp == n ? 1 : 0, hw.QT, nbp,
                     hw.Ui, hw.Li, hw.US, hw.RF, nbp, V, ldv, Rout, ldr, tau, hw.flag);
  // V(n:Mp, :) = Q(n:Mp, :) U^-1 = Q1(n:Mp, :) (R2^-1 U^-1); Tw = -U S L1^-T.
  if (Mp > n) {
    HR_CHK(gemm(st, PREC_FP64, false, false, n, n, n, 1.0, hw.R2i, nbp, hw.Ui, nbp, 0.0, hw.R1i,
                nbp, nullptr, 0));
    HR_CHK(gemm(st, PREC_FP64, false, false, Mp - n, n, n, 1.0, hw.Q1 + n, Mp, hw.R1i, nbp, 0.0,
                V + n, ldv, split, se));
  }
  HR_CHK(gemm(st, PREC_FP64, false, true, n, n, n, -1.0, hw.US, nbp, hw.Li, nbp, 0.0, Tw, ldtw,
              nullptr, 0));
#undef HR_CHK
  return hipGetLastError();
}

hipError_t hr_panel(hipStream_t st, int Mp, int nb, double* P, int64_t ldp, double* V,
                    int64_t ldv, double* Rout, int64_t ldr, double* tau, double* Tw, int64_t ldtw,
                    const HrWork& hw, double* split, size_t se) {
  if (nb <= kBlk) return hr_block(st, Mp, nb, P, ldp, V, ldv, Rout, ldr, tau, Tw, ldtw, hw, split, se, true);
  // Two blocks: [P1 P2], n1 = 128.  H1 = I - V1 Tw1 V1^T from the first;
  // the second factors the trailing rows of H1^T P2 (a copy); then
  // Tw = [Tw1, -Tw1 (V1^T V2) Tw2; 0, Tw2] and R = [R11, (H1^T P2)(0:n1,:); 0, R22].
  const int n1 = kBlk, n2 = nb - kBlk;
  hipError_t e;
#define HR_CHK(x)                           \
  do {                                      \
    if ((e = (x)) != hipSuccess) return e;  \
  } while (0)
  HR_CHK(hr_block(st, Mp, n1, P, ldp, V, ldv, Rout, ldr, tau, Tw, ldtw, hw, split, se, true));
  double* P2 = hw.P2;
  HR_CHK(copy_matrix(st, Mp, n2, P + (int64_t)n1 * ldp, ldp, P2, Mp));
  HR_CHK(gemm(st, PREC_FP64, true, false, n1, n2, Mp, 1.0, V, ldv, P2, Mp, 0.0, hw.Wc, kBlk, split, se));
  HR_CHK(gemm(st, PREC_FP64, true, false, n1, n2, n1, 1.0, Tw, ldtw, hw.Wc, kBlk, 0.0, hw.Cc, kBlk,
              nullptr, 0));
  HR_CHK(gemm(st, PREC_FP64, false, false, Mp, n2, n1, -1.0, V, ldv, hw.Cc, kBlk, 1.0, P2, Mp,
              nullptr, 0));
  double* V2 = V + n1 + (int64_t)n1 * ldv;
  double* Tw2 = Tw + n1 + (int64_t)n1 * ldtw;
  HR_CHK(hr_block(st, Mp - n1, n2, P2 + n1, Mp, V2, ldv, Rout ? Rout + n1 + (int64_t)n1 * ldr : nullptr,
                  ldr, tau + n1, Tw2, ldtw, hw, split, se, false));
  HR_CHK(set_zero(st, n1, n2, V + (int64_t)n1 * ldv, ldv));
  if (Rout) {
    HR_CHK(copy_matrix(st, n1, n2, P2, Mp, Rout + (int64_t)n1 * ldr, ldr));
    HR_CHK(set_zero(st, n2, n1, Rout + n1, ldr));
  }
  HR_CHK(gemm(st, PREC_FP64, true, false, n1, n2, Mp - n1, 1.0, V + n1, ldv, V2, ldv, 0.0, hw.Wc,
              kBlk, split, se));
  HR_CHK(gemm(st, PREC_FP64, false, false, n1, n2, n1, 1.0, Tw, ldtw, hw.Wc, kBlk, 0.0, hw.Cc, kBlk,
              nullptr, 0));
  HR_CHK(gemm(st, PREC_FP64, false, false, n1, n2, n2, -1.0, hw.Cc, kBlk, Tw2, ldtw, 0.0,
              Tw + (int64_t)n1 * ldtw, ldtw, nullptr, 0));
  HR_CHK(set_zero(st, n2, n1, Tw + n1, ldtw));
#undef HR_CHK
  return hipSuccess;
}

}  // namespace

hipError_t panel_qr_hr(hipStream_t st, int Mp, int nb, double* P, int64_t ldp, double* V,
                       int64_t ldv, double* Rout, int64_t ldr, double* tau, double* Tw,
                       int64_t ldtw, const HrWork& hw, const PanelWork& pw, double* split,
                       size_t split_elems) {
  if (nb <= 0) return hipSuccess;
  if (nb > 2 * kBlk || Mp < nb) return hipErrorInvalidValue;
  const int slot = prof_mark(st, PC_PANEL);
  prof_suppress(1);
  gemm_panel_scope(1);
  hipError_t e = hr_panel(st, Mp, nb, P, ldp, V, ldv, Rout, ldr, tau, Tw, ldtw, hw, split,
                          split_elems);
  // Fallback, gated on the flag: column-by-column Householder of the
  // (untouched) panel, then its V and R.
  if (e == hipSuccess) e = panel_qr(st, Mp, nb, P, ldp, tau, Tw, ldtw, pw, hw.flag);
  if (e == hipSuccess) e = panel_extract(st, Mp, nb, P, ldp, V, ldv, Rout, ldr, hw.flag);
  gemm_panel_scope(-1);
  prof_suppress(-1);
  prof_done(st, slot, PC_PANEL, 2.0 * Mp * (double)nb * nb, 16.0 * Mp * (double)nb);
  return e == hipSuccess ? hipGetLastError() : e;
}

hipError_t tri_inv(hipStream_t st, int n, const double* X, int64_t ldx, double* Xi, int64_t ldxi,
                   bool upper) {
  if (n <= 0) return hipSuccess;
  if (n > kBlk) return hipErrorInvalidValue;
  const int nt = (n + TS - 1) / TS;
  hipLaunchKernelGGL(k_tri_inv, dim3(1), dim3(kThreads), 0, st, n, nt, X, ldx, Xi, ldxi,
                     upper ? 1 : 0);
  return hipGetLastError();
}

hipError_t pack_qr(hipStream_t st, int Mp, int nb, const double* V, int64_t ldv,
                   const double* R, int64_t ldr, double* P, int64_t ldp) {
  const int64_t total = (int64_t)Mp * nb;
  if (total == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pack_qr, dim3(blocks), dim3(256), 0, st, Mp, nb, V, ldv, R, ldr, P, ldp);
  return hipGetLastError();
}

}  // namespace rutv
