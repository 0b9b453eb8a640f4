// SVD of the small diagonal blocks (Figure "The algorithm randUTV": the SVD
// of each step's b x b block R; Section 2.4 eq. smallSVD).
//
// One-sided (Hestenes) Jacobi on the transpose: the columns of W = R^T are
// rotated pairwise until mutually orthogonal, accumulating the rotations in
// V, so that W = R^T V has orthogonal columns of norms sigma_j and
// R = V Sigma (W Sigma^-1)^T: the rotations are R's left singular vectors
// and the normalized columns of W its right ones.  The R blocks come from
// Householder QRs and their rows are graded; Jacobi on the rows converges
// in far fewer sweeps than on the columns (an over-sampled 138 x 138 factor
// of the 4000 x 4000 workload: 9 sweeps against 21; a 256 x 256 block of the
// 8000 x 8000 one: 10 against 11).
//
// Block form for the GPU: the columns are cut into blocks of kBW.  Each
// launch of k_bj_round is one round of a round-robin tournament over the
// blocks: a workgroup takes one pair of blocks, holds their columns of W
// and V in LDS, and rotates every column pair across the two blocks once
// (plus, in the first round of a sweep, the pairs inside each block), so a
// sweep visits every column pair exactly once, as cyclic scalar Jacobi
// does.  Each 16-lane DPP row of a wave takes one pair of a sub-round (four
// pairs per wave, the kBW pairs of a sub-round on four waves, one per
// SIMD), so the scalar rotation arithmetic of four pairs shares each
// instruction, and in the cross sub-rounds a row keeps its block-bp column
// in registers while the block-bq columns move between rows, by lane
// shuffles inside a wave and through LDS between waves.  Blocks stay in
// place in global memory, so
// the kernel boundary between rounds is the only synchronization.  A sweep
// is nblk-1 rounds; the SVDs of all randUTV steps advance together (grid.y
// = matrix), and a matrix stops as soon as a whole sweep rotated nothing:
// later rounds see that on the device and return at once, so the host
// enqueues the whole sweep budget without waiting.
//
// Output conventions: sigma descending (ties by index); each (u_j, v_j)
// flipped so the largest-magnitude entry of v_j is positive (first index on
// ties); columns of Vs with sigma_j == 0 are completed by Gram-Schmidt on
// e_1, e_2, ... (and then signed the same way).  Matrices wider than
// kMaxLdsN use a single-workgroup global-memory kernel.
#include <algorithm>
#include <utility>

#include "common.h"

namespace rutv {
namespace {

constexpr int MAXN = 1024;
constexpr int kBW = 16;          // Jacobi block width
// Lanes per column pair in a round: 16 (one DPP row), the kBW pairs of a
// sub-round on four waves, one per SIMD.  (32 lanes, two DPP rows and eight
// waves so that two per SIMD overlap their latencies, measured the same:
// 31-39 us per round of 256-row blocks either way.)
#ifndef JACOBI_LPP
#define JACOBI_LPP 16
#endif
constexpr int kLPP = JACOBI_LPP;
constexpr int kRoundThreads = kLPP * kBW;
constexpr int kMaxLdsN = 256;    // largest order handled by the LDS block kernel
// Sweeps run as block rounds (a launch per round); the rest of the budget,
// needed only by matrices not converged by then, runs in one launch.  The
// factorization's b x b blocks take about 11 sweeps.
constexpr int kBlockSweeps = 14;
// LDS column stride of a round, in doubles: 16 rows per lane-row chunk plus
// a pad (see k_bj_round).
#ifndef JACOBI_LDS_PAD
#define JACOBI_LDS_PAD 1
#endif
constexpr int lds_stride(int nt) { return kLPP * nt + JACOBI_LDS_PAD; }

// DPP move of a double (two 32-bit halves) with control CTRL.
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
__device__ inline double lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the 64 lanes of a wave, the same value in every lane.  Called
// with all lanes active.  Within each row of 16 lanes: butterflies over
// lane ^ 1, lane ^ 2 (quad_perm), the other quad of the half row
// (row_half_mirror) and the other half (row_mirror); then the four row
// sums from lanes 0, 16, 32, 48.  No LDS traffic, unlike a shuffle-based
// butterfly.
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// The largest value over the wave and its index, the smallest index among
// equal values (a total order, so the reduction tree does not matter), in
// every lane.  Same butterflies as wave_sum; called with all lanes active.
template <int CTRL>
__device__ inline void argmax_step(double& best, int& bi) {
  const double ob = dpp_d<CTRL>(best);
  const int oi = __builtin_amdgcn_update_dpp(0, bi, CTRL, 0xF, 0xF, false);
  if (ob > best || (ob == best && oi < bi)) best = ob, bi = oi;
}
__device__ inline void wave_argmax(double& best, int& bi) {
  argmax_step<0xB1>(best, bi);
  argmax_step<0x4E>(best, bi);
  argmax_step<0x141>(best, bi);
  argmax_step<0x140>(best, bi);
  double b = lane_d(best, 0);
  int i = __builtin_amdgcn_readlane(bi, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    const double ob = lane_d(best, r);
    const int oi = __builtin_amdgcn_readlane(bi, r);
    if (ob > b || (ob == b && oi < i)) b = ob, i = oi;
  }
  best = b, bi = i;
}

// Sum over the 16 lanes of a DPP row (the first four steps of wave_sum), in
// every lane of the row.  Called with all lanes active.
__device__ inline double row_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}

__device__ inline double jacobi_tol(int nb) { return 4.0 * 2.220446049250313e-16 * sqrt((double)nb); }

// The rotation (c, s) of the one-sided Jacobi method for two columns with
// squared norms al, be and inner product ga: [x, y] <- [c x - s y, s x + c y]
// makes them orthogonal.  False if they already are, to tolerance.
__device__ inline bool jacobi_cs(double al, double be, double ga, double tol, double* c,
                                 double* s) {
  if (ga == 0.0 || al == 0.0 || be == 0.0) return false;
  if (fabs(ga) <= tol * sqrt(al) * sqrt(be)) return false;
  const double zeta = (be - al) / (2.0 * ga);
  double t;
  if (fabs(zeta) > 1e150) t = 0.5 / zeta;
  else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = *c * t;
  return true;
}

// Rotate columns (wp, wq) of W and (vp, vq) of V so that wp^T wq = 0, if
// they are not already orthogonal to tolerance.  One wave; returns true if
// a rotation was applied.  Column length n, lane-strided.
__device__ inline bool rotate_pair(double* wp, double* wq, double* vp, double* vq, int n,
                                   int lane, double tol) {
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double x = wp[i], y = wq[i];
    al += x * x;
    be += y * y;
    ga += x * y;
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  double c, s;
  if (!jacobi_cs(al, be, ga, tol, &c, &s)) return false;
  for (int i = lane; i < n; i += 64) {
    const double x = wp[i], y = wq[i];
    wp[i] = c * x - s * y;
    wq[i] = s * x + c * y;
  }
  for (int i = lane; i < n; i += 64) {
    const double x = vp[i], y = vq[i];
    vp[i] = c * x - s * y;
    vq[i] = s * x + c * y;
  }
  return true;
}

// Pair k of round r of the round-robin (circle method) over n2 players.
__device__ inline void rr_pair(int n2, int r, int k, int* p, int* q) {
  if (k == 0) {
    *p = r;
    *q = n2 - 1;
  } else {
    *p = (r + k) % (n2 - 1);
    *q = (r - k + n2 - 1) % (n2 - 1);
  }
}

// From the orthogonalized W = R^T V and the rotations V in global memory:
// Us gets V's columns and Vs W's normalized ones, sorted by sigma_j =
// ||w_j||, each pair signed by its Vs column; Vs columns with sigma = 0 are
// completed.  Whole workgroup; sig, ssig, sgn (doubles) and rank (ints)
// are LDS arrays of nb entries.
__device__ void finish_svd(int nb, int ld, const double* __restrict__ W,
                           const double* __restrict__ V, double* __restrict__ Uo,
                           double* __restrict__ Vo, double* __restrict__ Do, double* sig,
                           double* ssig, double* sgn, int* rank) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  // Per column j (unsorted): sigma_j = ||w_j|| and the sign that makes the
  // largest-magnitude entry of w_j (of v_j = w_j / sigma_j) positive, first
  // index on ties.  Four columns per wave at a time, so that their loads
  // are in flight together.
  for (int j0 = 4 * wave; j0 < nb; j0 += 4 * nw) {
    double s[4] = {0.0, 0.0, 0.0, 0.0}, best[4] = {-1.0, -1.0, -1.0, -1.0};
    int bi[4] = {0, 0, 0, 0};
    for (int i = lane; i < nb; i += 64) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int j = j0 + k < nb ? j0 + k : j0;
        const double x = W[i + (int64_t)j * ld];
        s[k] += x * x;
        if (fabs(x) > best[k]) best[k] = fabs(x), bi[k] = i;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double sk = wave_sum(s[k]);
      wave_argmax(best[k], bi[k]);
      if (lane == 0 && j0 + k < nb) {
        sig[j0 + k] = sqrt(sk);
        sgn[j0 + k] = W[bi[k] + (int64_t)(j0 + k) * ld] < 0.0 ? -1.0 : 1.0;
      }
    }
  }
  __syncthreads();
  for (int j = tid; j < nb; j += blockDim.x) {
    int rk = 0;
    const double sj = sig[j];
    for (int k = 0; k < nb; ++k) rk += (sig[k] > sj) || (sig[k] == sj && k < j);
    rank[j] = rk;
  }
  __syncthreads();
  for (int j = tid; j < nb; j += blockDim.x) ssig[rank[j]] = sig[j];
  // Eight entries per thread at a time, their loads issued together.
  const int nbt = blockDim.x;
  for (int base = 0; base < nb * nb; base += 8 * nbt) {
    double wv[8], vv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int idx = base + k * nbt + tid;
      const int i = idx % nb, j = idx / nb;
      const bool in = idx < nb * nb;
      wv[k] = in ? W[i + (int64_t)j * ld] : 0.0;
      vv[k] = in ? V[i + (int64_t)j * ld] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int idx = base + k * nbt + tid;
      if (idx >= nb * nb) break;
      const int i = idx % nb, j = idx / nb;
      const int o = rank[j];
      const double sj = sig[j], g = sgn[j];
      Uo[i + (int64_t)o * ld] = g * vv[k];
      Vo[i + (int64_t)o * ld] = sj > 0.0 ? g * (wv[k] / sj) : 0.0;
      if (i == 0) Do[o] = sj;
    }
  }
  __syncthreads();
  // Columns of Vs with sigma = 0 (the last ones): Gram-Schmidt on e_1,
  // e_2, ... against the columns before them; then the pair's sign from the
  // completed column.
  if (wave == 0 && !(ssig[nb - 1] > 0.0)) {
    for (int j = 0; j < nb; ++j) {
      if (ssig[j] > 0.0) continue;  // (a NaN is completed too)
      double* vj = Vo + (int64_t)j * ld;
      for (int e = 0; e < nb; ++e) {
        for (int i = lane; i < nb; i += 64) vj[i] = i == e ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass) {
          for (int k = 0; k < j; ++k) {
            const double* vk = Vo + (int64_t)k * ld;
            double d = 0.0;
            for (int i = lane; i < nb; i += 64) d += vk[i] * vj[i];
            d = wave_sum(d);
            for (int i = lane; i < nb; i += 64) vj[i] -= d * vk[i];
          }
        }
        double nr = 0.0;
        for (int i = lane; i < nb; i += 64) nr += vj[i] * vj[i];
        nr = sqrt(wave_sum(nr));
        if (nr > 0.5 / sqrt((double)nb)) {
          for (int i = lane; i < nb; i += 64) vj[i] = vj[i] / nr;
          break;
        }
      }
      double best = -1.0, bv = 0.0;
      int bi = 0;
      for (int i = lane; i < nb; i += 64)
        if (fabs(vj[i]) > best) best = fabs(vj[i]), bv = vj[i], bi = i;
      wave_argmax(best, bi);
      // The winning entry's value, from the lane that holds it.
      if (lane_d(bv, bi & 63) < 0.0) {
        double* uj = Uo + (int64_t)j * ld;
        for (int i = lane; i < nb; i += 64) {
          vj[i] = -vj[i];
          uj[i] = -uj[i];
        }
      }
    }
  }
}

// ------------------------------------------------------------ block Jacobi
__global__ void k_bj_init(const int* __restrict__ nbs, int ld, const double* __restrict__ R,
                          int64_t strideR, double* __restrict__ Wk, double* __restrict__ Vk,
                          int64_t strideUV, int* __restrict__ rotcount, int max_sweeps) {
  const int mi = blockIdx.y;
  const int nb = nbs[mi];
  const double* Ri = R + mi * strideR;
  double* W = Wk + mi * strideUV;
  double* V = Vk + mi * strideUV;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nb * nb;
       idx += gridDim.x * blockDim.x) {
    const int i = idx % nb, j = idx / nb;
    W[i + (int64_t)j * ld] = Ri[j + (int64_t)i * ld];  // W = R^T
    V[i + (int64_t)j * ld] = i == j ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0)
    for (int s = threadIdx.x; s < max_sweeps; s += blockDim.x) rotcount[mi * max_sweeps + s] = 0;
}

// Sum over the kLPP lanes of a pair (one or two DPP rows), in every lane
// of the pair.  Called with all lanes active.
__device__ inline double pair_sum(double v) {
  v = row_sum(v);
  if (kLPP == 32) v += __shfl_xor(v, 16, 64);
  return v;
}

// Rows i = lp + kLPP t (t < NT) of two columns x, y held in registers,
// rotated by the Jacobi rotation of the pair when `ok` and they are not
// orthogonal to tolerance; otherwise (c, s) = (1, 0) leaves them exactly as
// they are, so the code has no branch.  kLPP lanes per pair; every lane of
// the wave calls it (the sums use DPP).
template <int NT>
__device__ inline bool rotate_regs(double (&xw)[NT], double (&xv)[NT], double (&yw)[NT],
                                   double (&yv)[NT], double tol, bool ok) {
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    al += xw[t] * xw[t];
    be += yw[t] * yw[t];
    ga += xw[t] * yw[t];
  }
  al = pair_sum(al);
  be = pair_sum(be);
  ga = pair_sum(ga);
  double c = 1.0, s = 0.0;
  const bool rot = ok && jacobi_cs(al, be, ga, tol, &c, &s);
  if (!rot) c = 1.0, s = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double x = xw[t], y = yw[t];
    xw[t] = c * x - s * y;
    yw[t] = s * x + c * y;
    const double u = xv[t], v = yv[t];
    xv[t] = c * u - s * v;
    yv[t] = s * u + c * v;
  }
  return rot;
}

// A column of the LDS block: rows lp + kLPP t; the rows from nb to kLPP NT
// hold zeros, which rotations keep.
template <int NT>
__device__ inline void lds_col_load(double (&r)[NT], const double* col, int lp) {
#pragma unroll
  for (int t = 0; t < NT; ++t) r[t] = col[lp + kLPP * t];
}
template <int NT>
__device__ inline void lds_col_store(const double (&r)[NT], double* col, int lp) {
#pragma unroll
  for (int t = 0; t < NT; ++t) col[lp + kLPP * t] = r[t];
}

// Binary reflected Gray code: gray(r) and gray(r + 1) differ in one bit.
__device__ constexpr int gray(int r) { return r ^ (r >> 1); }
// How many of the moves before sub-round r + 1 cross waves (the moves whose
// bit is at least 64 / kLPP slots), counting the one after sub-round r.
__device__ constexpr int cross_move_index(int r) {
  int c = 0;
  for (int i = 0; i < r; ++i)
    if ((gray(i) ^ gray(i + 1)) * kLPP >= 64) ++c;
  return c;
}
// Exchange a register column with the lanes LANES apart (16 or 32: the
// other DPP row of a row pair, or the other half of the wave).
template <int LANES, int NT>
__device__ inline void swap_rows(double (&r)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) r[t] = __shfl_xor(r[t], LANES, 64);
}

// One round of the block tournament: every column pair across blocks bp and
// bq (and in round 0 the pairs inside each of them).  NT = ceil(ld / kLPP)
// rows per lane.
template <int NT>
__global__ __launch_bounds__(kRoundThreads) void k_bj_round(const int* __restrict__ nbs, int ld,
                                                  double* __restrict__ Wk, double* __restrict__ Vk,
                                                  int64_t strideUV, int* __restrict__ rotcount,
                                                  int max_sweeps, int sweep, int round) {
  extern __shared__ double sm[];
  const int mi = blockIdx.y, pi = blockIdx.x;
  const int nb = nbs[mi];
  const int nblk = (nb + kBW - 1) / kBW;
  const int nblk2 = nblk + (nblk & 1);
  if (nb <= 1 || pi >= nblk2 / 2 || round >= nblk2 - 1) return;
  if (sweep > 0 && rotcount[mi * max_sweeps + sweep - 1] == 0) return;  // converged
  int bp, bq;
  rr_pair(nblk2, round, pi, &bp, &bq);
  constexpr int ldl = lds_stride(NT);  // LDS column stride: kLPP NT rows and the pad
  double* sW = sm;
  double* sV = sm + 2 * kBW * ldl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int slot = tid / kLPP, lp = tid % kLPP;  // pair index, lane in the pair
  constexpr int kWaves = kRoundThreads / 64;
  double* W = Wk + mi * strideUV;
  double* V = Vk + mi * strideUV;
  auto gcol = [&](int c) -> int {  // global column of local column c, or -1
    const int blk = c < kBW ? bp : bq;
    const int g = blk * kBW + (c % kBW);
    return (blk < nblk && g < nb) ? g : -1;
  };
  // Wave w loads columns w, w + kWaves, ... of the pair, rows lane + 64 u,
  // and issues every load before its first LDS store: with one workgroup
  // per CU the round is otherwise bound by the latency of these loads.
  constexpr int NU = (kLPP * NT + 63) / 64;  // 64-row chunks per column
  constexpr int kCols = 2 * kBW / kWaves;
  {
    double lw[kCols][NU], lv[kCols][NU];
#pragma unroll
    for (int v = 0; v < kCols; ++v) {
      const int g = gcol(wave + kWaves * v);
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int i = lane + 64 * u;
        const bool in = g >= 0 && i < nb;
        lw[v][u] = in ? W[i + (int64_t)g * ld] : 0.0;
        lv[v][u] = in ? V[i + (int64_t)g * ld] : 0.0;
      }
    }
#pragma unroll
    for (int v = 0; v < kCols; ++v) {
      const int c = wave + kWaves * v;
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int i = lane + 64 * u;
        if (i < kLPP * NT) {  // zeros from row nb on
          sW[c * ldl + i] = lw[v][u];
          sV[c * ldl + i] = lv[v][u];
        }
      }
    }
  }
  const double tol = jacobi_tol(nb);
  bool rot = false;
  double xw[NT], xv[NT], yw[NT], yv[NT];
  __syncthreads();
  // Round 0 of a sweep also visits the pairs inside each block (every block
  // is in exactly one pair per round): round-robin over the kBW columns of
  // each of the two blocks, kBW / 2 pairs per block and sub-round.
  if (round == 0) {
    for (int r = 0; r < kBW - 1; ++r) {
      const int half = slot / (kBW / 2), kk = slot % (kBW / 2);
      int p, q;
      rr_pair(kBW, r, kk, &p, &q);
      p += half * kBW;
      q += half * kBW;
      lds_col_load(xw, sW + p * ldl, lp);
      lds_col_load(xv, sV + p * ldl, lp);
      lds_col_load(yw, sW + q * ldl, lp);
      lds_col_load(yv, sV + q * ldl, lp);
      rot |= rotate_regs(xw, xv, yw, yv, tol, gcol(p) >= 0 && gcol(q) >= 0);
      lds_col_store(xw, sW + p * ldl, lp);
      lds_col_store(xv, sV + p * ldl, lp);
      lds_col_store(yw, sW + q * ldl, lp);
      lds_col_store(yv, sV + q * ldl, lp);
      __syncthreads();
    }
  }
  // Cross pairs (column p of block bp, column j of block bq): kBW
  // sub-rounds; in sub-round r the pair slot p, which keeps column p of bp
  // in registers throughout, meets column j = p ^ gray(r) of bq, so over the
  // kBW sub-rounds it meets every column of bq once.  Between sub-rounds r
  // and r + 1 the bq columns move from slot p ^ m to slot p, m = gray(r) ^
  // gray(r + 1) a single bit: for m = 1 and 2 the two slots are DPP rows of
  // one wave (lanes ^ 16, ^ 32) and the columns cross by lane shuffles; for
  // m = 4 and 8 (three of the kBW - 1 moves) they cross waves through LDS.
  const int p = slot;
  const bool okp = gcol(p) >= 0;
  lds_col_load(xw, sW + p * ldl, lp);
  lds_col_load(xv, sV + p * ldl, lp);
  lds_col_load(yw, sW + (kBW + p) * ldl, lp);
  lds_col_load(yv, sV + (kBW + p) * ldl, lp);
  __syncthreads();  // every slot holds its columns before LDS is written again
#pragma unroll
  for (int r = 0; r < kBW; ++r) {
    const int j = p ^ gray(r);
    rot |= rotate_regs(xw, xv, yw, yv, tol, okp && gcol(kBW + j) >= 0);
    if (r + 1 == kBW) break;
    const int m = gray(r) ^ gray(r + 1);
    if (m * kLPP == 16) {
      swap_rows<16>(yw);
      swap_rows<16>(yv);
    } else if (m * kLPP == 32) {
      swap_rows<32>(yw);
      swap_rows<32>(yv);
    } else {
      // The LDS moves alternate between the halves of the block buffers (bq's
      // first, then bp's, whose columns are in registers by now), so a move
      // never writes where the previous one may still be read.
      const int half = (cross_move_index(r) & 1) ? 0 : kBW;
      lds_col_store(yw, sW + (half + j) * ldl, lp);
      lds_col_store(yv, sV + (half + j) * ldl, lp);
      __syncthreads();
      const int jn = p ^ gray(r + 1);
      lds_col_load(yw, sW + (half + jn) * ldl, lp);
      lds_col_load(yv, sV + (half + jn) * ldl, lp);
    }
  }
  // Both columns of each slot go back from registers: column p of bp and
  // column p ^ gray(kBW - 1) of bq.
  {
    const int gp = gcol(p), gq = gcol(kBW + (p ^ gray(kBW - 1)));
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int i = lp + kLPP * t;
      if (i < nb) {
        if (gp >= 0) {
          W[i + (int64_t)gp * ld] = xw[t];
          V[i + (int64_t)gp * ld] = xv[t];
        }
        if (gq >= 0) {
          W[i + (int64_t)gq * ld] = yw[t];
          V[i + (int64_t)gq * ld] = yv[t];
        }
      }
    }
  }
  if (__syncthreads_or(rot) && tid == 0) atomicAdd(&rotcount[mi * max_sweeps + sweep], 1);
}

using RoundFn = void (*)(const int*, int, double*, double*, int64_t, int*, int, int, int);
template <int... NTs>
RoundFn round_fn(int nt, std::integer_sequence<int, NTs...>) {
  RoundFn fns[] = {k_bj_round<NTs + 1>...};
  return fns[nt - 1];
}

__global__ __launch_bounds__(1024) void k_bj_finish(const int* __restrict__ nbs, int ld,
                                                   const double* __restrict__ Wk,
                                                   const double* __restrict__ Vk,
                                                   int64_t strideUV, double* __restrict__ Us,
                                                   double* __restrict__ Vs,
                                                   double* __restrict__ D, int64_t strideD,
                                                   const int* __restrict__ rotcount,
                                                   int max_sweeps, int* __restrict__ status,
                                                   int* __restrict__ fail) {
  __shared__ double sig[kMaxLdsN], ssig[kMaxLdsN], sgn[kMaxLdsN];
  __shared__ int rank[kMaxLdsN];
  const int mi = blockIdx.x;
  const int nb = nbs[mi];
  if (nb > 0)
    finish_svd(nb, ld, Wk + mi * strideUV, Vk + mi * strideUV, Us + mi * strideUV,
               Vs + mi * strideUV, D + mi * strideD, sig, ssig, sgn, rank);
  if (threadIdx.x == 0) {
    int st = -1;
    for (int s = 0; s < max_sweeps; ++s)
      if (rotcount[mi * max_sweeps + s] == 0) {
        st = s + 1;
        break;
      }
    if (nb <= 1) st = 0;
    status[mi] = st;
    if (st < 0 && fail) atomicOr(fail, 1);
  }
}

// Cyclic one-sided Jacobi sweeps first .. max_sweeps - 1 over W and V in
// global memory, one workgroup (a wave per pair of a round-robin round),
// until a sweep rotates nothing.  Returns the number of sweeps counted from
// 0 (the converged sweep included), or -1 if the budget ran out.  With
// `swept` set, sweep s records whether it rotated in swept[s].  `rotated`
// is an LDS int.
__device__ int cyclic_sweeps(int nb, int ld, double* W, double* V, int first, int max_sweeps,
                             int* swept, int* rotated) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n2 = nb + (nb & 1);
  const double tol = jacobi_tol(nb);
  if (nb <= 1) return first;
  for (int sw = first; sw < max_sweeps; ++sw) {
    if (tid == 0) *rotated = 0;
    __syncthreads();
    for (int r = 0; r < n2 - 1; ++r) {
      for (int k = wave; k < n2 / 2; k += nw) {
        int p, q;
        rr_pair(n2, r, k, &p, &q);
        if (p >= nb || q >= nb) continue;
        if (rotate_pair(W + (int64_t)p * ld, W + (int64_t)q * ld, V + (int64_t)p * ld,
                        V + (int64_t)q * ld, nb, lane, tol) &&
            lane == 0)
          *rotated = 1;
      }
      __syncthreads();
    }
    const bool conv = *rotated == 0;
    if (swept && tid == 0) swept[sw] = conv ? 0 : 1;
    __syncthreads();
    if (conv) return sw + 1;
  }
  return -1;
}

// The sweeps of the budget after the first kBlockSweeps, for the matrices
// that the block rounds have not brought to convergence by then (rare):
// one workgroup per matrix, so that this part costs one launch instead of
// a launch per round when, as usual, every matrix has converged.
__global__ __launch_bounds__(1024) void k_bj_tail(const int* __restrict__ nbs, int ld,
                                                  double* __restrict__ Wk, double* __restrict__ Vk,
                                                  int64_t strideUV, int* __restrict__ rotcount,
                                                  int max_sweeps, int first) {
  __shared__ int rotated;
  const int mi = blockIdx.x;
  const int nb = nbs[mi];
  if (nb <= 1 || rotcount[mi * max_sweeps + first - 1] == 0) return;
  (void)cyclic_sweeps(nb, ld, Wk + mi * strideUV, Vk + mi * strideUV, first, max_sweeps,
                      rotcount + mi * max_sweeps, &rotated);
}

// ------------------------------------------------ single-workgroup fallback
__global__ __launch_bounds__(256) void k_jacobi(const int* __restrict__ nbs, int ld,
                                                const double* __restrict__ R, int64_t strideR,
                                                double* __restrict__ Us,
                                                double* __restrict__ Vs, int64_t strideUV,
                                                double* __restrict__ D, int64_t strideD,
                                                double* __restrict__ Wk, double* __restrict__ Vk,
                                                int* __restrict__ status, int max_sweeps,
                                                int* __restrict__ fail) {
  __shared__ double sig[MAXN], ssig[MAXN], sgn[MAXN];
  __shared__ int rank[MAXN];
  __shared__ int rotated;
  const int mi = blockIdx.x;
  const int nb = nbs[mi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Ri = R + mi * strideR;
  double* W = Wk + mi * strideUV;
  double* V = Vk + mi * strideUV;
  if (nb <= 0) {
    if (tid == 0) status[mi] = 0;
    return;
  }
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int i = idx % nb, j = idx / nb;
    W[i + (int64_t)j * ld] = Ri[j + (int64_t)i * ld];  // W = R^T
    V[i + (int64_t)j * ld] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  const int sweeps = cyclic_sweeps(nb, ld, W, V, 0, max_sweeps, nullptr, &rotated);
  const bool conv = sweeps >= 0;
  finish_svd(nb, ld, W, V, Us + mi * strideUV, Vs + mi * strideUV, D + mi * strideD, sig, ssig,
             sgn, rank);
  if (tid == 0) {
    status[mi] = sweeps;
    if (!conv && fail) atomicOr(fail, 1);
  }
}

}  // namespace

hipError_t batched_svd(hipStream_t st, int count, const int* nb_dev, int ld, const double* R,
                       int64_t strideR, double* Us, double* Vs, int64_t strideUV, double* D,
                       int64_t strideD, double* Wk, double* Vk, int* status, int max_sweeps,
                       int* fail) {
  if (count <= 0) return hipSuccess;
  if (ld > MAXN) return hipErrorInvalidValue;
  const int slot = prof_mark(st, PC_SVD);
  if (ld > kMaxLdsN) {
    hipLaunchKernelGGL(k_jacobi, dim3(count), dim3(256), 0, st, nb_dev, ld, R, strideR, Us, Vs,
                       strideUV, D, strideD, Wk, Vk, status, max_sweeps, fail);
    prof_done(st, slot, PC_SVD, 0.0, 0.0);
    return hipGetLastError();
  }
  constexpr int kMaxNT = kMaxLdsN / kLPP;
  // LDS of a round: W and V columns of two blocks, lds_stride(NT) rows each.
  const int nt = (ld + kLPP - 1) / kLPP;
  const size_t shmem = (size_t)4 * kBW * lds_stride(nt) * sizeof(double);
  const RoundFn round = round_fn(nt, std::make_integer_sequence<int, kMaxNT>());
  {
    const hipError_t e = ensure_dyn_lds((const void*)round, (int)shmem);
    if (e != hipSuccess) return e;
  }
  // Per-matrix sweep counters follow the status words: count * max_sweeps ints.
  int* rotcount = status + count;
  hipLaunchKernelGGL(k_bj_init, dim3(16, count), dim3(256), 0, st, nb_dev, ld, R, strideR, Wk, Vk,
                     strideUV, rotcount, max_sweeps);
  const int nblk = (ld + kBW - 1) / kBW;
  const int nblk2 = nblk + (nblk & 1);
  // The whole sweep budget is enqueued and the convergence decision is taken
  // on the device: a matrix whose last sweep rotated nothing skips every
  // later round (its workgroups return at once), and k_bj_finish reports a
  // matrix that still rotated in the last sweep of the budget.  The host
  // never waits for the device here.
  const int block_sweeps = std::min(max_sweeps, kBlockSweeps);
  for (int sw = 0; sw < block_sweeps; ++sw)
    for (int r = 0; r < nblk2 - 1; ++r)
      hipLaunchKernelGGL(round, dim3(nblk2 / 2, count), dim3(kRoundThreads), shmem, st, nb_dev,
                         ld, Wk, Vk, strideUV, rotcount, max_sweeps, sw, r);
  if (max_sweeps > block_sweeps)
    hipLaunchKernelGGL(k_bj_tail, dim3(count), dim3(1024), 0, st, nb_dev, ld, Wk, Vk, strideUV,
                       rotcount, max_sweeps, block_sweeps);
  hipLaunchKernelGGL(k_bj_finish, dim3(count), dim3(1024), 0, st, nb_dev, ld, Wk, Vk, strideUV, Us,
                     Vs, D, strideD, rotcount, max_sweeps, status, fail);
  prof_done(st, slot, PC_SVD, 0.0, 0.0);
  return hipGetLastError();
}

}  // namespace rutv
