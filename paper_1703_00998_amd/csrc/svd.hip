// SVD of the small diagonal blocks (Figure "The algorithm randUTV": the SVD
// of each step's b x b block R; Section 2.4 eq. smallSVD).
//
// One-sided (Hestenes) Jacobi: columns of W = R are rotated pairwise until
// mutually orthogonal, accumulating the rotations in V; then sigma_j =
// ||w_j|| and u_j = w_j / sigma_j.
//
// Block form for the GPU: the columns are cut into blocks of kBW.  Each
// launch of k_bj_round is one round of a round-robin tournament over the
// blocks: a workgroup takes one pair of blocks, holds their columns of W
// and V in LDS, and rotates every column pair across the two blocks once
// (plus, in the first round of a sweep, the pairs inside each block), so a
// sweep visits every column pair exactly once, as cyclic scalar Jacobi
// does; waves take disjoint pairs.  Blocks stay in place in global memory, so
// the kernel boundary between rounds is the only synchronization.  A sweep
// is nblk-1 rounds; the SVDs of all randUTV steps advance together (grid.y
// = matrix), and a matrix stops as soon as a whole sweep rotated nothing:
// later rounds see that on the device and return at once, so the host
// enqueues the whole sweep budget without waiting.
//
// Output conventions: sigma descending (ties by index); each (u_j, v_j)
// flipped so the largest-magnitude entry of v_j is positive (first index on
// ties); columns of Us with sigma_j == 0 are completed by Gram-Schmidt on
// e_1, e_2, ...  Matrices wider than kMaxLdsN use a single-workgroup
// global-memory kernel.
#include <algorithm>

#include "common.h"

namespace rutv {
namespace {

constexpr int MAXN = 1024;
constexpr int kBW = 16;          // Jacobi block width
constexpr int kRoundThreads = 64 * kBW;  // one wave per column pair of a sub-round
constexpr int kMaxLdsN = 256;    // largest order handled by the LDS block kernel

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

__device__ inline double jacobi_tol(int nb) { return 4.0 * 2.220446049250313e-16 * sqrt((double)nb); }

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
  if (ga == 0.0 || al == 0.0 || be == 0.0) return false;
  if (fabs(ga) <= tol * sqrt(al) * sqrt(be)) return false;
  const double zeta = (be - al) / (2.0 * ga);
  double t;
  if (fabs(zeta) > 1e150) t = 0.5 / zeta;
  else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
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

// From the orthogonalized W (= U Sigma) and V in global memory: sort by
// ||w_j||, normalize, complete zero columns, fix signs.  Whole workgroup.
__device__ void finish_svd(int nb, int ld, const double* W, const double* V, double* Uo,
                           double* Vo, double* Do, double* sig, int* rank) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  for (int j = wave; j < nb; j += nw) {
    double s = 0.0;
    for (int i = lane; i < nb; i += 64) {
      const double x = W[i + (int64_t)j * ld];
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < nb; j += blockDim.x) {
    int rk = 0;
    const double sj = sig[j];
    for (int k = 0; k < nb; ++k) rk += (sig[k] > sj) || (sig[k] == sj && k < j);
    rank[j] = rk;
  }
  __syncthreads();
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    const int i = idx % nb, j = idx / nb;
    const int o = rank[j];
    const double sj = sig[j];
    Vo[i + (int64_t)o * ld] = V[i + (int64_t)j * ld];
    Uo[i + (int64_t)o * ld] = sj > 0.0 ? W[i + (int64_t)j * ld] / sj : 0.0;
    if (i == 0) Do[o] = sj;
  }
  __syncthreads();
  if (wave == 0) {
    for (int j = 0; j < nb; ++j) {
      if (Do[j] > 0.0) continue;
      for (int e = 0; e < nb; ++e) {
        for (int i = lane; i < nb; i += 64) Uo[i + (int64_t)j * ld] = i == e ? 1.0 : 0.0;
        for (int pass = 0; pass < 2; ++pass) {
          for (int k = 0; k < j; ++k) {
            double d = 0.0;
            for (int i = lane; i < nb; i += 64) d += Uo[i + (int64_t)k * ld] * Uo[i + (int64_t)j * ld];
            d = wave_sum(d);
            for (int i = lane; i < nb; i += 64) Uo[i + (int64_t)j * ld] -= d * Uo[i + (int64_t)k * ld];
          }
        }
        double nr = 0.0;
        for (int i = lane; i < nb; i += 64) {
          const double x = Uo[i + (int64_t)j * ld];
          nr += x * x;
        }
        nr = sqrt(wave_sum(nr));
        if (nr > 0.5 / sqrt((double)nb)) {
          for (int i = lane; i < nb; i += 64) Uo[i + (int64_t)j * ld] /= nr;
          break;
        }
      }
    }
  }
  __syncthreads();
  for (int j = wave; j < nb; j += nw) {
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < nb; i += 64) {
      const double x = fabs(Vo[i + (int64_t)j * ld]);
      if (x > best) {
        best = x;
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (Vo[bi + (int64_t)j * ld] < 0.0) {
      for (int i = lane; i < nb; i += 64) {
        Vo[i + (int64_t)j * ld] = -Vo[i + (int64_t)j * ld];
        Uo[i + (int64_t)j * ld] = -Uo[i + (int64_t)j * ld];
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
    W[i + (int64_t)j * ld] = Ri[i + (int64_t)j * ld];
    V[i + (int64_t)j * ld] = i == j ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0)
    for (int s = threadIdx.x; s < max_sweeps; s += blockDim.x) rotcount[mi * max_sweeps + s] = 0;
}

__global__ __launch_bounds__(kRoundThreads) void k_bj_round(const int* __restrict__ nbs, int ld,
                                                  double* __restrict__ Wk, double* __restrict__ Vk,
                                                  int64_t strideUV, int* __restrict__ rotcount,
                                                  int max_sweeps, int sweep, int round) {
  extern __shared__ double sm[];
  __shared__ int srot;
  const int mi = blockIdx.y, pi = blockIdx.x;
  const int nb = nbs[mi];
  const int nblk = (nb + kBW - 1) / kBW;
  const int nblk2 = nblk + (nblk & 1);
  if (nb <= 1 || pi >= nblk2 / 2 || round >= nblk2 - 1) return;
  if (sweep > 0 && rotcount[mi * max_sweeps + sweep - 1] == 0) return;  // converged
  int bp, bq;
  rr_pair(nblk2, round, pi, &bp, &bq);
  const int ldl = nb | 1;
  double* sW = sm;
  double* sV = sm + 2 * kBW * ldl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* W = Wk + mi * strideUV;
  double* V = Vk + mi * strideUV;
  auto gcol = [&](int c) -> int {  // global column of local column c, or -1
    const int blk = c < kBW ? bp : bq;
    const int g = blk * kBW + (c % kBW);
    return (blk < nblk && g < nb) ? g : -1;
  };
  // Column c of the pair per wave, rows lane-strided (no index division).
  for (int c = wave; c < 2 * kBW; c += kRoundThreads / 64) {
    const int g = gcol(c);
    for (int i = lane; i < nb; i += 64) {
      sW[c * ldl + i] = g >= 0 ? W[i + (int64_t)g * ld] : 0.0;
      sV[c * ldl + i] = g >= 0 ? V[i + (int64_t)g * ld] : 0.0;
    }
  }
  const double tol = jacobi_tol(nb);
  if (tid == 0) srot = 0;
  __syncthreads();
  // Round 0 of a sweep also visits the pairs inside each block (every block
  // is in exactly one pair per round): round-robin over the kBW columns of
  // each of the two blocks.
  if (round == 0) {
    for (int r = 0; r < kBW - 1; ++r) {
      for (int k = wave; k < kBW; k += kRoundThreads / 64) {
        const int half = k / (kBW / 2), kk = k % (kBW / 2);
        int p, q;
        rr_pair(kBW, r, kk, &p, &q);
        p += half * kBW;
        q += half * kBW;
        if (gcol(p) < 0 || gcol(q) < 0) continue;
        if (rotate_pair(sW + p * ldl, sW + q * ldl, sV + p * ldl, sV + q * ldl, nb, lane, tol) &&
            lane == 0)
          srot = 1;
      }
      __syncthreads();
    }
  }
  // Cross pairs (p in block bp, q in block bq): kBW sub-rounds of kBW
  // disjoint pairs (k, kBW + (k + r) mod kBW).
  for (int r = 0; r < kBW; ++r) {
    for (int k = wave; k < kBW; k += kRoundThreads / 64) {
      const int p = k, q = kBW + (k + r) % kBW;
      if (gcol(p) < 0 || gcol(q) < 0) continue;
      if (rotate_pair(sW + p * ldl, sW + q * ldl, sV + p * ldl, sV + q * ldl, nb, lane, tol) &&
          lane == 0)
        srot = 1;
    }
    __syncthreads();
  }
  const bool any = srot != 0;
  for (int c = wave; c < 2 * kBW; c += kRoundThreads / 64) {
    const int g = gcol(c);
    if (g < 0) continue;
    for (int i = lane; i < nb; i += 64) {
      W[i + (int64_t)g * ld] = sW[c * ldl + i];
      V[i + (int64_t)g * ld] = sV[c * ldl + i];
    }
  }
  if (any && tid == 0) atomicAdd(&rotcount[mi * max_sweeps + sweep], 1);
}

__global__ __launch_bounds__(256) void k_bj_finish(const int* __restrict__ nbs, int ld,
                                                   const double* __restrict__ Wk,
                                                   const double* __restrict__ Vk,
                                                   int64_t strideUV, double* __restrict__ Us,
                                                   double* __restrict__ Vs,
                                                   double* __restrict__ D, int64_t strideD,
                                                   const int* __restrict__ rotcount,
                                                   int max_sweeps, int* __restrict__ status,
                                                   int* __restrict__ fail) {
  __shared__ double sig[kMaxLdsN];
  __shared__ int rank[kMaxLdsN];
  const int mi = blockIdx.x;
  const int nb = nbs[mi];
  if (nb > 0)
    finish_svd(nb, ld, Wk + mi * strideUV, Vk + mi * strideUV, Us + mi * strideUV,
               Vs + mi * strideUV, D + mi * strideD, sig, rank);
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

// ------------------------------------------------ single-workgroup fallback
__global__ __launch_bounds__(256) void k_jacobi(const int* __restrict__ nbs, int ld,
                                                const double* __restrict__ R, int64_t strideR,
                                                double* __restrict__ Us,
                                                double* __restrict__ Vs, int64_t strideUV,
                                                double* __restrict__ D, int64_t strideD,
                                                double* __restrict__ Wk, double* __restrict__ Vk,
                                                int* __restrict__ status, int max_sweeps,
                                                int* __restrict__ fail) {
  __shared__ double sig[MAXN];
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
    W[i + (int64_t)j * ld] = Ri[i + (int64_t)j * ld];
    V[i + (int64_t)j * ld] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  const int n2 = nb + (nb & 1);
  const double tol = jacobi_tol(nb);
  int sweeps = 0;
  bool conv = nb == 1;
  for (int sw = 0; sw < max_sweeps && !conv; ++sw) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < n2 - 1; ++r) {
      for (int k = wave; k < n2 / 2; k += 4) {
        int p, q;
        rr_pair(n2, r, k, &p, &q);
        if (p >= nb || q >= nb) continue;
        if (rotate_pair(W + (int64_t)p * ld, W + (int64_t)q * ld, V + (int64_t)p * ld,
                        V + (int64_t)q * ld, nb, lane, tol) &&
            lane == 0)
          rotated = 1;
      }
      __syncthreads();
    }
    ++sweeps;
    conv = rotated == 0;
    __syncthreads();
  }
  finish_svd(nb, ld, W, V, Us + mi * strideUV, Vs + mi * strideUV, D + mi * strideD, sig, rank);
  if (tid == 0) {
    status[mi] = conv ? sweeps : -1;
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
  static bool attr_set = false;
  const size_t shmem = (size_t)4 * kBW * (ld | 1) * sizeof(double);
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_bj_round, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)((size_t)4 * kBW * (kMaxLdsN | 1) * sizeof(double)));
    (void)hipGetLastError();
    attr_set = true;
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
  for (int sw = 0; sw < max_sweeps; ++sw)
    for (int r = 0; r < nblk2 - 1; ++r)
      hipLaunchKernelGGL(k_bj_round, dim3(nblk2 / 2, count), dim3(kRoundThreads), shmem, st,
                         nb_dev, ld, Wk, Vk, strideUV, rotcount, max_sweeps, sw, r);
  hipLaunchKernelGGL(k_bj_finish, dim3(count), dim3(256), 0, st, nb_dev, ld, Wk, Vk, strideUV, Us,
                     Vs, D, strideD, rotcount, max_sweeps, status, fail);
  prof_done(st, slot, PC_SVD, 0.0, 0.0);
  return hipGetLastError();
}

}  // namespace rutv
