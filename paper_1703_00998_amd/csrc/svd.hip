// SVD of the small diagonal blocks (Figure "The algorithm randUTV":
// [Us, Ds, Vs] = svd(R(1:b,1:b)); Section 2.4 eq. smallSVD).
//
// One-sided (Hestenes) Jacobi: columns of W = R are rotated pairwise until
// mutually orthogonal, accumulating the rotations in V; then sigma_j =
// ||w_j||, u_j = w_j / sigma_j.  One workgroup per matrix; each wave takes
// column pairs of a round-robin tournament round (all pairs of a round are
// disjoint, so waves never touch the same column within a round).  The
// SVDs of all steps are independent, so they run batched, one workgroup per
// step.  Output conventions: sigma descending (ties by index), and each
// (u_j, v_j) flipped so the largest-magnitude entry of v_j is positive
// (first index on ties); columns of Us with sigma_j == 0 are completed by
// Gram-Schmidt on e_1, e_2, ...
#include <algorithm>

#include "common.h"

namespace rutv {
namespace {

constexpr int MAXN = 1024;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_jacobi(const int* __restrict__ nbs, int ld,
                                                const double* __restrict__ R, int64_t strideR,
                                                double* __restrict__ Us,
                                                double* __restrict__ Vs, int64_t strideUV,
                                                double* __restrict__ D, int64_t strideD,
                                                double* __restrict__ Wk, double* __restrict__ Vk,
                                                int* __restrict__ status, int max_sweeps) {
  __shared__ double sig[MAXN];
  __shared__ int rank[MAXN];
  __shared__ int rotated;
  const int mi = blockIdx.x;
  const int nb = nbs[mi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* Ri = R + mi * strideR;
  double* W = Wk + mi * strideUV;
  double* V = Vk + mi * strideUV;
  double* Uo = Us + mi * strideUV;
  double* Vo = Vs + mi * strideUV;
  double* Do = D + mi * strideD;
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
  const double tol = 4.0 * 2.220446049250313e-16 * sqrt((double)nb);
  int sweeps = 0;
  bool conv = nb == 1;
  for (int sw = 0; sw < max_sweeps && !conv; ++sw) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < n2 - 1; ++r) {
      for (int k = wave; k < n2 / 2; k += 4) {
        int p, q;
        if (k == 0) { p = r; q = n2 - 1; }
        else { p = (r + k) % (n2 - 1); q = (r - k + n2 - 1) % (n2 - 1); }
        if (p >= nb || q >= nb) continue;
        double* wp = W + (int64_t)p * ld;
        double* wq = W + (int64_t)q * ld;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < nb; i += 64) {
          const double x = wp[i], y = wq[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga == 0.0 || al == 0.0 || be == 0.0) continue;
        if (fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
        const double zeta = (be - al) / (2.0 * ga);
        double t;
        if (fabs(zeta) > 1e150) t = 0.5 / zeta;
        else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = lane; i < nb; i += 64) {
          const double x = wp[i], y = wq[i];
          wp[i] = c * x - s * y;
          wq[i] = s * x + c * y;
        }
        double* vp = V + (int64_t)p * ld;
        double* vq = V + (int64_t)q * ld;
        for (int i = lane; i < nb; i += 64) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    ++sweeps;
    conv = rotated == 0;
    __syncthreads();
  }
  // sigma_j = ||w_j||
  for (int j = wave; j < nb; j += 4) {
    double s = 0.0;
    for (int i = lane; i < nb; i += 64) {
      const double x = W[i + (int64_t)j * ld];
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) sig[j] = sqrt(s);
  }
  __syncthreads();
  for (int j = tid; j < nb; j += 256) {
    int rk = 0;
    const double sj = sig[j];
    for (int k = 0; k < nb; ++k) rk += (sig[k] > sj) || (sig[k] == sj && k < j);
    rank[j] = rk;
  }
  __syncthreads();
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int i = idx % nb, j = idx / nb;
    const int o = rank[j];
    const double sj = sig[j];
    Vo[i + (int64_t)o * ld] = V[i + (int64_t)j * ld];
    Uo[i + (int64_t)o * ld] = sj > 0.0 ? W[i + (int64_t)j * ld] / sj : 0.0;
    if (i == 0) Do[o] = sj;
  }
  __syncthreads();
  // Complete columns of Us with zero singular value (they sit last).
  if (wave == 0) {
    for (int j = 0; j < nb; ++j) {
      if (Do[j] > 0.0) continue;
      for (int e = 0; e < nb; ++e) {
        // u = e_e minus its projection on columns 0..j-1, twice.
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
  // Canonical signs: largest |v_j| entry positive (first index on ties).
  for (int j = wave; j < nb; j += 4) {
    double best = -1.0;
    int bi = 0;
    for (int i = lane; i < nb; i += 64) {
      const double x = fabs(Vo[i + (int64_t)j * ld]);
      if (x > best) { best = x; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const bool flip = Vo[bi + (int64_t)j * ld] < 0.0;
    if (flip) {
      for (int i = lane; i < nb; i += 64) {
        Vo[i + (int64_t)j * ld] = -Vo[i + (int64_t)j * ld];
        Uo[i + (int64_t)j * ld] = -Uo[i + (int64_t)j * ld];
      }
    }
  }
  if (tid == 0) status[mi] = conv ? sweeps : -1;
}

}  // namespace

hipError_t batched_svd(hipStream_t st, int count, const int* nb_dev, int ld, const double* R,
                       int64_t strideR, double* Us, double* Vs, int64_t strideUV, double* D,
                       int64_t strideD, double* Wk, double* Vk, int* status, int max_sweeps) {
  if (count <= 0) return hipSuccess;
  if (ld > MAXN) return hipErrorInvalidValue;
  const int slot = prof_mark(st);
  hipLaunchKernelGGL(k_jacobi, dim3(count), dim3(256), 0, st, nb_dev, ld, R, strideR, Us, Vs,
                     strideUV, D, strideD, Wk, Vk, status, max_sweeps);
  prof_done(st, slot, PC_SVD, 0.0);
  return hipGetLastError();
}

}  // namespace rutv
