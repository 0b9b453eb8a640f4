// Householder QR of a tall b-column panel (Section 2.4, eq. unpivQR) and its
// compact-WY factor (eq. WYrepresentation, written as I - V Tw V^T).
//
// randUTV factors two tall panels per step (the sampling matrix Y and the
// updated column block T([I2,I3],J2)); their flops are negligible but the
// b reflectors form a sequential chain, so the panel is latency-bound.
//
// Design: one cooperative launch.  Each of `nwg` workgroups owns a slab of
// consecutive rows.  Columns are taken in sub-panels of kPanelNB; the
// current sub-panel's slice of each slab lives in LDS.  For column c the
// only cross-slab quantities are the dot products of the column with itself
// and with the sub-panel's other columns plus the pivot row, so one
// reduction (one grid barrier) per column suffices: every workgroup then
// forms alpha, beta, tau and the rank-1 update of its rows redundantly and
// identically (fixed reduction order).  After a sub-panel, a second
// reduction forms Vs^T [V_prev | Vs | P_rest] (kPanelNB x b), which gives
// (a) the block-reflector update of the rest of the panel and (b) the
// off-diagonal block of Tw via Tw12 = -Tw11 (V_prev^T Vs) Ts, the
// recursive form of the compact-WY T factor, so no separate triangular
// inversion is needed.  Householder vectors follow LAPACK dlarfg: beta =
// -sign(alpha) ||x|| with sign(0) = +1, tau = (beta - alpha)/beta, tau = 0
// when the part below the diagonal is zero.
#include <algorithm>

#include "common.h"

namespace rutv {
namespace {

constexpr int PNB = kPanelNB;
constexpr int MAXB = 256;  // widest panel this kernel takes

struct PanelArgs {
  int Mp, nb, nwg, chunk;
  double* P;
  int64_t ldp;
  double* tau;
  double* Tw;
  int64_t ldtw;
  double* part;
  double* bcast;
  double* bpart;
  double* red;
  unsigned* bar;
  int* err;
};

__device__ inline void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ inline void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Grid-wide barrier over the nwg co-resident workgroups of a cooperative
// launch.  bar[0] counts arrivals, bar[1] is the generation.  Every wait is
// bounded: on timeout the error flag is raised and all later waits return
// at once, so the kernel always drains.
__device__ void grid_sync(unsigned* bar, unsigned nwg, int* err) {
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0 && nwg > 1) {
    const unsigned g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned a = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (a == nwg - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned it = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (++it > kSpinLimit) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  __syncthreads();
  fence_acquire();
}

// Sum over the 16 lanes of an aligned 16-lane group.
__device__ inline double sum16(double v) {
  v += __shfl_xor(v, 8, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 1, 16);
  return v;
}

__global__ __launch_bounds__(256) void k_panel(PanelArgs a) {
  __shared__ double S[PNB][kPanelMaxRows];  // sub-panel slice of my rows
  __shared__ double sred[PNB][MAXB];        // reduced Vs^T [V_prev | Vs | P_rest]
  __shared__ double sZ[MAXB][PNB];          // (V_prev^T Vs) Ts
  __shared__ double sTs[PNB][PNB];
  __shared__ double sg[PNB], srow[PNB], sw[PNB], stau[MAXB];
  __shared__ double shh[3];  // beta, tau, scale of the current column

  const int tid = threadIdx.x;
  const int w = blockIdx.x;
  const int nwg = a.nwg, nb = a.nb, Mp = a.Mp;
  const int rb = w * a.chunk;
  const int re = min(Mp, rb + a.chunk);
  const int nrows = max(0, re - rb);
  const int64_t ldp = a.ldp;
  double* P = a.P;
  int colstep = 0;

  for (int c0 = 0; c0 < nb; c0 += PNB) {
    const int pw = min(PNB, nb - c0);
    // Load the sub-panel slice of my rows.
    for (int idx = tid; idx < pw * nrows; idx += 256) {
      const int t = idx / nrows, rl = idx % nrows;
      S[t][rl] = P[rb + rl + (int64_t)(c0 + t) * ldp];
    }
    __syncthreads();

    for (int cc = 0; cc < pw; ++cc, ++colstep) {
      const int c = c0 + cc;
      const int buf = colstep & 1;
      double* part = a.part + buf * (kPanelMaxWG * PNB);
      double* bcast = a.bcast + buf * PNB;
      // Partial dot products of column c with columns j >= c of the
      // sub-panel over my rows strictly below row c.
      {
        const int j = tid >> 4, li = tid & 15;
        double s = 0.0;
        if (j >= cc && j < pw) {
          for (int rl = li; rl < nrows; rl += 16)
            if (rb + rl > c) s += S[cc][rl] * S[j][rl];
        }
        s = sum16(s);
        if (li == 0 && j >= cc && j < pw) part[w * PNB + j] = s;
        if (c >= rb && c < re && tid < pw) bcast[tid] = S[tid][c - rb];
      }
      grid_sync(a.bar, nwg, a.err);
      {
        const int j = tid >> 4, li = tid & 15;
        double s = 0.0;
        if (j >= cc && j < pw)
          for (int v = li; v < nwg; v += 16) s += part[v * PNB + j];
        s = sum16(s);
        if (li == 0 && j >= cc && j < pw) sg[j] = s;
        if (tid < pw) srow[tid] = bcast[tid];
      }
      __syncthreads();
      if (tid == 0) {
        const double alpha = srow[cc], xn2 = sg[cc];
        double beta, tau, scale;
        if (xn2 == 0.0) {
          beta = alpha;
          tau = 0.0;
          scale = 0.0;
        } else {
          const double nrm = sqrt(alpha * alpha + xn2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        shh[0] = beta;
        shh[1] = tau;
        shh[2] = scale;
        stau[c] = tau;
        if (w == 0) a.tau[c] = tau;
      }
      __syncthreads();
      if (tid < pw && tid > cc) {
        // w_j = tau * v^T p_j with v = (1, x2 * scale).
        sw[tid] = shh[1] * (srow[tid] + shh[2] * sg[tid]);
      }
      __syncthreads();
      {
        const double beta = shh[0], scale = shh[2];
        for (int rl = tid; rl < nrows; rl += 256) {
          const int r = rb + rl;
          if (r > c) {
            const double x = S[cc][rl];
            const double v = x * scale;
            for (int jj = cc + 1; jj < pw; ++jj) S[jj][rl] -= v * sw[jj];
            S[cc][rl] = v;
          } else if (r == c) {
            for (int jj = cc + 1; jj < pw; ++jj) S[jj][rl] -= sw[jj];
            S[cc][rl] = beta;
          }
        }
      }
      __syncthreads();
    }
    // Write the factored sub-panel back.
    for (int idx = tid; idx < pw * nrows; idx += 256) {
      const int t = idx / nrows, rl = idx % nrows;
      P[rb + rl + (int64_t)(c0 + t) * ldp] = S[t][rl];
    }
    // Vs(r, t): explicit unit-lower trapezoidal sub-panel reflectors.
    auto vs = [&](int rl, int t) -> double {
      const int r = rb + rl, d = c0 + t;
      return r > d ? S[t][rl] : (r == d ? 1.0 : 0.0);
    };
    // Partial products Vs^T [V_prev | Vs | P_rest] over my rows (rows < c0
    // contribute nothing since Vs is zero there).
    {
      double* bp = a.bpart + (int64_t)w * PNB * nb;
      for (int j = tid; j < nb; j += 256) {
        double acc[PNB];
#pragma unroll
        for (int t = 0; t < PNB; ++t) acc[t] = 0.0;
        for (int rl = max(0, c0 - rb); rl < nrows; ++rl) {
          const int r = rb + rl;
          double rop;
          if (j < c0) rop = P[r + (int64_t)j * ldp];  // r >= c0 > j: stored tail
          else if (j < c0 + pw) rop = vs(rl, j - c0);
          else rop = P[r + (int64_t)j * ldp];
#pragma unroll
          for (int t = 0; t < PNB; ++t)
            if (t < pw) acc[t] += vs(rl, t) * rop;
        }
#pragma unroll
        for (int t = 0; t < PNB; ++t)
          if (t < pw) bp[t * nb + j] = acc[t];
      }
    }
    grid_sync(a.bar, nwg, a.err);
    {
      const int E = pw * nb;
      const int e0 = (int)((int64_t)w * E / nwg), e1 = (int)((int64_t)(w + 1) * E / nwg);
      for (int e = e0 + tid; e < e1; e += 256) {
        const int t = e / nb, j = e % nb;
        double s = 0.0;
        for (int v = 0; v < nwg; ++v) s += a.bpart[(int64_t)v * PNB * nb + t * nb + j];
        a.red[t * nb + j] = s;
      }
    }
    grid_sync(a.bar, nwg, a.err);
    for (int e = tid; e < pw * nb; e += 256) sred[e / nb][e % nb] = a.red[e];
    __syncthreads();
    // Ts: compact-WY factor of the sub-panel (column recurrence
    // Ts(0:t,t) = -tau_t Ts(0:t,0:t) Gram(0:t,t), Ts(t,t) = tau_t).
    for (int t = 0; t < pw; ++t) {
      if (tid < t) {
        double s = 0.0;
        for (int k = tid; k < t; ++k) s += sTs[tid][k] * sred[k][c0 + t];
        sTs[tid][t] = -stau[c0 + t] * s;
      } else if (tid < PNB) {
        sTs[tid][t] = tid == t ? stau[c0 + t] : 0.0;
      }
      __syncthreads();
    }
    // Z = (V_prev^T Vs) Ts : c0 x pw.
    for (int e = tid; e < c0 * pw; e += 256) {
      const int k = e / pw, t = e % pw;
      double s = 0.0;
      for (int tp = 0; tp <= t; ++tp) s += sred[tp][k] * sTs[tp][t];
      sZ[k][t] = s;
    }
    __syncthreads();
    // Tw blocks: diagonal block (workgroup 0), zero rows c0.. of earlier
    // columns (workgroup 0), and off-diagonal rows split over workgroups:
    // Tw(i, c0+t) = -sum_{k=i}^{c0-1} Tw(i,k) Z(k,t).
    if (w == 0) {
      for (int e = tid; e < pw * PNB; e += 256) {
        const int i = e / PNB, t = e % PNB;
        if (t < pw) a.Tw[(c0 + i) + (int64_t)(c0 + t) * a.ldtw] = sTs[i][t];
      }
      for (int e = tid; e < pw * c0; e += 256) {
        const int i = e % pw, j = e / pw;
        a.Tw[(c0 + i) + (int64_t)j * a.ldtw] = 0.0;
      }
    }
    for (int e = tid; e < c0 * pw; e += 256) {
      const int i = e / pw, t = e % pw;
      if (i % nwg != w) continue;
      double s = 0.0;
      for (int k = i; k < c0; ++k) s += a.Tw[i + (int64_t)k * a.ldtw] * sZ[k][t];
      a.Tw[i + (int64_t)(c0 + t) * a.ldtw] = -s;
    }
    // Block-reflector update of the rest of the panel on my rows:
    // P_rest -= Vs (Ts^T W), W = Vs^T P_rest.
    const int jr0 = c0 + pw;
    for (int j = jr0 + tid; j < nb; j += 256) {
      double wp[PNB];
#pragma unroll
      for (int t = 0; t < PNB; ++t) {
        double s = 0.0;
        for (int tp = 0; tp <= t && tp < pw; ++tp) s += sTs[tp][t] * sred[tp][j];
        wp[t] = t < pw ? s : 0.0;
      }
      for (int rl = max(0, c0 - rb); rl < nrows; ++rl) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < PNB; ++t)
          if (t < pw) s += vs(rl, t) * wp[t];
        P[rb + rl + (int64_t)j * ldp] -= s;
      }
    }
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// LDS-resident variant (used whenever the slabs fit): each workgroup keeps
// its whole row slab of the panel (all nb columns) in LDS for the entire
// factorization, so the only global traffic is the initial load, the final
// write-back and the small cross-slab reduction partials, which are written
// and read with device-coherent (agent-scope) accesses.
struct PanelArgs2 {
  int Mp, nb, nwg, chunk, ldS;
  double* P;
  int64_t ldp;
  double* tau;
  double* Tw;
  int64_t ldtw;
  double* part;
  double* bcast;
  double* bpart;
  double* red;
  unsigned* bar;
  int* err;
};

__device__ inline void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier whose agent-scope release/acquire fences are issued by one
// wave only (the workgroup barriers order the other waves around it).
__device__ void grid_sync_lean(unsigned* bar, unsigned nwg, int* err) {
  __syncthreads();
  if (threadIdx.x == 0 && nwg > 1) {
    fence_release();
    const unsigned g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned a = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a == nwg - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned it = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (++it > kSpinLimit) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    fence_acquire();
  }
  __syncthreads();
}

constexpr int kFixedLdsDoubles(int nb) { return PNB * nb + PNB * PNB + 2 * nb + 3 * PNB + 8; }

__global__ __launch_bounds__(256) void k_panel_lds(PanelArgs2 a) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int w = blockIdx.x;
  const int nwg = a.nwg, nb = a.nb, Mp = a.Mp, ldS = a.ldS;
  const int rb = w * a.chunk;
  const int re = min(Mp, rb + a.chunk);
  const int nrows = max(0, re - rb);
  double* S = smem;                        // column j of my slab at S + j*ldS
  double* sred = S + (size_t)nb * ldS;     // [t*nb + j]
  double* sTs = sred + PNB * nb;           // [i*PNB + t]
  double* stau = sTs + PNB * PNB;          // [nb]
  double* srowTw = stau + nb;              // [nb]
  double* sg = srowTw + nb;
  double* srow = sg + PNB;
  double* sw = srow + PNB;
  double* shh = sw + PNB;
  const int64_t ldp = a.ldp;

  for (int idx = tid; idx < nb * nrows; idx += 256) {
    const int j = idx / nrows, rl = idx % nrows;
    S[j * ldS + rl] = a.P[rb + rl + (int64_t)j * ldp];
  }
  __syncthreads();
  int colstep = 0;
  for (int c0 = 0; c0 < nb; c0 += PNB) {
    const int pw = min(PNB, nb - c0);
    for (int cc = 0; cc < pw; ++cc, ++colstep) {
      const int c = c0 + cc;
      const int buf = colstep & 1;
      double* part = a.part + buf * (kPanelMaxWG * PNB);
      double* bcast = a.bcast + buf * PNB;
      const double* xc = S + c * ldS;
      {
        const int j = tid >> 4, li = tid & 15;
        double s = 0.0;
        if (j >= cc && j < pw) {
          const double* pj = S + (c0 + j) * ldS;
          for (int rl = li; rl < nrows; rl += 16)
            if (rb + rl > c) s += xc[rl] * pj[rl];
        }
        s = sum16(s);
        if (li == 0 && j >= cc && j < pw) st_coh(&part[w * PNB + j], s);
        if (c >= rb && c < re && tid < pw) st_coh(&bcast[tid], S[(c0 + tid) * ldS + (c - rb)]);
      }
      grid_sync_lean(a.bar, nwg, a.err);
      {
        const int j = tid >> 4, li = tid & 15;
        double s = 0.0;
        if (j >= cc && j < pw)
          for (int v = li; v < nwg; v += 16) s += ld_coh(&part[v * PNB + j]);
        s = sum16(s);
        if (li == 0 && j >= cc && j < pw) sg[j] = s;
        if (tid < pw) srow[tid] = ld_coh(&bcast[tid]);
      }
      __syncthreads();
      if (tid == 0) {
        const double alpha = srow[cc], xn2 = sg[cc];
        double beta, tau, scale;
        if (xn2 == 0.0) {
          beta = alpha;
          tau = 0.0;
          scale = 0.0;
        } else {
          const double nrm = sqrt(alpha * alpha + xn2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        shh[0] = beta;
        shh[1] = tau;
        shh[2] = scale;
        stau[c] = tau;
        if (w == 0) a.tau[c] = tau;
      }
      __syncthreads();
      if (tid < pw && tid > cc) sw[tid] = shh[1] * (srow[tid] + shh[2] * sg[tid]);
      __syncthreads();
      {
        const double beta = shh[0], scale = shh[2];
        double* xw = S + c * ldS;
        for (int rl = tid; rl < nrows; rl += 256) {
          const int r = rb + rl;
          if (r > c) {
            const double v = xw[rl] * scale;
            for (int jj = cc + 1; jj < pw; ++jj) S[(c0 + jj) * ldS + rl] -= v * sw[jj];
            xw[rl] = v;
          } else if (r == c) {
            for (int jj = cc + 1; jj < pw; ++jj) S[(c0 + jj) * ldS + rl] -= sw[jj];
            xw[rl] = beta;
          }
        }
      }
      __syncthreads();
    }
    auto vs = [&](int rl, int t) -> double {
      const int r = rb + rl, d = c0 + t;
      return r > d ? S[d * ldS + rl] : (r == d ? 1.0 : 0.0);
    };
    const int rl0 = max(0, c0 - rb);
    // Partial products Vs^T [V_prev | Vs | P_rest] over my rows.
    for (int j = tid; j < nb; j += 256) {
      double acc[PNB];
#pragma unroll
      for (int t = 0; t < PNB; ++t) acc[t] = 0.0;
      for (int rl = rl0; rl < nrows; ++rl) {
        const double rop = (j >= c0 && j < c0 + pw) ? vs(rl, j - c0) : S[j * ldS + rl];
#pragma unroll
        for (int t = 0; t < PNB; ++t)
          if (t < pw) acc[t] += vs(rl, t) * rop;
      }
#pragma unroll
      for (int t = 0; t < PNB; ++t)
        if (t < pw) st_coh(&a.bpart[((int64_t)w * PNB + t) * nb + j], acc[t]);
    }
    grid_sync_lean(a.bar, nwg, a.err);
    {
      const int E = pw * nb;
      const int e0 = (int)((int64_t)w * E / nwg), e1 = (int)((int64_t)(w + 1) * E / nwg);
      for (int e = e0 + tid; e < e1; e += 256) {
        const int t = e / nb, j = e % nb;
        double s = 0.0;
        for (int v = 0; v < nwg; ++v) s += ld_coh(&a.bpart[((int64_t)v * PNB + t) * nb + j]);
        st_coh(&a.red[e], s);
      }
    }
    grid_sync_lean(a.bar, nwg, a.err);
    for (int e = tid; e < pw * nb; e += 256) sred[e] = ld_coh(&a.red[e]);
    __syncthreads();
    for (int t = 0; t < pw; ++t) {
      if (tid < t) {
        double s = 0.0;
        for (int k = tid; k < t; ++k) s += sTs[tid * PNB + k] * sred[k * nb + c0 + t];
        sTs[tid * PNB + t] = -stau[c0 + t] * s;
      } else if (tid < PNB) {
        sTs[tid * PNB + t] = tid == t ? stau[c0 + t] : 0.0;
      }
      __syncthreads();
    }
    // Z(k,t) = sum_tp (V_prev^T Vs)(k,tp) Ts(tp,t), in place over sred[., k<c0].
    for (int k = tid; k < c0; k += 256) {
      double mk[PNB];
#pragma unroll
      for (int t = 0; t < PNB; ++t) mk[t] = t < pw ? sred[t * nb + k] : 0.0;
#pragma unroll
      for (int t = 0; t < PNB; ++t) {
        if (t >= pw) continue;
        double z = 0.0;
        for (int tp = 0; tp <= t; ++tp) z += mk[tp] * sTs[tp * PNB + t];
        sred[t * nb + k] = z;
      }
    }
    __syncthreads();
    if (w == 0) {
      for (int e = tid; e < pw * pw; e += 256) {
        const int i = e / pw, t = e % pw;
        st_coh(&a.Tw[(c0 + i) + (int64_t)(c0 + t) * a.ldtw], sTs[i * PNB + t]);
      }
      for (int e = tid; e < pw * c0; e += 256) {
        const int i = e % pw, j = e / pw;
        st_coh(&a.Tw[(c0 + i) + (int64_t)j * a.ldtw], 0.0);
      }
    }
    // Tw(i, c0+t) = -sum_{k=i}^{c0-1} Tw(i,k) Z(k,t), rows i = w, w+nwg, ...
    for (int i = w; i < c0; i += nwg) {
      for (int k = i + tid; k < c0; k += 256) srowTw[k] = ld_coh(&a.Tw[i + (int64_t)k * a.ldtw]);
      __syncthreads();
      if (tid < pw) {
        double s = 0.0;
        for (int k = i; k < c0; ++k) s += srowTw[k] * sred[tid * nb + k];
        st_coh(&a.Tw[i + (int64_t)(c0 + tid) * a.ldtw], -s);
      }
      __syncthreads();
    }
    // P_rest -= Vs (Ts^T W) on my rows, in LDS.
    for (int j = c0 + pw + tid; j < nb; j += 256) {
      double wp[PNB];
#pragma unroll
      for (int t = 0; t < PNB; ++t) {
        double s = 0.0;
        if (t < pw)
          for (int tp = 0; tp <= t; ++tp) s += sTs[tp * PNB + t] * sred[tp * nb + j];
        wp[t] = s;
      }
      double* pj = S + j * ldS;
      for (int rl = rl0; rl < nrows; ++rl) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < PNB; ++t)
          if (t < pw) s += vs(rl, t) * wp[t];
        pj[rl] -= s;
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nrows; idx += 256) {
    const int j = idx / nrows, rl = idx % nrows;
    a.P[rb + rl + (int64_t)j * ldp] = S[j * ldS + rl];
  }
}

__global__ void k_init_sync(unsigned* bar) {
  if (threadIdx.x == 0) {
    bar[0] = 0u;
    bar[1] = 0u;
  }
}

__global__ void k_extract(int Mp, int nb, const double* __restrict__ P, int64_t ldp,
                          double* __restrict__ V, int64_t ldv, double* __restrict__ R,
                          int64_t ldr) {
  const int64_t total = (int64_t)Mp * nb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % Mp);
    const int j = (int)(idx / Mp);
    const double p = P[i + (int64_t)j * ldp];
    V[i + (int64_t)j * ldv] = i > j ? p : (i == j ? 1.0 : 0.0);
    if (R && i < nb) R[i + (int64_t)j * ldr] = i <= j ? p : 0.0;
  }
}

}  // namespace

size_t panel_work_bytes(int bmax) {
  size_t d = 2 * kPanelMaxWG * PNB + 2 * PNB + (size_t)kPanelMaxWG * PNB * bmax + PNB * bmax;
  return d * sizeof(double) + 256;
}

void panel_work_carve(void* base, int bmax, PanelWork* w) {
  double* p = (double*)base;
  w->part = p;
  p += 2 * kPanelMaxWG * PNB;
  w->bcast = p;
  p += 2 * PNB;
  w->bpart = p;
  p += (size_t)kPanelMaxWG * PNB * bmax;
  w->red = p;
  p += PNB * bmax;
  w->bar = (unsigned*)p;
  w->err = (int*)(w->bar + 2);
}

hipError_t panel_qr(hipStream_t st, int Mp, int nb, double* P, int64_t ldp, double* tau,
                    double* Tw, int64_t ldtw, const PanelWork& w) {
  if (nb <= 0) return hipSuccess;
  if (nb > MAXB || Mp < nb) return hipErrorInvalidValue;
  static int cu_count = 0;
  static int kLdsBytes = 0;
  static bool attr_set = false;
  if (!cu_count) {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu_count, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cu_count = 1;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lds = 64 * 1024;
    kLdsBytes = std::min(lds, 160 * 1024);
    if (hipFuncSetAttribute((const void*)k_panel_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kLdsBytes) == hipSuccess)
      attr_set = true;
    (void)hipGetLastError();
  }
  // LDS-resident variant: slab of `chunk` rows x nb columns per workgroup.
  const int fixed = kFixedLdsDoubles(nb);
  const int max_ld = (kLdsBytes / 8 - fixed) / nb;
  const int chunk_max = std::min(kPanelMaxRows, max_ld - 1);
  if (attr_set && chunk_max >= 1) {
    int nwg = (Mp + chunk_max - 1) / chunk_max;
    if (nwg <= std::min(cu_count, kPanelMaxWG)) {
      const int chunk = (Mp + nwg - 1) / nwg;
      nwg = (Mp + chunk - 1) / chunk;
      const int ldS = chunk | 1;
      const size_t shmem = ((size_t)nb * ldS + fixed) * sizeof(double);
      hipLaunchKernelGGL(k_init_sync, dim3(1), dim3(64), 0, st, w.bar);
      PanelArgs2 a{Mp, nb, nwg, chunk, ldS, P, ldp, tau, Tw, ldtw, w.part, w.bcast, w.bpart,
                   w.red, w.bar, w.err};
      void* args[] = {&a};
      const int slot = prof_mark(st);
      hipError_t e = hipLaunchCooperativeKernel((const void*)k_panel_lds, dim3(nwg), dim3(256),
                                                args, (unsigned)shmem, st);
      prof_done(st, slot, PC_PANEL, 2.0 * Mp * (double)nb * nb);
      return e;
    }
  }
  // Global-memory variant for slabs that do not fit in LDS.
  int nwg = (Mp + 63) / 64;
  nwg = std::max(1, std::min(nwg, kPanelMaxWGGlobal));
  int chunk = (Mp + nwg - 1) / nwg;
  if (chunk > kPanelMaxRows) return hipErrorInvalidValue;
  nwg = (Mp + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_init_sync, dim3(1), dim3(64), 0, st, w.bar);
  PanelArgs a{Mp, nb, nwg, chunk, P, ldp, tau, Tw, ldtw, w.part, w.bcast, w.bpart, w.red,
              w.bar, w.err};
  void* args[] = {&a};
  const int slot = prof_mark(st);
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_panel, dim3(nwg), dim3(256), args, 0, st);
  prof_done(st, slot, PC_PANEL, 2.0 * Mp * (double)nb * nb);
  return e;
}

hipError_t panel_extract(hipStream_t st, int Mp, int nb, const double* P, int64_t ldp,
                         double* V, int64_t ldv, double* Rout, int64_t ldr) {
  const int64_t total = (int64_t)Mp * nb;
  if (total == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_extract, dim3(blocks), dim3(256), 0, st, Mp, nb, P, ldp, V, ldv, Rout,
                     ldr);
  return hipGetLastError();
}

}  // namespace rutv
