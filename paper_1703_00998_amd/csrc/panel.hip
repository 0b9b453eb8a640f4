// Householder QR of a tall b-column panel (Section 2.4, eq. unpivQR) and its
// compact-WY factor (eq. WYrepresentation, written as I - V Tw V^T).
//
// randUTV factors two tall panels per step (the sampling matrix Y and the
// updated column block T([I2,I3],J2)); their flops are negligible but the
// b reflectors form a sequential chain, so the panel is latency-bound.
// The factorization normally takes the CholeskyQR2 + Householder
// reconstruction path (panel_hr.hip); the kernels here are its fallback
// for panels that path declines, launched gated on its device flag.
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
  const int* gate;  // run only if NULL or *gate != 0 (read uniformly by every thread)
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
  if (a.gate && *a.gate == 0) return;  // uniform over the grid: no barrier is entered
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
  int Mp, nb, nwg, chunk, ldS, use_hr;
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
  const int* gate;
  double* gram;  // 2 * kPanelMaxWG * 256 Gram partials
  double* qtop;  // kPanelNB^2 published top rows of Q
};

__device__ inline void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier for the LDS-resident kernel.  Data exchanged across its
// workgroups is written and read with device-coherent (agent-scope atomic)
// accesses; the barrier itself is the release / acquire one above (an
// agent-scope release fence in every thread before arriving, the arrival as
// an acquire-release atomic, the generation published with release, and an
// agent-scope acquire fence in every thread after it is observed), so the
// exchange is ordered by the HIP memory model rather than by waiting for
// store acknowledgements.  Bounded like grid_sync.
__device__ inline void grid_sync_coh(unsigned* bar, unsigned nwg, int* err) {
  grid_sync(bar, nwg, err);
}

// LDS besides the slab: sred, sTs, stau, srowTw, sg/srow/sw/shh, the
// sub-panel copy (PNB columns of the slab stride, counted in the slab) and
// six PNB x PNB matrices + signs + flags of the CholeskyQR2 path.
constexpr int kFixedLdsDoubles(int nb) {
  return PNB * nb + PNB * PNB + 2 * nb + 3 * PNB + 8 + 6 * PNB * PNB + PNB + 8;
}


// ---- CholeskyQR2 + Householder reconstruction of one sub-panel ----------
__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Order LDS accesses among the lanes of one wave (no workgroup barrier).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The Gram matrix X^T X of the sub-panel's active rows (>= c0), summed over
// all workgroups in a fixed order.  One grid barrier.  Result in sG (full).
__device__ void gram_reduce(const double* S, int c0, int ldS, int rl0, int nrows, int pw,
                            double* gpart, int w, int nwg, double* sG, unsigned* bar, int* err) {
  const int tid = threadIdx.x;
  const int i = tid >> 4, j = tid & 15;
  const bool act = i < pw && j < pw && i <= j;
  double s = 0.0;
  if (act) {
    const double* xi = S + (c0 + i) * ldS;
    const double* xj = S + (c0 + j) * ldS;
    for (int rl = rl0; rl < nrows; ++rl) s += xi[rl] * xj[rl];
  }
  st_coh(&gpart[w * 256 + tid], s);
  grid_sync_coh(bar, nwg, err);
  double tot = 0.0;
  if (act) {
    for (int v0 = 0; v0 < nwg; v0 += 32) {
      double vals[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) vals[k] = v0 + k < nwg ? ld_coh(&gpart[(v0 + k) * 256 + tid]) : 0.0;
#pragma unroll
      for (int k = 0; k < 32; ++k) tot += vals[k];
    }
    sG[i * PNB + j] = tot;
    sG[j * PNB + i] = tot;
  }
  __syncthreads();
}

// Upper Cholesky factor R (R^T R = G), pw x pw, computed by one wave.
// Returns false when a pivot falls below rel * max diag(G) (same value in
// every lane).
__device__ bool chol_wave(const double* sG, double* sR, int pw, double rel) {
  const int lane = threadIdx.x & 63;
  double gmax = 0.0;
  for (int k = 0; k < pw; ++k) gmax = fmax(gmax, sG[k * PNB + k]);
  const double thr = rel * gmax;
  bool ok = true;
  for (int k = 0; k < pw; ++k) {
    double d = sG[k * PNB + k];
    for (int m = 0; m < k; ++m) d -= sR[m * PNB + k] * sR[m * PNB + k];
    ok = ok && (d > thr);
    const double rkk = sqrt(d > thr ? d : 1.0);
    if (lane < pw) {
      double v = 0.0;
      if (lane > k) {
        v = sG[k * PNB + lane];
        for (int m = 0; m < k; ++m) v -= sR[m * PNB + k] * sR[m * PNB + lane];
        v /= rkk;
      } else if (lane == k) {
        v = rkk;
      }
      sR[k * PNB + lane] = v;
    }
    wave_sync();
  }
  return ok;
}

// In place X <- X R^{-1} on rows [r0, r1) of the sub-panel columns (one
// thread per row; R upper triangular pw x pw).
__device__ void rsolve_rows(double* S, int c0, int ldS, int r0, int r1, int pw, const double* sR) {
  for (int rl = r0 + threadIdx.x; rl < r1; rl += blockDim.x) {
    double x[PNB];
#pragma unroll
    for (int jc = 0; jc < PNB; ++jc) {
      if (jc >= pw) break;
      double v = S[(c0 + jc) * ldS + rl];
      for (int i = 0; i < jc; ++i) v -= x[i] * sR[i * PNB + jc];
      x[jc] = v / sR[jc * PNB + jc];
    }
#pragma unroll
    for (int jc = 0; jc < PNB; ++jc) {
      if (jc >= pw) break;
      S[(c0 + jc) * ldS + rl] = x[jc];
    }
  }
}

struct HrBufs {
  double *sP0, *sG, *sR1, *sR2, *sQt, *sLU, *ssgn;
  int* sflag;
};

// Factor the sub-panel columns c0..c0+pw-1 (active rows >= c0) by
// CholeskyQR2, then rebuild its Householder vectors, tau and R from Q by the
// LU of Q - S (S = diag(s), s_k = -sign of the running pivot, which is the
// dlarfg choice), so the result matches column-by-column Householder QR in
// exact arithmetic.  Two grid barriers; the 16 x 16 factorizations run in
// wave 0.  Returns false, with the sub-panel untouched, when the sub-panel is
// too ill-conditioned for CholeskyQR2 or a column has an exactly zero tail
// (dlarfg's tau = 0 case).
__device__ bool subpanel_cholqr_hr(double* S, int c0, int pw, int ldS, int rb, int nrows,
                                   int w, int nwg, const PanelArgs2& a, const HrBufs& hb,
                                   double* stau) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rl0 = max(0, c0 - rb);
  for (int idx = tid; idx < pw * nrows; idx += 256) {
    const int i = idx / nrows, rl = idx % nrows;
    hb.sP0[i * ldS + rl] = S[(c0 + i) * ldS + rl];
  }
  gram_reduce(S, c0, ldS, rl0, nrows, pw, a.gram, w, nwg, hb.sG, a.bar, a.err);
  if (wave == 0) {
    const bool ok1 = chol_wave(hb.sG, hb.sR1, pw, 1e-13);
    if (lane == 0) hb.sflag[0] = ok1;
  }
  __syncthreads();
  if (!hb.sflag[0]) return false;
  rsolve_rows(S, c0, ldS, rl0, nrows, pw, hb.sR1);
  __syncthreads();
  // Publish Q1's rows c0..c0+pw-1 (those I own).
  for (int idx = tid; idx < pw * pw; idx += 256) {
    const int rho = idx / pw, i = idx % pw;
    const int r = c0 + rho;
    if (r >= rb && r < rb + nrows) st_coh(&a.qtop[rho * PNB + i], S[(c0 + i) * ldS + (r - rb)]);
  }
  gram_reduce(S, c0, ldS, rl0, nrows, pw, a.gram + kPanelMaxWG * 256, w, nwg, hb.sG, a.bar,
              a.err);
  for (int idx = tid; idx < pw * pw; idx += 256) {
    const int rho = idx / pw, i = idx % pw;
    hb.sQt[rho * PNB + i] = ld_coh(&a.qtop[rho * PNB + i]);
  }
  __syncthreads();
  if (wave == 0) {
    // ||Q1^T Q1 - I||_max < 0.1, else CholeskyQR lost too much orthogonality.
    bool ok = true;
    for (int e = lane; e < pw * pw; e += 64) {
      const int i = e / pw, j = e % pw;
      ok = ok && fabs(hb.sG[i * PNB + j] - (i == j ? 1.0 : 0.0)) < 0.1;
    }
    ok = __all(ok);
    ok = chol_wave(hb.sG, hb.sR2, pw, 1e-3) && ok;
    // Qt <- Qt R2^{-1}; R <- R2 R1 (into sLU, then back to sR1).
    if (lane < pw) {
      double x[PNB];
#pragma unroll
      for (int jc = 0; jc < PNB; ++jc) {
        if (jc >= pw) break;
        double v = hb.sQt[lane * PNB + jc];
        for (int i = 0; i < jc; ++i) v -= x[i] * hb.sR2[i * PNB + jc];
        x[jc] = v / hb.sR2[jc * PNB + jc];
      }
#pragma unroll
      for (int jc = 0; jc < PNB; ++jc) {
        if (jc >= pw) break;
        hb.sQt[lane * PNB + jc] = x[jc];
      }
    }
    for (int e = lane; e < pw * pw; e += 64) {
      const int i = e / pw, jc = e % pw;
      double v = 0.0;
      for (int k = i; k <= jc; ++k) v += hb.sR2[i * PNB + k] * hb.sR1[k * PNB + jc];
      hb.sLU[i * PNB + jc] = i <= jc ? v : 0.0;
    }
    wave_sync();
    for (int e = lane; e < pw * pw; e += 64) {
      const int i = e / pw, jc = e % pw;
      hb.sR1[i * PNB + jc] = hb.sLU[i * PNB + jc];
      hb.sLU[i * PNB + jc] = hb.sQt[i * PNB + jc];
    }
    wave_sync();
    // LU of Qt - diag(s) without pivoting; s_k = -sign(running pivot).
    double* A = hb.sLU;
    for (int k = 0; k < pw; ++k) {
      const double d = A[k * PNB + k];
      ok = ok && fabs(d) < 1.0 - 1.0 / 1125899906842624.0;  // else a zero tail
      const double sk = d >= 0.0 ? -1.0 : 1.0;
      const double piv = d - sk;
      wave_sync();
      if (lane == 0) {
        hb.ssgn[k] = sk;
        A[k * PNB + k] = piv;
      }
      if (lane > k && lane < pw) A[lane * PNB + k] /= piv;
      wave_sync();
      for (int e = lane; e < pw * pw; e += 64) {
        const int r = e / pw, cc = e % pw;
        if (r > k && cc > k) A[r * PNB + cc] -= A[r * PNB + k] * A[k * PNB + cc];
      }
      wave_sync();
    }
    if (lane == 0) hb.sflag[1] = ok;
  }
  __syncthreads();
  if (!hb.sflag[1]) {
    for (int idx = tid; idx < pw * nrows; idx += 256) {
      const int i = idx / nrows, rl = idx % nrows;
      S[(c0 + i) * ldS + rl] = hb.sP0[i * ldS + rl];
    }
    __syncthreads();
    return false;
  }
  // Second CholeskyQR pass on my rows: Q = Q1 R2^{-1}.
  rsolve_rows(S, c0, ldS, rl0, nrows, pw, hb.sR2);
  __syncthreads();
  // Rows below the sub-panel's top: V = Q U^{-1} (U = upper part of the LU).
  const int rtop = max(rl0, min(nrows, c0 + pw - rb));
  rsolve_rows(S, c0, ldS, rtop, nrows, pw, hb.sLU);
  // Top rows c0..c0+pw-1 that I own: R (signs applied) on/above, L below.
  for (int idx = tid; idx < pw * pw; idx += 256) {
    const int rho = idx / pw, i = idx % pw;
    const int r = c0 + rho;
    if (r >= rb && r < rb + nrows)
      S[(c0 + i) * ldS + (r - rb)] =
          rho <= i ? hb.ssgn[rho] * hb.sR1[rho * PNB + i] : hb.sLU[rho * PNB + i];
  }
  if (tid < pw) {
    const double tau = -hb.sLU[tid * PNB + tid] * hb.ssgn[tid];
    stau[c0 + tid] = tau;
    if (w == 0) a.tau[c0 + tid] = tau;
  }
  __syncthreads();
  return true;
}

__global__ __launch_bounds__(256) void k_panel_lds(PanelArgs2 a) {
  if (a.gate && *a.gate == 0) return;  // uniform over the grid: no barrier is entered
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  HrBufs hb;
  hb.sG = shh + 8;
  hb.sR1 = hb.sG + PNB * PNB;
  hb.sR2 = hb.sR1 + PNB * PNB;
  hb.sQt = hb.sR2 + PNB * PNB;
  hb.sLU = hb.sQt + PNB * PNB;
  hb.ssgn = hb.sLU + PNB * PNB;
  hb.sflag = (int*)(hb.ssgn + PNB);
  hb.sP0 = hb.ssgn + PNB + 8;  // PNB columns of stride ldS
  double* sVd = hb.sP0;        // dense sub-panel reflectors once factored
  const int64_t ldp = a.ldp;

  for (int idx = tid; idx < nb * nrows; idx += 256) {
    const int j = idx / nrows, rl = idx % nrows;
    S[j * ldS + rl] = a.P[rb + rl + (int64_t)j * ldp];
  }
  __syncthreads();
  int colstep = 0;
  for (int c0 = 0; c0 < nb; c0 += PNB) {
    const int pw = min(PNB, nb - c0);
    const bool hr_done =
        a.use_hr && pw > 1 && subpanel_cholqr_hr(S, c0, pw, ldS, rb, nrows, w, nwg, a, hb, stau);
    for (int cc = 0; cc < pw && !hr_done; ++cc, ++colstep) {
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
      grid_sync_coh(a.bar, nwg, a.err);
      {
        const int j = tid >> 4, li = tid & 15;
        double s = 0.0;
        if (j >= cc && j < pw) {
          double vals[kPanelMaxWG / 16];
#pragma unroll
          for (int k = 0; k < kPanelMaxWG / 16; ++k) {
            const int v = li + 16 * k;
            vals[k] = v < nwg ? ld_coh(&part[v * PNB + j]) : 0.0;
          }
#pragma unroll
          for (int k = 0; k < kPanelMaxWG / 16; ++k) s += vals[k];
        }
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
    const int rl0 = max(0, c0 - rb);
    // Dense reflectors of the sub-panel on my rows: Vd(t, rl), zero above
    // the diagonal and for t >= pw, one on it.
    for (int idx = tid; idx < PNB * nrows; idx += 256) {
      const int t = idx / nrows, rl = idx % nrows;
      const int r = rb + rl, d = c0 + t;
      sVd[t * ldS + rl] = t < pw ? (r > d ? S[d * ldS + rl] : (r == d ? 1.0 : 0.0)) : 0.0;
    }
    __syncthreads();
    // Partial products Vs^T [V_prev | Vs | P_rest] (kPanelNB x nb) over my
    // rows on FP64 MFMA: A = Vd^T (t x rows), B = the slab (rows x columns),
    // the sub-panel's own columns taken from Vd.  Output D(t, j) sits in
    // register r of lane l at t = l/16 + 4r, j = j0 + l%16.
    for (int jb = wave; jb < (nb + 15) / 16; jb += 4) {
      v4d acc = {0.0, 0.0, 0.0, 0.0};
      const int j = jb * 16 + (lane & 15);
      const bool jin = j < nb;
      const bool jv = j >= c0 && j < c0 + pw;
      for (int k0 = rl0; k0 < nrows; k0 += 4) {
        const int rl = k0 + (lane >> 4);
        const bool rin = rl < nrows;
        const double av = rin ? sVd[(lane & 15) * ldS + rl] : 0.0;
        const double bv = (rin && jin) ? (jv ? sVd[(j - c0) * ldS + rl] : S[j * ldS + rl]) : 0.0;
        acc = mfma64(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = (lane >> 4) + 4 * r;
        if (t < pw && jin) st_coh(&a.bpart[((int64_t)w * PNB + t) * nb + j], acc[r]);
      }
    }
    grid_sync_coh(a.bar, nwg, a.err);
    {
      // Entries [e0, e1) of the kPanelNB x nb product are summed here over
      // the nwg partials: 8 threads per entry, each over every 8th partial
      // with independent loads in flight, then a fixed-order 8-lane sum.
      const int E = pw * nb;
      const int e0 = (int)((int64_t)w * E / nwg), e1 = (int)((int64_t)(w + 1) * E / nwg);
      const int sub = tid & 7;
      for (int eb = e0; eb < e1; eb += 32) {
        const int e = eb + (tid >> 3);
        double s = 0.0;
        if (e < e1) {
          const int t = e / nb, j = e % nb;
          double vals[kPanelMaxWG / 8];
#pragma unroll
          for (int k = 0; k < kPanelMaxWG / 8; ++k) {
            const int v = sub + 8 * k;
            vals[k] = v < nwg ? ld_coh(&a.bpart[((int64_t)v * PNB + t) * nb + j]) : 0.0;
          }
#pragma unroll
          for (int k = 0; k < kPanelMaxWG / 8; ++k) s += vals[k];
        }
        s += __shfl_xor(s, 4, 8);
        s += __shfl_xor(s, 2, 8);
        s += __shfl_xor(s, 1, 8);
        if (e < e1 && sub == 0) st_coh(&a.red[e], s);
      }
    }
    grid_sync_coh(a.bar, nwg, a.err);
    {
      const int E = pw * nb;
      for (int e0 = 0; e0 < E; e0 += 256 * 8) {
        double vals[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int e = e0 + tid + 256 * k;
          vals[k] = e < E ? ld_coh(&a.red[e]) : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int e = e0 + tid + 256 * k;
          if (e < E) sred[e] = vals[k];
        }
      }
    }
    __syncthreads();
    // Ts: compact-WY factor of the sub-panel, column recurrence
    // Ts(0:t,t) = -tau_t Ts(0:t,0:t) Gram(0:t,t), Ts(t,t) = tau_t (wave 0).
    if (wave == 0) {
      for (int t = 0; t < PNB; ++t) {
        if (lane < PNB) {
          double v = 0.0;
          if (t < pw) {
            if (lane < t) {
              for (int k = lane; k < t; ++k) v += sTs[lane * PNB + k] * sred[k * nb + c0 + t];
              v = -stau[c0 + t] * v;
            } else if (lane == t) {
              v = stau[c0 + t];
            }
          }
          sTs[lane * PNB + t] = v;
        }
        wave_sync();
      }
    }
    __syncthreads();
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
    // W' = Ts^T W in place over sred[., j >= c0+pw].
    for (int j = c0 + pw + tid; j < nb; j += 256) {
      double wj[PNB];
#pragma unroll
      for (int t = 0; t < PNB; ++t) wj[t] = t < pw ? sred[t * nb + j] : 0.0;
#pragma unroll
      for (int t = 0; t < PNB; ++t) {
        if (t >= pw) continue;
        double v = 0.0;
        for (int tp = 0; tp <= t; ++tp) v += sTs[tp * PNB + t] * wj[tp];
        sred[t * nb + j] = v;
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
    // P_rest -= Vd W' on my rows, FP64 MFMA over 16 x 16 tiles:
    // A(row, t) = Vd(t, row), B(t, j) = W'(t, j), K = kPanelNB.
    {
      const int jr0 = c0 + pw;
      const int ncb = (nb - jr0 + 15) / 16, nrb = (nrows - rl0 + 15) / 16;
      for (int tile = wave; tile < ncb * nrb; tile += 4) {
        const int rt = tile % nrb, ct = tile / nrb;
        const int r0 = rl0 + rt * 16, j0 = jr0 + ct * 16;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t0 = 0; t0 < PNB; t0 += 4) {
          const int rl = r0 + (lane & 15), t = t0 + (lane >> 4);
          const int j = j0 + (lane & 15);
          const double av = (rl < nrows && t < pw) ? sVd[t * ldS + rl] : 0.0;
          const double bv = (j < nb && t < pw) ? sred[t * nb + j] : 0.0;
          acc = mfma64(av, bv, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rl = r0 + (lane >> 4) + 4 * r, j = j0 + (lane & 15);
          if (rl < nrows && j < nb) S[j * ldS + rl] -= acc[r];
        }
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
                          int64_t ldr, const int* gate) {
  if (gate && *gate == 0) return;
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
  size_t d = 2 * kPanelMaxWG * PNB + 2 * PNB + (size_t)kPanelMaxWG * PNB * bmax + PNB * bmax +
             2 * kPanelMaxWG * 256 + PNB * PNB;
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
  w->gram = p;
  p += 2 * kPanelMaxWG * 256;
  w->qtop = p;
  p += PNB * PNB;
  w->bar = (unsigned*)p;
  w->err = (int*)(w->bar + 2);
}

hipError_t panel_qr(hipStream_t st, int Mp, int nb, double* P, int64_t ldp, double* tau,
                    double* Tw, int64_t ldtw, const PanelWork& w, const int* gate) {
  if (nb <= 0) return hipSuccess;
  if (nb > MAXB || Mp < nb) return hipErrorInvalidValue;
  int dev = 0, cu_count = 1, lds = 64 * 1024;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cu_count, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cu_count = 1;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    lds = 64 * 1024;
  const int kLdsBytes = std::min(lds, 160 * 1024);
  const bool attr_set = ensure_dyn_lds((const void*)k_panel_lds, kLdsBytes) == hipSuccess;
  (void)hipGetLastError();
  // LDS-resident variant: slab of `chunk` rows x nb columns per workgroup.
  const int fixed = kFixedLdsDoubles(nb);
  const int max_ld = (kLdsBytes / 8 - fixed) / (nb + PNB);
  const int chunk_max = std::min(kPanelMaxRows, max_ld - 1);
  if (attr_set && chunk_max >= 1) {
    int nwg = (Mp + chunk_max - 1) / chunk_max;
    if (nwg <= std::min(cu_count, kPanelMaxWG)) {
      const int chunk = (Mp + nwg - 1) / nwg;
      nwg = (Mp + chunk - 1) / chunk;
      const int ldS = chunk | 1;
      const size_t shmem = ((size_t)(nb + PNB) * ldS + fixed) * sizeof(double);
      hipLaunchKernelGGL(k_init_sync, dim3(1), dim3(64), 0, st, w.bar);
      PanelArgs2 a{Mp, nb, nwg, chunk, ldS, nwg > 1 ? 1 : 0, P, ldp, tau, Tw, ldtw, w.part,
                   w.bcast, w.bpart, w.red, w.bar, w.err, gate, w.gram, w.qtop};
      void* args[] = {&a};
      const int slot = prof_mark(st, PC_PANEL);
      hipError_t e;
      if (gate) {
        // Gated (fallback) use: nearly always skipped, every workgroup
        // returning at once, so it is an ordinary launch on the caller's
        // stream; a cooperative launch goes through a queue of its own, and
        // the two cross-queue waits cost tens of microseconds per panel.
        // When it does run, its nwg <= CU-count workgroups (one per CU by
        // LDS) all become resident once the other streams' workgroups drain
        // (those streams wait on this one for new work), and every grid
        // barrier wait is bounded (the error word is raised on timeout).
        hipLaunchKernelGGL(k_panel_lds, dim3(nwg), dim3(256), shmem, st, a);
        e = hipGetLastError();
      } else {
        e = hipLaunchCooperativeKernel((const void*)k_panel_lds, dim3(nwg), dim3(256), args,
                                       (unsigned)shmem, st);
      }
      prof_done(st, slot, PC_PANEL, 2.0 * Mp * (double)nb * nb, 16.0 * Mp * (double)nb);
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
              w.bar, w.err, gate};
  void* args[] = {&a};
  const int slot = prof_mark(st, PC_PANEL);
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_panel, dim3(nwg), dim3(256), args, 0, st);
  prof_done(st, slot, PC_PANEL, 2.0 * Mp * (double)nb * nb, 16.0 * Mp * (double)nb);
  return e;
}

hipError_t panel_extract(hipStream_t st, int Mp, int nb, const double* P, int64_t ldp,
                         double* V, int64_t ldv, double* Rout, int64_t ldr, const int* gate) {
  const int64_t total = (int64_t)Mp * nb;
  if (total == 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_extract, dim3(blocks), dim3(256), 0, st, Mp, nb, P, ldp, V, ldv, Rout,
                     ldr, gate);
  return hipGetLastError();
}

}  // namespace rutv
