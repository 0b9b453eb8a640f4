// Elementwise and reduction helpers of the randUTV driver: copies, zeroing
// (Figure "The algorithm randUTV": T(I3,J2) = 0), writing the diagonal block
// T(I2,J2) = Ds, identity initialisation of U and V, and the Frobenius norm
// of the trailing block used by the early-stop test (Section 1.1 (ii)), and
// the status words a call leaves in its workspace.
// All of them are HBM-bound single passes over column-major data.
#include <algorithm>
#include <mutex>
#include <set>
#include <utility>

#include "../../include/randutv.h"
#include "common.h"

namespace rutv {
namespace {

inline int grid_for(int64_t total) {
  return (int)std::min<int64_t>((total + 255) / 256, 8192);
}

__global__ void k_copy(int M, int N, const double* __restrict__ A, int64_t lda,
                       double* __restrict__ B, int64_t ldb) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M);
    const int64_t j = idx / M;
    B[i + j * ldb] = A[i + j * lda];
  }
}

__global__ void k_fill(int M, int N, double* __restrict__ A, int64_t lda, double diag,
                       double off) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M);
    const int64_t j = idx / M;
    A[i + j * lda] = (i == j) ? diag : off;
  }
}

__global__ void k_diag_block(int M, int nb, const double* __restrict__ D, double* __restrict__ A,
                             int64_t lda) {
  const int64_t total = (int64_t)M * nb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M);
    const int j = (int)(idx / M);
    A[i + (int64_t)j * lda] = (i == j) ? D[j] : 0.0;
  }
}

__global__ void k_status_init(StatusBlock* blk) {
  if (threadIdx.x == 0) {
    blk->sync_err = 0;
    blk->svd_fail = 0;
    blk->k = -1;
    blk->magic = 0;
    blk->pad = 0;
  }
}

__global__ void k_status_done(StatusBlock* blk, long long k) {
  if (threadIdx.x == 0) {
    blk->k = k;
    blk->magic = kStatusMagic;
  }
}

__global__ void k_sumsq_part(int M, int N, const double* __restrict__ A, int64_t lda,
                             double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t total = (int64_t)M * N;
  double s = 0.0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % M);
    const int64_t j = idx / M;
    const double x = A[i + j * lda];
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sumsq_final(int nparts, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

hipError_t copy_matrix(hipStream_t st, int M, int N, const double* A, int64_t lda, double* B,
                       int64_t ldb) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(grid_for((int64_t)M * N)), dim3(256), 0, st, M, N, A, lda, B,
                     ldb);
  return hipGetLastError();
}

hipError_t set_zero(hipStream_t st, int M, int N, double* A, int64_t lda) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)M * N)), dim3(256), 0, st, M, N, A, lda, 0.0,
                     0.0);
  return hipGetLastError();
}

hipError_t set_identity(hipStream_t st, int M, int N, double* A, int64_t lda) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)M * N)), dim3(256), 0, st, M, N, A, lda, 1.0,
                     0.0);
  return hipGetLastError();
}

hipError_t set_diag_block(hipStream_t st, int M, int nb, const double* D, double* A,
                          int64_t lda) {
  if (M <= 0 || nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_block, dim3(grid_for((int64_t)M * nb)), dim3(256), 0, st, M, nb, D,
                     A, lda);
  return hipGetLastError();
}

hipError_t sumsq(hipStream_t st, int M, int N, const double* A, int64_t lda, double* scratch,
                 double* out) {
  const int nparts = 1024;
  if (M <= 0 || N <= 0) {
    hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(256), 0, st, 0, scratch, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_sumsq_part, dim3(nparts), dim3(256), 0, st, M, N, A, lda, scratch);
  hipLaunchKernelGGL(k_sumsq_final, dim3(1), dim3(256), 0, st, nparts, scratch, out);
  return hipGetLastError();
}

hipError_t status_init(hipStream_t st, StatusBlock* blk) {
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, st, blk);
  return hipGetLastError();
}

hipError_t status_done(hipStream_t st, StatusBlock* blk, long long k) {
  hipLaunchKernelGGL(k_status_done, dim3(1), dim3(64), 0, st, blk, k);
  return hipGetLastError();
}

int read_status(const void* work, int64_t* k_out, hipStream_t st) {
  hipError_t e = hipStreamSynchronize(st);
  StatusBlock h{};
  if (e == hipSuccess) e = hipMemcpy(&h, work, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return RANDUTV_E_HIP - (int)e;
  if (h.magic != kStatusMagic) return RANDUTV_E_UNSUPPORTED;
  if (k_out) *k_out = h.k;
  if (h.sync_err) return RANDUTV_E_SYNC;
  return h.svd_fail ? 1 : 0;
}

hipError_t ensure_dyn_lds(const void* fn, int bytes) {
  static std::mutex mu;
  static std::set<std::pair<int, const void*>> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({dev, fn})) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) done.insert({dev, fn});
  return e;
}

}  // namespace rutv
