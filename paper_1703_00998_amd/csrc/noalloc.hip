// Allocation-free form of randutv_factor, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).  The workspace randutv_factor takes from the caller
// is a file-scope device array here, one copy per GPU, held until the process
// ends; its address on each device is looked up once, with that device
// current, and kept.  The array lives in this translation unit only, so a
// process that never calls this entry point never loads it.
#include <mutex>

#include "../../include/randutv.h"
#include "common.h"

// 128 MiB: the workspace of a 3800 x 3800 factorization with b = 128 and U, V
// formed (123 MiB) fits; larger ones (4000 x 4000 with b = 128 needs
// 129 MiB) are rejected.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device
std::mutex g_scratch_mu;

}  // namespace

extern "C" {

int randutv_factor_noalloc(int64_t m, int64_t n, int64_t b, int q, double* T, int64_t ldt,
                           const double* G, int64_t ldg, double* U, int64_t ldu, double* V,
                           int64_t ldv, int64_t k_stop, double tol, int prec, unsigned flags,
                           int64_t* k_out, void* stream) {
  size_t need = 0;
  const int s = randutv_workspace_size(m, n, b, q, prec, flags, &need);
  if (s != 0) {  // map the sizing call's argument numbers onto this call's
    switch (s) {
      case -1: return -1;
      case -3: return -2;
      case -4: return -3;
      case -5: return -10;
      case -6: return -11;
      default: return s;
    }
  }
  // The pointer arguments are checked here too, before the device is asked
  // for the array's address.
  if (!T || ldt < m) return -4;
  if (randutv_g_cols(m, n, b) > 0 && (!G || ldg < m)) return -5;
  if ((flags & RANDUTV_FORM_U) && (!U || ldu < m)) return -6;
  if ((flags & RANDUTV_FORM_V) && (!V || ldv < n)) return -7;
  if (need > kScratchBytes) return RANDUTV_E_WORKSPACE;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return RANDUTV_E_HIP - (int)e;
  if (dev < 0 || dev >= kMaxDevices) return RANDUTV_E_UNSUPPORTED;
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
      e = hipGetSymbolAddress(&g_scratch[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        g_scratch[dev] = nullptr;
        return RANDUTV_E_HIP - (int)e;
      }
    }
    ptr = g_scratch[dev];
  }
  // The factorization initialises every part of its workspace it reads
  // (status words, barrier counters, sweep counters) on the stream, so the
  // previous call's contents do no harm; calls that overlap on one GPU share
  // the array and race.
  return rutv::factor_core(m, n, b, 0, q, T, ldt, G, ldg, U, ldu, V, ldv, k_stop, tol, prec, flags,
                           ptr, kScratchBytes, k_out, stream, nullptr, false);
}

}  // extern "C"
