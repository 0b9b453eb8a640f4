// Optional per-kernel timing with HIP events recorded on the launch stream
// around each instrumented kernel (thin GEMMs, split-K reductions, panel QR,
// small SVDs).  Off unless randutv_profile_begin() was called; not
// thread-safe (one factorization at a time per process while profiling).
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/randutv.h"
#include "common.h"

namespace rutv {
namespace {

struct Rec {
  hipEvent_t a, b;
  int cls;
  double flops, bytes;
};

bool g_on = false;
int g_only = -1;     // >= 0: time launches of this class only
int g_suppress = 0;  // > 0 inside a composite region timed as one class
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

// Events are released when the process exits, before the HIP runtime's
// own teardown (the handler is registered after the runtime initialised).
void release_events() {
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  for (hipEvent_t e : g_pool)
    if (e) (void)hipEventDestroy(e);
  g_pool.clear();
}

hipEvent_t take_event() {
  static bool registered = false;
  if (!registered) {
    std::atexit(release_events);
    registered = true;
  }
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Class names: gemm_<op(A)op(B)>_<arithmetic>_<tile>, e.g. gemm_nt_fp32_t128
// is k_gemm<PREC_FP32, false, true, 128, 128, 2, 2>.
std::string class_name(int c) {
  if (c == PC_SPLITK) return "splitk_reduce";
  if (c == PC_PANEL) return "panel_qr";
  if (c == PC_SVD) return "small_svd";
  if (c == PC_GEMM_SMALL) return "gemm_small_fp64";
  static const char* ops[4] = {"nn", "tn", "nt", "tt"};
  if (c >= PC_UV) return std::string("gemm_") + ops[c - PC_UV] + "_fp64_t64_uv";
  static const char* precs[4] = {"fp64", "fp32", "bf16x3", "bf16x6"};
  static const char* tiles[2] = {"t64", "t128"};
  return std::string("gemm_") + ops[c % 4] + "_" + precs[(c / 4) % 4] + "_" + tiles[c / 16];
}

std::vector<std::string> g_names;

}  // namespace

bool prof_on() { return g_on; }

void prof_suppress(int delta) { g_suppress += delta; }

int prof_mark(hipStream_t st, int cls) {
  if (!g_on || g_suppress > 0 || (g_only >= 0 && cls != g_only)) return -1;
  hipEvent_t a = take_event(), b = take_event();
  if (!a || !b) return -1;
  if (hipEventRecord(a, st) != hipSuccess) return -1;
  g_recs.push_back(Rec{a, b, -1, 0.0, 0.0});
  return (int)g_recs.size() - 1;
}

void prof_done(hipStream_t st, int slot, int cls, double flops, double bytes) {
  if (slot < 0 || slot >= (int)g_recs.size()) return;
  Rec& r = g_recs[slot];
  r.cls = cls;
  r.flops = flops;
  r.bytes = bytes;
  (void)hipEventRecord(r.b, st);
}

}  // namespace rutv

using namespace rutv;

extern "C" {

int randutv_profile_begin_class(int cls) {
  if (cls >= PC_COUNT) return -1;
  for (auto& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_only = cls < 0 ? -1 : cls;
  g_on = true;
  return 0;
}

int randutv_profile_begin(void) { return randutv_profile_begin_class(-1); }

int randutv_profile_end(int max_classes, double* ms, double* flops, double* bytes,
                        int64_t* launches) {
  g_on = false;
  const int nc = max_classes < PC_COUNT ? max_classes : PC_COUNT;
  for (int c = 0; c < nc; ++c) {
    if (ms) ms[c] = 0.0;
    if (flops) flops[c] = 0.0;
    if (bytes) bytes[c] = 0.0;
    if (launches) launches[c] = 0;
  }
  int status = 0;
  for (auto& r : g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) status = RANDUTV_E_HIP;
    float t = 0.f;
    if (r.cls >= 0 && r.cls < nc && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      if (ms) ms[r.cls] += t;
      if (flops) flops[r.cls] += r.flops;
      if (bytes) bytes[r.cls] += r.bytes;
      if (launches) launches[r.cls] += 1;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  return status ? status : nc;
}

const char* randutv_profile_class_name(int cls) {
  if (g_names.empty())
    for (int c = 0; c < PC_COUNT; ++c) g_names.push_back(class_name(c));
  return cls >= 0 && cls < PC_COUNT ? g_names[cls].c_str() : "";
}

}  // extern "C"
