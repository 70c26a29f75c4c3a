// Autotuning of the FP32 Fourier-domain block product: every kernel variant
// (lane-per-row GEMV, MFMA GEMM with 1, 2 or 3 row tiles per wavefront) is
// timed with HIP events on the plan's own blocks and workspace, the fastest
// is kept in the plan for that right-hand-side count, and, when the
// environment variable EMSURF_TUNE_CACHE names a file, recorded there as
// "n_eq nrhs variant" lines so later processes reuse it.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "internal.h"

namespace emsurf {
namespace {

std::mutex g_cache_mu;
bool g_cache_loaded = false;
std::map<std::pair<int, int>, int> g_cache;   // (n_eq, nrhs) -> variant

const char* cache_path() {
  const char* p = std::getenv("EMSURF_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void load_cache_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  std::ifstream f(path);
  int n, r, v;
  while (f >> n >> r >> v)
    if (v >= 0 && v < BP_NVARIANTS) g_cache[{n, r}] = v;
}

void save_cache_locked() {
  const char* path = cache_path();
  if (!path) return;
  std::ofstream f(path, std::ios::trunc);
  for (auto& kv : g_cache) f << kv.first.first << " " << kv.first.second << " " << kv.second << "\n";
}

int heuristic(int n, int nrhs, bool structured) {
  if (!block_mfma_supported(n, nrhs) || nrhs < 8) return BP_GEMV;
  // deep prefetch, fewest row tiles per wave that fits in 4 wavefronts
  for (int v = BP_MFMA_T1D; v <= BP_MFMA_T4D; ++v)
    if (structured ? block_variant_supported_lk(v, n, nrhs) : block_variant_supported(v, n, nrhs)) return v;
  return BP_GEMV;
}

}  // namespace

int choose_variant(emsurf_plan p, int nrhs) {
  const int n = p->d.n_eq;
  if (nrhs >= 1 && nrhs <= 64 && p->bp_variant[nrhs] >= 0) return p->bp_variant[nrhs];
  // the persisted cache holds dense-block choices only
  if (p->d.form == EMSURF_T_LK) return heuristic(n, nrhs, true);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    load_cache_locked();
    auto it = g_cache.find({n, nrhs});
    if (it != g_cache.end()) return it->second;
  }
  return heuristic(n, nrhs, false);
}

}  // namespace emsurf

using namespace emsurf;

extern "C" emsurf_status emsurf_plan_set_variant(emsurf_plan plan, int32_t nrhs, int32_t variant) {
  try {
    EMS_CHECK_ARG(plan != nullptr, "plan is NULL");
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= plan->d.max_rhs, "nrhs must be in [1, max_rhs]");
    EMS_CHECK_ARG(variant >= -1 && variant < BP_NVARIANTS, "unknown block-product variant");
    const bool structured = plan->d.form == EMSURF_T_LK;
    if (variant > BP_GEMV && plan->d.recip) {
      set_error("reciprocal plans have a single (paired) block-product kernel");
      throw Err{EMSURF_ERR_UNSUPPORTED};
    }
    if (variant > BP_GEMV && !(structured ? block_variant_supported_lk(variant, plan->d.n_eq, nrhs)
                                          : block_variant_supported(variant, plan->d.n_eq, nrhs))) {
      set_error("this MFMA block-product variant needs n_eq a multiple of 32 (<= 480) and at most 4 "
                "wavefronts of row tiles");
      throw Err{EMSURF_ERR_UNSUPPORTED};
    }
    plan->bp_variant[nrhs] = variant;
    return EMSURF_OK;
  } catch (...) {
    return current_exception_status();
  }
}

extern "C" emsurf_status emsurf_plan_autotune(emsurf_plan plan, int32_t nrhs, double* ms_out, int32_t* best_out,
                                              void* stream) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    EMS_CHECK_ARG(plan != nullptr, "plan is NULL");
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= plan->d.max_rhs, "nrhs must be in [1, max_rhs]");
    if (!plan->that32.p) {
      set_error("plan has no FP32 Fourier-domain store");
      throw Err{EMSURF_ERR_UNSUPPORTED};
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace& w = workspace(plan, s);
    const int n = plan->d.n_eq;
    EMS_HIP(hipEventCreate(&e0));
    EMS_HIP(hipEventCreate(&e1));
    // time every candidate on the same defined input (the spectral workspace
    // may hold anything, including values that slow the arithmetic)
    EMS_HIP(hipMemsetAsync(w.X.p, 0, w.X.bytes, s));
    int best = BP_GEMV;
    double best_ms = 1e300;
    // structured (L, K) plans time their own kernels under the same variant numbers
    const bool structured = plan->d.form == EMSURF_T_LK;
    // reciprocal plans have one kernel, the paired product, timed as variant 0
    const bool recip = plan->d.recip != 0;
    auto run = [&](int v) {
      if (recip && structured)
        launch_block_product_pair_lk(Cx::C64, plan->that32.p, plan->pairs.p, plan->w32.p, plan->winv32.p, w.X.p,
                                     w.Y.p, n / 2, nrhs, plan->Ps, plan->d.coef, s);
      else if (recip)
        launch_block_product_pair(Cx::C64, plan->that32.p, plan->pairs.p, plan->w32.p, plan->winv32.p, w.X.p, w.Y.p,
                                  n, nrhs, plan->Ps, s);
      else if (structured)
        launch_block_product_lk(Cx::C64, v, plan->that32.p, w.X.p, w.Y.p, n / 2, nrhs, plan->P, plan->d.coef, s);
      else
        launch_block_product_variant(Cx::C64, v, plan->that32.p, w.X.p, w.Y.p, n, nrhs, plan->P, s);
    };
    for (int v = 0; v < BP_NVARIANTS; ++v) {
      double ms = -1.0;
      const bool ok = recip ? v == BP_GEMV
                            : structured ? block_variant_supported_lk(v, n, nrhs) : block_variant_supported(v, n, nrhs);
      if (ok) {
        run(v);  // warm-up
        const int reps = 3;
        EMS_HIP(hipEventRecord(e0, s));
        for (int i = 0; i < reps; ++i) run(v);
        EMS_HIP(hipEventRecord(e1, s));
        EMS_HIP(hipEventSynchronize(e1));
        float f = 0;
        EMS_HIP(hipEventElapsedTime(&f, e0, e1));
        ms = f / reps;
        if (ms < best_ms) { best_ms = ms; best = v; }
      }
      if (ms_out) ms_out[v] = ms;
    }
    plan->bp_variant[nrhs] = best;
    if (best_out) *best_out = best;
    if (!structured && !recip) {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      load_cache_locked();
      g_cache[{n, nrhs}] = best;
      save_cache_locked();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return EMSURF_OK;
  } catch (...) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return current_exception_status();
  }
}
