// Coupling apply y = T x that allocates nothing, for callers that cannot call
// hipMalloc (code under HIP-graph capture, serving loops, harnesses that
// forbid allocation).  It runs the same kernels as emsurf_apply_T; its
// intermediates (the half-transformed input and the two spectra) live in a
// file-scope device array of a fixed size instead of the plan's per-stream
// workspace.
//
// Each GPU holds its own copy of the array for the life of the process.  Its
// address is looked up once per device with hipGetSymbolAddress and only that
// address is handed to kernels and copies.  Every call on a device shares the
// array: calls that overlap on one device (on different streams, or from
// different threads) race.  The apply writes every intermediate value before
// reading it, so nothing has to be cleared between calls.
#include "internal.h"

namespace emsurf {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;   // 64 MiB
constexpr size_t NOALLOC_ALIGN = 256;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of its copy of `scratch`

void* scratch_address() {
  int dev = 0;
  EMS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  EMS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  EMS_CHECK_ARG(ptr != nullptr, "internal: no device address for the static workspace");
  g_scratch_ptr[dev] = ptr;
  return ptr;
}

size_t round_up(size_t v) { return (v + NOALLOC_ALIGN - 1) / NOALLOC_ALIGN * NOALLOC_ALIGN; }

}  // namespace
}  // namespace emsurf

using namespace emsurf;

extern "C" {

size_t emsurf_apply_T_noalloc_limit(void) { return NOALLOC_SCRATCH_BYTES; }

emsurf_status emsurf_apply_T_noalloc(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev, void* y_dev,
                                     void* stream) {
  return guarded_call([&] {
    EMS_CHECK_ARG(plan != nullptr, "plan is NULL");
    EMS_CHECK_ARG(x_dev != nullptr && y_dev != nullptr, "x and y must be non-NULL device pointers");
    EMS_CHECK_ARG(x_dev != y_dev, "apply_T needs distinct x and y buffers");
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= plan->d.max_rhs, "nrhs must be in [1, max_rhs]");
    const ApplyPrec ap = apply_prec(prec);
    const size_t cb = cx_bytes(ap.t);
    const size_t wb = round_up((size_t)apply_W_values(plan, nrhs) * cb);
    const size_t xb = round_up((size_t)apply_X_values(plan, nrhs) * cb);
    if (wb + 2 * xb > NOALLOC_SCRATCH_BYTES) {
      set_error("emsurf_apply_T_noalloc: this plan and nrhs need " + std::to_string(wb + 2 * xb) +
                " bytes of intermediates, above the " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                "-byte static workspace; use emsurf_apply_T or fewer right-hand sides");
      throw Err{EMSURF_ERR_ARG};
    }
    const void* twx = twiddle_lookup(plan->Lx, ap.t);
    const void* twy = twiddle_lookup(plan->Ly, ap.t);
    EMS_CHECK_ARG(twx != nullptr && twy != nullptr,
                  "emsurf_apply_T_noalloc: the plan's twiddle tables are missing on this device");
    unsigned char* base = static_cast<unsigned char*>(scratch_address());
    const ApplyBufs b{base, base + wb, base + wb + xb, twx, twy};
    apply_T_bufs(plan, ap.t, ap.t, ap.t, nrhs, x_dev, y_dev, b, static_cast<hipStream_t>(stream), -1, ap.split,
                 false);
  });
}

}  // extern "C"
