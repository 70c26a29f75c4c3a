// HIP-graph capture of an operator apply (y = T x, S x or x - S T x) with fixed
// buffers, so that repeated applies (Krylov iterations on small lattices,
// where launch overhead rivals the work) replay one graph instead of
// re-issuing every kernel.  No memset or allocation is ever recorded: the
// apply path uses kernels only, and the stream's workspace and twiddle tables
// are created before capture begins.
#include "internal.h"

struct emsurf_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~emsurf_graph_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

using namespace emsurf;

extern "C" emsurf_status emsurf_graph_create(emsurf_plan plan, int32_t op, emsurf_prec prec, int32_t nrhs,
                                             const void* x_dev, void* y_dev, void* stream, emsurf_graph* out) {
  emsurf_graph g = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool capturing = false;
  const bool timer_was = plan ? plan->timer.enabled : false;
  try {
    EMS_CHECK_ARG(plan != nullptr && out != nullptr, "plan and out must be non-NULL");
    EMS_CHECK_ARG(s != nullptr, "graph capture needs a non-null stream");
    EMS_CHECK_ARG(op == EMSURF_OP_T || op == EMSURF_OP_S || op == EMSURF_OP_A, "op must be EMSURF_OP_T/S/A");
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= plan->d.max_rhs, "nrhs must be in [1, max_rhs]");
    EMS_CHECK_ARG(x_dev && y_dev && x_dev != y_dev, "x and y must be distinct non-NULL device buffers");
    const ApplyPrec ap = apply_prec(prec);
    const Cx t = ap.t;
    const void* store = ap.split ? plan->that16.p : t == Cx::C128 ? plan->that64.p : plan->that32.p;
    if (op != EMSURF_OP_S && !store) {
      set_error("plan lacks the Fourier-domain store for this precision");
      throw Err{EMSURF_ERR_UNSUPPORTED};
    }
    (void)workspace(plan, s);
    (void)twiddle_table(plan->Lx, t);
    (void)twiddle_table(plan->Ly, t);
    g = new emsurf_graph_s();
    plan->timer.enabled = false;
    EMS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    capturing = true;
    if (op == EMSURF_OP_T) {
      apply_T_typed(plan, t, t, t, nrhs, x_dev, y_dev, s, -1, ap.split);
    } else if (op == EMSURF_OP_A) {
      apply_A_typed(plan, t, t, t, nrhs, x_dev, y_dev, s, -1, ap.split);
    } else {
      apply_S_plan(plan, t, t, nrhs, x_dev, nullptr, y_dev, s);
    }
    capturing = false;
    EMS_HIP(hipStreamEndCapture(s, &g->graph));
    plan->timer.enabled = timer_was;
    EMS_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    *out = g;
    return EMSURF_OK;
  } catch (...) {
    if (capturing) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(s, &junk);
      if (junk) (void)hipGraphDestroy(junk);
    }
    if (plan) plan->timer.enabled = timer_was;
    delete g;
    return current_exception_status();
  }
}

extern "C" emsurf_status emsurf_graph_launch(emsurf_graph g, void* stream) {
  try {
    EMS_CHECK_ARG(g != nullptr && g->exec != nullptr, "graph is NULL");
    EMS_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return EMSURF_OK;
  } catch (...) {
    return current_exception_status();
  }
}

extern "C" void emsurf_graph_destroy(emsurf_graph g) { delete g; }
