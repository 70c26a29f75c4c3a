// Host driver of the batched restarted GMRES solve (Sec. IV-A) and of the
// FP32-inner / FP64-refinement variant.
//
// Reading of the solver (the paper only names GMRES): restarted GMRES(m) of
// Saad and Schultz; classical Gram-Schmidt applied twice per Arnoldi step with
// the Hermitian inner product; complex Givens rotations (real cosine) on the
// host in FP64; a cycle stops when the estimated relative residual meets the
// tolerance, on a lucky breakdown (h_{j+1,j} <= 1e-14 ||A v_j||), at the step
// limit or at the end of the cycle; then x += V y and, for the top-level solve,
// the true residual ||b - A x|| decides whether to stop or restart.  Every
// right-hand side runs its own instance; they advance in lockstep so that all
// share one batched operator apply, and an instance that has stopped carries a
// zero basis vector until the cycle ends.
//
// Mixed precision (GMRES-IR): outer r = b - A x with the FP64 operator; inner
// GMRES on A d = r with the FP32 operator (FP32 FFTs and products, FP64 basis,
// inner products and Hessenberg); x += d.
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"
#include "vecops.h"

namespace emsurf {
namespace {

using cd = std::complex<double>;

}  // namespace

// Buffers grow to the largest (nrhs, restart) a stream has used and are reused
// by later solves on that stream.
struct SolveWork {
  int nrhs = 0, m = 0;
  long long N = 0;
  int nblk = 0, rstride = 0;
  DevBuf V;        // (m+1) x nrhs x N
  DevBuf r, t;     // nrhs x N
  DevBuf partial;  // nrhs x nblk x (m+2)
  DevBuf red;      // nrhs x rstride
  DevBuf scale;    // nrhs doubles
  DevBuf ycoef;    // nrhs x m complex
  DevBuf mask;     // nrhs ints
  DevBuf ir_r, ir_d, ir_t;  // refinement residual, correction, operator output: nrhs x N each
  DevBuf pz, pz2;           // right preconditioning: P^-1 v and P^-1 V y, nrhs x N each
  PinnedBuf h_red, h_scale, h_y, h_mask;
  void init(int nrhs_, int m_, long long N_) {
    nrhs = nrhs_;
    m = m_;
    N = N_;
    nblk = dot_blocks(N);
    rstride = 2 * (m + 2) + 4;
    V.reserve((size_t)(m + 1) * nrhs * N * 16);
    r.reserve((size_t)nrhs * N * 16);
    t.reserve((size_t)nrhs * N * 16);
    partial.reserve((size_t)nrhs * nblk * (m + 2) * 16);
    red.reserve((size_t)nrhs * rstride * 16);
    scale.reserve((size_t)nrhs * 8);
    ycoef.reserve((size_t)nrhs * m * 16);
    mask.reserve((size_t)nrhs * 4);
    h_red.reserve((size_t)nrhs * rstride * 16);
    h_scale.reserve((size_t)nrhs * 8);
    h_y.reserve((size_t)nrhs * m * 16);
    h_mask.reserve((size_t)nrhs * 4);
  }
  double2* Vp(int l) const { return V.as<double2>() + (size_t)l * nrhs * N; }
  void init_refinement() {
    ir_r.reserve((size_t)nrhs * N * 16);
    ir_d.reserve((size_t)nrhs * N * 16);
    ir_t.reserve((size_t)nrhs * N * 16);
  }
  void init_precond() {
    pz.reserve((size_t)nrhs * N * 16);
    pz2.reserve((size_t)nrhs * N * 16);
  }
  size_t bytes() const {
    return V.bytes + r.bytes + t.bytes + partial.bytes + red.bytes + scale.bytes + ycoef.bytes + mask.bytes +
           ir_r.bytes + ir_d.bytes + ir_t.bytes + pz.bytes + pz2.bytes;
  }
};

void destroy_solve_work(SolveWork* w) { delete w; }
size_t solve_work_bytes(const SolveWork* w) { return w ? w->bytes() : 0; }

namespace {

using OpFn = void (*)(emsurf_plan, int, const void*, void*, hipStream_t);

void op_fp64(emsurf_plan p, int nrhs, const void* x, void* y, hipStream_t s) {
  apply_A_typed(p, Cx::C128, Cx::C128, Cx::C128, nrhs, x, y, s);
}
void op_fp32(emsurf_plan p, int nrhs, const void* x, void* y, hipStream_t s) {
  apply_A_typed(p, Cx::C128, Cx::C64, Cx::C128, nrhs, x, y, s);
}

// per-RHS norms of vec ([nrhs][N]) into host array
void norms(SolveWork& w, const void* vec, std::vector<double>& out, hipStream_t s) {
  launch_dot(nullptr, 0, 0, vec, w.N, w.nrhs, w.partial.p, w.nblk, w.red.p, w.rstride, 0, s);
  EMS_HIP(hipMemcpyAsync(w.h_red.p, w.red.p, (size_t)w.nrhs * w.rstride * 16, hipMemcpyDeviceToHost, s));
  EMS_HIP(hipStreamSynchronize(s));
  const double2* h = w.h_red.as<double2>();
  out.resize(w.nrhs);
  for (int r = 0; r < w.nrhs; ++r) out[r] = std::sqrt(h[(size_t)r * w.rstride].x);
}

void givens(cd a, cd b, double& c, cd& s) {
  if (b == 0.0) { c = 1.0; s = 0.0; return; }
  if (a == 0.0) { c = 0.0; s = std::conj(b) / std::abs(b); return; }
  const double r = std::hypot(std::abs(a), std::abs(b));
  c = std::abs(a) / r;
  s = (a / std::abs(a)) * std::conj(b) / r;
}

struct RhsState {
  double bnorm = 0;
  bool done = false, converged = false;
  int iters = 0, cycles = 0;
  double rel = 0;
  // per cycle
  bool stopped = false, est_ok = false;
  int kend = 0;
  std::vector<cd> H;   // (m+1) x m column-major
  std::vector<double> cs;
  std::vector<cd> sn, g;
};

// Batched GMRES on op(x) = b.  x holds the start (zeros or x0).  `confirm`
// selects the true-residual check after a converged cycle (top-level solve).
// pc (or NULL): right preconditioner, the Arnoldi process runs on op P^-1 and
// a cycle ends with x += P^-1 V y.
void gmres(emsurf_plan p, OpFn op, emsurf_precond pc, SolveWork& w, int nrhs, const double2* b, double2* x,
           const std::vector<double>& tol, int max_iter, bool confirm, bool start_zero, std::vector<RhsState>& st,
           hipStream_t s) {
  const int m = w.m;
  const long long N = w.N;
  const long long vstride = (long long)nrhs * N;
  for (bool first = true;; first = false) {
    // ---- (true) residual r = b - A x for RHS still running (r = b when x = 0)
    int* hm = w.h_mask.as<int>();
    bool any = false;
    for (int r = 0; r < nrhs; ++r) { hm[r] = st[r].done ? 0 : 1; any = any || hm[r]; }
    if (!any) return;
    if (first && start_zero) {
      double* hs0 = w.h_scale.as<double>();
      for (int r = 0; r < nrhs; ++r) hs0[r] = hm[r] ? 1.0 : 0.0;
      EMS_HIP(hipMemcpyAsync(w.scale.p, hs0, (size_t)nrhs * 8, hipMemcpyHostToDevice, s));
      launch_scale(b, w.scale.p, w.r.p, N, nrhs, s);
    } else {
      EMS_HIP(hipMemcpyAsync(w.mask.p, hm, (size_t)nrhs * 4, hipMemcpyHostToDevice, s));
      op(p, nrhs, x, w.t.p, s);
      launch_sub(b, w.t.p, w.mask.as<int>(), w.r.p, N, nrhs, s);
    }
    std::vector<double> beta;
    norms(w, w.r.p, beta, s);
    for (int r = 0; r < nrhs; ++r) {
      if (st[r].done) continue;
      st[r].rel = beta[r] / st[r].bnorm;
      if (st[r].rel <= tol[r]) { st[r].done = true; st[r].converged = true; }
      else if (st[r].iters >= max_iter) { st[r].done = true; st[r].converged = false; }
    }
    any = false;
    for (int r = 0; r < nrhs; ++r) any = any || !st[r].done;
    if (!any) return;
    // ---- start a cycle: v0 = r / beta
    double* hs = w.h_scale.as<double>();
    for (int r = 0; r < nrhs; ++r) {
      RhsState& q = st[r];
      q.stopped = q.done;
      q.est_ok = false;
      q.kend = 0;
      q.H.assign((size_t)(m + 1) * m, cd(0));
      q.cs.assign(m, 0.0);
      q.sn.assign(m, cd(0));
      q.g.assign(m + 1, cd(0));
      q.g[0] = beta[r];
      hs[r] = q.done ? 0.0 : 1.0 / beta[r];
    }
    EMS_HIP(hipMemcpyAsync(w.scale.p, hs, (size_t)nrhs * 8, hipMemcpyHostToDevice, s));
    launch_scale(w.r.p, w.scale.p, w.Vp(0), N, nrhs, s);
    for (int j = 0; j < m; ++j) {
      double2* wv = w.Vp(j + 1);
      if (pc) {
        precond_apply(pc, nrhs, w.Vp(j), w.pz.p, s);
        op(p, nrhs, w.pz.p, wv, s);
      } else {
        op(p, nrhs, w.Vp(j), wv, s);
      }
      // CGS2: red layout per RHS: [c1 (j+1)][|w0|^2][c2 (j+1)][|w1|^2][|w2|^2]
      const int nv = j + 1;
      const int o1 = 0, o2 = nv + 1, o3 = 2 * nv + 2;
      launch_dot(w.V.p, vstride, nv, wv, N, nrhs, w.partial.p, w.nblk, w.red.p, w.rstride, o1, s);
      launch_update(w.V.p, vstride, nv, w.red.p, w.rstride, o1, wv, N, nrhs, s);
      launch_dot(w.V.p, vstride, nv, wv, N, nrhs, w.partial.p, w.nblk, w.red.p, w.rstride, o2, s);
      launch_update(w.V.p, vstride, nv, w.red.p, w.rstride, o2, wv, N, nrhs, s);
      launch_dot(nullptr, 0, 0, wv, N, nrhs, w.partial.p, w.nblk, w.red.p, w.rstride, o3, s);
      EMS_HIP(hipMemcpyAsync(w.h_red.p, w.red.p, (size_t)w.nrhs * w.rstride * 16, hipMemcpyDeviceToHost, s));
      EMS_HIP(hipStreamSynchronize(s));
      const double2* hr = w.h_red.as<double2>();
      bool all_stopped = true;
      for (int r = 0; r < nrhs; ++r) {
        RhsState& q = st[r];
        if (q.stopped) { hs[r] = 0.0; continue; }
        const double2* R = hr + (size_t)r * w.rstride;
        cd* Hc = &q.H[(size_t)j * (m + 1)];
        for (int i = 0; i <= j; ++i) Hc[i] = cd(R[o1 + i].x, R[o1 + i].y) + cd(R[o2 + i].x, R[o2 + i].y);
        const double wn0 = std::sqrt(R[o1 + nv].x);
        const double hn = std::sqrt(R[o3].x);
        Hc[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
          const cd tmp = q.cs[i] * Hc[i] + q.sn[i] * Hc[i + 1];
          Hc[i + 1] = -std::conj(q.sn[i]) * Hc[i] + q.cs[i] * Hc[i + 1];
          Hc[i] = tmp;
        }
        givens(Hc[j], Hc[j + 1], q.cs[j], q.sn[j]);
        Hc[j] = q.cs[j] * Hc[j] + q.sn[j] * Hc[j + 1];
        Hc[j + 1] = 0.0;
        q.g[j + 1] = -std::conj(q.sn[j]) * q.g[j];
        q.g[j] = q.cs[j] * q.g[j];
        q.iters += 1;
        const double est = std::abs(q.g[j + 1]) / q.bnorm;
        const bool lucky = hn <= 1e-14 * wn0;
        if (est <= tol[r] || lucky || q.iters >= max_iter || j == m - 1) {
          q.stopped = true;
          q.kend = j + 1;
          q.est_ok = est <= tol[r] || lucky;
          hs[r] = 0.0;
        } else {
          hs[r] = 1.0 / hn;
          all_stopped = false;
        }
      }
      if (all_stopped) break;
      EMS_HIP(hipMemcpyAsync(w.scale.p, hs, (size_t)nrhs * 8, hipMemcpyHostToDevice, s));
      launch_scale(wv, w.scale.p, wv, N, nrhs, s);
    }
    // ---- x += V y  (y from the triangular system of each RHS)
    cd* hy = reinterpret_cast<cd*>(w.h_y.p);
    int kmax = 0;
    for (int r = 0; r < nrhs; ++r) {
      RhsState& q = st[r];
      cd* y = hy + (size_t)r * m;
      for (int i = 0; i < m; ++i) y[i] = 0.0;
      const int k = q.done ? 0 : q.kend;
      for (int i = k - 1; i >= 0; --i) {
        cd acc = q.g[i];
        for (int l = i + 1; l < k; ++l) acc -= q.H[(size_t)l * (m + 1) + i] * y[l];
        y[i] = acc / q.H[(size_t)i * (m + 1) + i];
      }
      if (k > kmax) kmax = k;
      if (!q.done) q.cycles += 1;
    }
    EMS_HIP(hipMemcpyAsync(w.ycoef.p, hy, (size_t)nrhs * m * 16, hipMemcpyHostToDevice, s));
    if (pc) {
      EMS_HIP(hipMemsetAsync(w.pz.p, 0, (size_t)nrhs * N * 16, s));
      launch_axpy_basis(w.V.p, vstride, kmax, w.ycoef.p, m, w.pz.p, N, nrhs, s);
      precond_apply(pc, nrhs, w.pz.p, w.pz2.p, s);
      launch_add(x, w.pz2.p, (long long)nrhs * N, s);
    } else {
      launch_axpy_basis(w.V.p, vstride, kmax, w.ycoef.p, m, x, N, nrhs, s);
    }
    if (!confirm) {
      // inner solve: accept the estimate
      for (int r = 0; r < nrhs; ++r) {
        RhsState& q = st[r];
        if (q.done) continue;
        if (q.est_ok) { q.done = true; q.converged = true; q.rel = std::abs(q.g[q.kend]) / q.bnorm; }
        else if (q.iters >= max_iter) { q.done = true; q.converged = false; }
      }
    }
  }
}

void check_opts(emsurf_plan plan, const emsurf_solve_opts* o, int32_t nrhs) {
  EMS_CHECK_ARG(plan != nullptr, "plan is NULL");
  EMS_CHECK_ARG(o != nullptr, "opts is NULL");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= plan->d.max_rhs, "nrhs must be in [1, max_rhs]");
  EMS_CHECK_ARG(std::isfinite(o->tol) && o->tol > 0, "tol must be > 0");
  EMS_CHECK_ARG(o->restart >= 1 && o->restart <= 64, "restart must be in [1, 64]");
  EMS_CHECK_ARG(o->max_iter >= 1, "max_iter must be >= 1");
  EMS_CHECK_ARG(o->prec == EMSURF_FP64 || o->prec == EMSURF_FP32 || o->prec == EMSURF_FP32_IR,
                "prec must be EMSURF_FP64, EMSURF_FP32 or EMSURF_FP32_IR");
  if (o->prec == EMSURF_FP32_IR) {
    EMS_CHECK_ARG(std::isfinite(o->inner_tol) && o->inner_tol > 0 && o->inner_tol < 1, "inner_tol must be in (0, 1)");
    EMS_CHECK_ARG(o->max_outer >= 1, "max_outer must be >= 1");
  }
  const bool need64 = o->prec != EMSURF_FP32, need32 = o->prec != EMSURF_FP64;
  if ((need64 && !plan->that64.p) || (need32 && !plan->that32.p)) {
    set_error("plan lacks the Fourier-domain store this precision needs");
    throw Err{EMSURF_ERR_UNSUPPORTED};
  }
}

}  // namespace
}  // namespace emsurf

using namespace emsurf;

namespace {

emsurf_status solve_impl(emsurf_plan plan, emsurf_precond pc, const emsurf_solve_opts* opts, int32_t nrhs,
                         const void* b_dev, void* x_dev, emsurf_solve_info* info_host, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  bool all_conv = true;
  std::vector<RhsState> st;
  int outer = 0;
  try {
    check_opts(plan, opts, nrhs);
    EMS_CHECK_ARG(pc == nullptr || precond_plan(pc) == plan, "the preconditioner belongs to another plan");
    EMS_CHECK_ARG(b_dev != nullptr && x_dev != nullptr, "b and x must be non-NULL device pointers");
    EMS_CHECK_ARG(b_dev != x_dev, "b and x must be distinct buffers");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long N = (long long)plan->M * plan->d.n_eq;
    SolveWork* wp = nullptr;
    {
      std::lock_guard<std::mutex> lk(plan->mu);
      auto it = plan->solve_ws.find(s);
      if (it == plan->solve_ws.end()) it = plan->solve_ws.emplace(s, new SolveWork()).first;
      wp = it->second;
    }
    SolveWork& w = *wp;
    w.init(nrhs, opts->restart, N);
    if (pc) w.init_precond();
    // finiteness and norms of b
    int* hm = w.h_mask.as<int>();
    for (int r = 0; r < nrhs; ++r) hm[r] = 1;
    EMS_HIP(hipMemcpyAsync(w.mask.p, hm, (size_t)nrhs * 4, hipMemcpyHostToDevice, s));
    launch_finite(b_dev, N, nrhs, w.mask.as<int>(), s);
    EMS_HIP(hipMemcpyAsync(hm, w.mask.p, (size_t)nrhs * 4, hipMemcpyDeviceToHost, s));
    EMS_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) EMS_CHECK_ARG(hm[r] == 1, "b has a non-finite entry");
    std::vector<double> bn;
    norms(w, b_dev, bn, s);
    st.assign(nrhs, RhsState{});
    if (!opts->use_x0) EMS_HIP(hipMemsetAsync(x_dev, 0, (size_t)nrhs * N * 16, s));
    for (int r = 0; r < nrhs; ++r) {
      st[r].bnorm = bn[r];
      if (bn[r] == 0.0) {
        st[r].done = true;
        st[r].converged = true;
        st[r].rel = 0.0;
        EMS_HIP(hipMemsetAsync(static_cast<double2*>(x_dev) + (size_t)r * N, 0, (size_t)N * 16, s));
      }
    }
    if (opts->prec != EMSURF_FP32_IR) {
      OpFn op = opts->prec == EMSURF_FP64 ? op_fp64 : op_fp32;
      gmres(plan, op, pc, w, nrhs, static_cast<const double2*>(b_dev), static_cast<double2*>(x_dev),
            std::vector<double>(nrhs, opts->tol), opts->max_iter, true, !opts->use_x0, st, s);
      for (int r = 0; r < nrhs; ++r) outer = std::max(outer, st[r].cycles);
    } else {
      // outer refinement: residual in FP64, correction from an FP32 inner solve
      w.init_refinement();
      DevBuf &rr = w.ir_r, &d = w.ir_d, &tt = w.ir_t;
      std::vector<RhsState> inner(nrhs);
      for (outer = 0;; ++outer) {
        for (int r = 0; r < nrhs; ++r) hm[r] = st[r].done ? 0 : 1;
        std::vector<double> rn;
        if (outer == 0 && !opts->use_x0) {
          // x = 0: the residual is b itself, no operator apply needed
          double* hs0 = w.h_scale.as<double>();
          for (int r = 0; r < nrhs; ++r) hs0[r] = hm[r] ? 1.0 : 0.0;
          EMS_HIP(hipMemcpyAsync(w.scale.p, hs0, (size_t)nrhs * 8, hipMemcpyHostToDevice, s));
          launch_scale(b_dev, w.scale.p, rr.p, N, nrhs, s);
          rn.resize(nrhs);
          for (int r = 0; r < nrhs; ++r) rn[r] = hm[r] ? st[r].bnorm : 0.0;
        } else {
          op_fp64(plan, nrhs, x_dev, tt.p, s);
          EMS_HIP(hipMemcpyAsync(w.mask.p, hm, (size_t)nrhs * 4, hipMemcpyHostToDevice, s));
          launch_sub(b_dev, tt.p, w.mask.as<int>(), rr.p, N, nrhs, s);
          norms(w, rr.p, rn, s);
        }
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
          if (st[r].done) continue;
          st[r].rel = rn[r] / st[r].bnorm;
          if (st[r].rel <= opts->tol) { st[r].done = true; st[r].converged = true; }
          else if (outer >= opts->max_outer || st[r].iters >= opts->max_iter) { st[r].done = true; st[r].converged = false; }
          else any = true;
        }
        if (!any) break;
        // each inner solve aims straight at the outer tolerance (half of it, leaving
        // room for the FP32 operator's own error), but never below inner_tol
        std::vector<double> itol(nrhs, 0.5);
        for (int r = 0; r < nrhs; ++r) {
          inner[r] = RhsState{};
          inner[r].bnorm = rn[r];
          if (st[r].done || rn[r] == 0.0) { inner[r].done = true; inner[r].converged = true; continue; }
          itol[r] = std::min(0.5, std::max(opts->inner_tol, 0.5 * opts->tol * st[r].bnorm / rn[r]));
        }
        EMS_HIP(hipMemsetAsync(d.p, 0, (size_t)nrhs * N * 16, s));
        int budget = 0;
        for (int r = 0; r < nrhs; ++r)
          if (!st[r].done) budget = std::max(budget, opts->max_iter - st[r].iters);
        gmres(plan, op_fp32, pc, w, nrhs, rr.as<double2>(), d.as<double2>(), itol, std::max(1, budget), false, true,
              inner, s);
        for (int r = 0; r < nrhs; ++r) st[r].iters += inner[r].iters;
        launch_add(x_dev, d.p, (long long)nrhs * N, s);
      }
    }
    EMS_HIP(hipStreamSynchronize(s));
  } catch (...) {
    return current_exception_status();
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int r = 0; r < nrhs; ++r) {
    all_conv = all_conv && st[r].converged;
    if (info_host) {
      info_host[r].iters = st[r].iters;
      info_host[r].outer_iters = opts->prec == EMSURF_FP32_IR ? outer : st[r].cycles;
      info_host[r].converged = st[r].converged ? 1 : 0;
      info_host[r].rel_res_true = st[r].rel;
      info_host[r].ms = ms;
    }
  }
  if (!all_conv) {
    set_error("solve stopped before reaching tol for at least one right-hand side");
    return EMSURF_ERR_NOT_CONVERGED;
  }
  return EMSURF_OK;
}

}  // namespace

extern "C" emsurf_status emsurf_solve(emsurf_plan plan, const emsurf_solve_opts* opts, int32_t nrhs,
                                      const void* b_dev, void* x_dev, emsurf_solve_info* info_host, void* stream) {
  return solve_impl(plan, nullptr, opts, nrhs, b_dev, x_dev, info_host, stream);
}

extern "C" emsurf_status emsurf_solve_precond(emsurf_plan plan, emsurf_precond pc, const emsurf_solve_opts* opts,
                                              int32_t nrhs, const void* b_dev, void* x_dev,
                                              emsurf_solve_info* info_host, void* stream) {
  if (pc == nullptr) {
    set_error("pc is NULL");
    return EMSURF_ERR_ARG;
  }
  return solve_impl(plan, pc, opts, nrhs, b_dev, x_dev, info_host, stream);
}
