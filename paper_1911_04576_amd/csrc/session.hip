// Continuous batching of GMRES solves on one plan (serving).
//
// A session owns `max_slots` right-hand-side slots.  Each slot runs its own
// restarted GMRES instance (same algorithm as emsurf_solve, Sec. IV-A reading:
// CGS2, complex Givens, true-residual check at the end of every cycle), but
// the instances are not in lockstep: a slot joins at any step, runs at its own
// Arnoldi index and leaves when done.  One step gathers the operand vector of
// every slot that needs an operator apply, runs one batched apply (one for
// the FP64 operator and one for the FP32 operator in the refinement mode),
// scatters the results back and performs each slot's orthogonalisation with
// pointer-list kernels.  A slot's arithmetic is independent of its batch-mates
// (per-column FFTs and products, the FP32 product variant fixed per session,
// per-slot reductions), so a result is bitwise the same alone and in a mix.
//
// Modes: EMSURF_FP64 (FP64 operator throughout), EMSURF_FP32 (FP32 operator,
// FP64 basis), EMSURF_FP32_IR (Arnoldi with the FP32 operator, the residual at
// every cycle start with the FP64 operator; a cycle aims at
// max(inner_tol * beta, tol * ||b|| / 2), i.e. GMRES-IR with one cycle per
// refinement step).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"
#include "vecops.h"
#include "session.h"

namespace emsurf {
namespace {

using cd = std::complex<double>;

void givens(cd a, cd b, double& c, cd& s) {
  if (b == 0.0) { c = 1.0; s = 0.0; return; }
  if (a == 0.0) { c = 0.0; s = std::conj(b) / std::abs(b); return; }
  const double r = std::hypot(std::abs(a), std::abs(b));
  c = std::abs(a) / r;
  s = (a / std::abs(a)) * std::conj(b) / r;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace emsurf

using namespace emsurf;

emsurf_session_s::~emsurf_session_s() {
  if (stream) {
    (void)hipStreamSynchronize(stream);
    if (own_stream) (void)hipStreamDestroy(stream);
  }
  if (ev) (void)hipEventDestroy(ev);
}

namespace emsurf {

size_t session_fixed_bytes(const emsurf_plan_desc& d, int max_slots, int restart) {
  const size_t N = (size_t)d.nx * d.ny * d.n_eq;
  const size_t staging = 2 * (size_t)max_slots * N * 16;   // gathered operands, apply outputs
  const int nblk = dot_blocks((long long)N);
  const size_t red = (size_t)max_slots * (2 * (restart + 2) + 8) * 16 * 2;
  const size_t partial = (size_t)max_slots * nblk * (restart + 2) * 16;
  const size_t coef = (size_t)max_slots * restart * 16;
  return staging + red + partial + coef + (size_t)16 * max_slots * sizeof(VecItem);
}

size_t session_slot_bytes(const emsurf_plan_desc& d, int restart) {
  const size_t N = (size_t)d.nx * d.ny * d.n_eq;
  return (size_t)(restart + 4) * N * 16;
}

size_t session_bytes(const emsurf_plan_desc& d, int max_slots, int restart) {
  // a stream without an apply workspace in the plan gets one
  const int64_t Lx = fft_length_at_least(2 * d.nx - 1);
  const int64_t Ly = fft_length_at_least(2 * d.ny - 1);
  const int64_t B = (int64_t)d.max_rhs * d.n_eq;
  const size_t ws = (size_t)(d.ny * Lx * B) * 16 + 2 * (size_t)(Lx * Ly * B) * 16 + (size_t)(B * d.nx * d.ny) * 16;
  return session_fixed_bytes(d, max_slots, restart) + (size_t)max_slots * session_slot_bytes(d, restart) + ws;
}

size_t session_held_bytes(emsurf_session ss) {
  size_t b = 0;
  for (auto& m : ss->mem) b += m.bytes;
  return b;
}

int session_free_held(emsurf_session ss) {
  int c = 0;
  for (int s = 0; s < ss->S; ++s) c += ss->slot[s].ph == SessionSlot::FREE && ss->mem[s].p != nullptr;
  return c;
}

size_t session_trim(emsurf_session ss) {
  size_t freed = 0;
  for (int s = 0; s < ss->S; ++s)
    if (ss->slot[s].ph == SessionSlot::FREE && ss->mem[s].p) {
      freed += ss->mem[s].bytes;
      ss->mem[s].release();
    }
  return freed;
}

void session_init(emsurf_session ss, emsurf_plan plan, int max_slots, const emsurf_solve_opts& o, hipStream_t s,
                  bool own) {
  ss->plan = plan;
  ss->opts = o;
  ss->S = max_slots;
  ss->m = o.restart;
  ss->N = (long long)plan->M * plan->d.n_eq;
  ss->stream = s;
  ss->own_stream = own;
  const size_t vb = (size_t)ss->N * 16;
  // slot vectors and Krylov bases are allocated per slot at its first submit
  ss->mem.clear();
  ss->mem.resize(ss->S);
  ss->xin.alloc(vb * ss->S);
  ss->wout.alloc(vb * ss->S);
  ss->nblk = dot_blocks(ss->N);
  ss->ns = ss->m + 2;
  ss->rstride = 2 * (ss->m + 2) + 8;
  ss->partial.alloc((size_t)ss->S * ss->nblk * ss->ns * 16);
  ss->red.alloc((size_t)2 * ss->S * ss->rstride * 16);
  ss->h_red.alloc(ss->red.bytes);
  ss->coef.alloc((size_t)ss->S * ss->m * 16);
  ss->h_coef.alloc(ss->coef.bytes);
  ss->items.alloc((size_t)16 * ss->S * sizeof(VecItem));
  ss->h_items.alloc(ss->items.bytes);
  ss->slot.assign(ss->S, SessionSlot{});
  EMS_HIP(hipEventCreateWithFlags(&ss->ev, hipEventDisableTiming));
  // the FP32 product variant is fixed for the session's lifetime
  ss->variant32 = choose_variant(plan, std::min(ss->S, plan->d.max_rhs));
  (void)workspace(plan, s);
  EMS_HIP(hipStreamSynchronize(s));
}

namespace {

// List regions in the item buffers: launch lists 0..7, finish lists 8..15
VecItem* hitem(emsurf_session ss, int list) { return ss->h_items.as<VecItem>() + (size_t)list * ss->S; }
const VecItem* ditem(emsurf_session ss, int list) { return ss->items.as<VecItem>() + (size_t)list * ss->S; }

void push_items(emsurf_session ss, int list, int count) {
  if (count <= 0) return;
  EMS_HIP(hipMemcpyAsync(const_cast<VecItem*>(ditem(ss, list)), hitem(ss, list), (size_t)count * sizeof(VecItem),
                         hipMemcpyHostToDevice, ss->stream));
}

double2* vec(const DevBuf& buf, long long N, int s) { return buf.as<double2>() + (size_t)s * N; }
// vectors of slot s: right-hand side, iterate, residual, Krylov basis
double2* sb(emsurf_session ss, int s) { return ss->mem[s].as<double2>(); }
double2* sx(emsurf_session ss, int s) { return ss->mem[s].as<double2>() + ss->N; }
double2* sr(emsurf_session ss, int s) { return ss->mem[s].as<double2>() + 2 * ss->N; }
double2* basis(emsurf_session ss, int s, int l) { return ss->mem[s].as<double2>() + (size_t)(3 + l) * ss->N; }

Cx arnoldi_type(const emsurf_solve_opts& o) { return o.prec == EMSURF_FP64 ? Cx::C128 : Cx::C64; }
Cx resid_type(const emsurf_solve_opts& o) { return o.prec == EMSURF_FP32 ? Cx::C64 : Cx::C128; }

// one batched operator apply over `group` (slot, kind) entries; kind 0: residual
// r = b - A x, kind 1: Arnoldi w = A v_j
void batched_apply(emsurf_session ss, const std::vector<std::pair<int, int>>& group, Cx tc, int list_g, int list_s) {
  const int nq = (int)group.size();
  if (nq == 0) return;
  const long long N = ss->N;
  VecItem* g = hitem(ss, list_g);
  VecItem* sc = hitem(ss, list_s);
  for (int q = 0; q < nq; ++q) {
    const int s = group[q].first;
    const bool res = group[q].second == 0;
    g[q] = VecItem{res ? (const void*)sx(ss, s) : (const void*)basis(ss, s, ss->slot[s].j), nullptr,
                   vec(ss->xin, N, q), 1.0, 0, 0};
    sc[q] = res ? VecItem{vec(ss->wout, N, q), sb(ss, s), sr(ss, s), 1.0, 0, 0}
                : VecItem{vec(ss->wout, N, q), nullptr, basis(ss, s, ss->slot[s].j + 1), 1.0, 0, 0};
  }
  push_items(ss, list_g, nq);
  push_items(ss, list_s, nq);
  launch_copy_list(ditem(ss, list_g), nq, N, ss->stream);
  apply_A_typed(ss->plan, Cx::C128, tc, Cx::C128, nq, ss->xin.p, ss->wout.p, ss->stream,
                tc == Cx::C64 ? ss->variant32 : -1);
  launch_copy_list(ditem(ss, list_s), nq, N, ss->stream);
}

}  // namespace

// Launch one step's device work (no host wait).
void session_launch(emsurf_session ss) {
  const long long N = ss->N;
  ss->q_norm.clear();
  ss->q_arn.clear();
  std::vector<std::pair<int, int>> g64, g32;
  std::vector<int> init;
  for (int s = 0; s < ss->S; ++s) {
    SessionSlot& q = ss->slot[s];
    if (q.ph == SessionSlot::INIT) {
      init.push_back(s);
    } else if (q.ph == SessionSlot::RESID) {
      (resid_type(ss->opts) == Cx::C128 ? g64 : g32).push_back({s, 0});
    } else if (q.ph == SessionSlot::ARNOLDI) {
      (arnoldi_type(ss->opts) == Cx::C128 ? g64 : g32).push_back({s, 1});
    }
  }
  ss->launched = !(init.empty() && g64.empty() && g32.empty());
  if (!ss->launched) return;
  // r = b for new slots (x = 0)
  if (!init.empty()) {
    VecItem* it = hitem(ss, 0);
    for (size_t i = 0; i < init.size(); ++i)
      it[i] = VecItem{sb(ss, init[i]), nullptr, sr(ss, init[i]), 1.0, 0, 0};
    push_items(ss, 0, (int)init.size());
    launch_copy_list(ditem(ss, 0), (int)init.size(), N, ss->stream);
  }
  batched_apply(ss, g64, Cx::C128, 1, 2);
  batched_apply(ss, g32, Cx::C64, 3, 4);
  // residual norms: INIT and RESID slots
  for (int s : init) ss->q_norm.push_back(s);
  for (auto& e : g64) if (e.second == 0) ss->q_norm.push_back(e.first);
  for (auto& e : g32) if (e.second == 0) ss->q_norm.push_back(e.first);
  for (auto& e : g64) if (e.second == 1) ss->q_arn.push_back(e.first);
  for (auto& e : g32) if (e.second == 1) ss->q_arn.push_back(e.first);
  const int nn = (int)ss->q_norm.size(), na = (int)ss->q_arn.size();
  double2* red = ss->red.as<double2>();
  if (nn > 0) {
    VecItem* it = hitem(ss, 5);
    for (int i = 0; i < nn; ++i) it[i] = VecItem{nullptr, nullptr, sr(ss, ss->q_norm[i]), 1.0, 0, 0};
    push_items(ss, 5, nn);
    launch_dot_list(ditem(ss, 5), nn, 1, N, ss->partial.p, ss->nblk, red, ss->rstride, 0, ss->stream);
  }
  if (na > 0) {
    // CGS2 per slot; rows of the reduction buffer after the norm rows
    VecItem* it = hitem(ss, 6);
    int nvmax = 0;
    for (int i = 0; i < na; ++i) {
      const int s = ss->q_arn[i];
      const int nv = ss->slot[s].j + 1;
      nvmax = std::max(nvmax, nv);
      it[i] = VecItem{basis(ss, s, 0), nullptr, basis(ss, s, nv), 1.0, nv, 0};
    }
    push_items(ss, 6, na);
    double2* ra = red + (size_t)nn * ss->rstride;
    const int ns = nvmax + 1;
    const int o1 = 0, o2 = ss->m + 2, o3 = 2 * (ss->m + 2);
    launch_dot_list(ditem(ss, 6), na, ns, N, ss->partial.p, ss->nblk, ra, ss->rstride, o1, ss->stream);
    launch_update_list(ditem(ss, 6), na, N, ra, ss->rstride, o1, ss->stream);
    launch_dot_list(ditem(ss, 6), na, ns, N, ss->partial.p, ss->nblk, ra, ss->rstride, o2, ss->stream);
    launch_update_list(ditem(ss, 6), na, N, ra, ss->rstride, o2, ss->stream);
    // final norm: items with nv = 0 on the same w
    VecItem* it2 = hitem(ss, 7);
    for (int i = 0; i < na; ++i) it2[i] = VecItem{nullptr, nullptr, it[i].dst, 1.0, 0, 0};
    push_items(ss, 7, na);
    launch_dot_list(ditem(ss, 7), na, 1, N, ss->partial.p, ss->nblk, ra, ss->rstride, o3, ss->stream);
  }
  EMS_HIP(hipMemcpyAsync(ss->h_red.p, ss->red.p, (size_t)(nn + na) * ss->rstride * 16, hipMemcpyDeviceToHost,
                         ss->stream));
  EMS_HIP(hipEventRecord(ss->ev, ss->stream));
}

// Wait for the step, update every slot on the host and launch the basis
// scalings and solution updates.  Returns the number of slots that finished.
int session_finish(emsurf_session ss) {
  if (!ss->launched) return 0;
  EMS_HIP(hipEventSynchronize(ss->ev));
  const long long N = ss->N;
  const int m = ss->m;
  const emsurf_solve_opts& o = ss->opts;
  const double2* hr = ss->h_red.as<double2>();
  const int nn = (int)ss->q_norm.size(), na = (int)ss->q_arn.size();
  VecItem* scl = hitem(ss, 8);
  VecItem* axp = hitem(ss, 9);
  int nscl = 0, naxp = 0, finished = 0;
  cd* hy = reinterpret_cast<cd*>(ss->h_coef.p);
  auto end_cycle = [&](int s) {
    SessionSlot& q = ss->slot[s];
    const int k = q.kend;
    cd* y = hy + (size_t)s * m;
    for (int i = k - 1; i >= 0; --i) {
      cd acc = q.g[i];
      for (int l = i + 1; l < k; ++l) acc -= q.H[(size_t)l * (m + 1) + i] * y[l];
      y[i] = acc / q.H[(size_t)i * (m + 1) + i];
    }
    axp[naxp++] = VecItem{basis(ss, s, 0), reinterpret_cast<const double2*>(ss->coef.p) + (size_t)s * m,
                          sx(ss, s), 1.0, k, 0};
    q.cycles += 1;
    q.ph = SessionSlot::RESID;
  };
  // residual results
  for (int i = 0; i < nn; ++i) {
    const int s = ss->q_norm[i];
    SessionSlot& q = ss->slot[s];
    const double beta = std::sqrt(hr[(size_t)i * ss->rstride].x);
    if (q.ph == SessionSlot::INIT) {
      q.bnorm = beta;
      if (!std::isfinite(beta)) {
        q.ph = SessionSlot::DONE; q.converged = false; q.bad = true; q.rel = NAN;
        q.t_done = now_ms(); ++finished;
        continue;
      }
      if (beta == 0.0) {
        q.ph = SessionSlot::DONE; q.converged = true; q.rel = 0.0;
        q.t_done = now_ms(); ++finished;
        continue;
      }
    }
    q.rel = beta / q.bnorm;
    if (q.rel <= o.tol || q.iters >= o.max_iter) {
      q.ph = SessionSlot::DONE;
      q.converged = q.rel <= o.tol;
      q.t_done = now_ms();
      ++finished;
      continue;
    }
    // start a cycle: v0 = r / beta
    q.ph = SessionSlot::ARNOLDI;
    q.j = 0;
    q.beta = beta;
    q.target = o.prec == EMSURF_FP32_IR ? std::max(o.inner_tol * beta, 0.5 * o.tol * q.bnorm) : o.tol * q.bnorm;
    q.H.assign((size_t)(m + 1) * m, cd(0));
    q.cs.assign(m, 0.0);
    q.sn.assign(m, cd(0));
    q.g.assign(m + 1, cd(0));
    q.g[0] = beta;
    scl[nscl++] = VecItem{sr(ss, s), nullptr, basis(ss, s, 0), 1.0 / beta, 0, 0};
  }
  // Arnoldi results
  const double2* ha = hr + (size_t)nn * ss->rstride;
  const int o1 = 0, o2 = m + 2, o3 = 2 * (m + 2);
  for (int i = 0; i < na; ++i) {
    const int s = ss->q_arn[i];
    SessionSlot& q = ss->slot[s];
    const double2* R = ha + (size_t)i * ss->rstride;
    const int j = q.j, nv = j + 1;
    cd* Hc = &q.H[(size_t)j * (m + 1)];
    for (int l = 0; l <= j; ++l) Hc[l] = cd(R[o1 + l].x, R[o1 + l].y) + cd(R[o2 + l].x, R[o2 + l].y);
    const double wn0 = std::sqrt(R[o1 + nv].x);
    const double hn = std::sqrt(R[o3].x);
    Hc[j + 1] = hn;
    for (int l = 0; l < j; ++l) {
      const cd t = q.cs[l] * Hc[l] + q.sn[l] * Hc[l + 1];
      Hc[l + 1] = -std::conj(q.sn[l]) * Hc[l] + q.cs[l] * Hc[l + 1];
      Hc[l] = t;
    }
    givens(Hc[j], Hc[j + 1], q.cs[j], q.sn[j]);
    Hc[j] = q.cs[j] * Hc[j] + q.sn[j] * Hc[j + 1];
    Hc[j + 1] = 0.0;
    q.g[j + 1] = -std::conj(q.sn[j]) * q.g[j];
    q.g[j] = q.cs[j] * q.g[j];
    q.iters += 1;
    const double est = std::abs(q.g[j + 1]);
    const bool lucky = hn <= 1e-14 * wn0;
    if (est <= q.target || lucky || q.iters >= o.max_iter || j == m - 1) {
      q.kend = j + 1;
      end_cycle(s);
    } else {
      scl[nscl++] = VecItem{basis(ss, s, j + 1), nullptr, basis(ss, s, j + 1), 1.0 / hn, 0, 0};
      q.j = j + 1;
    }
  }
  if (naxp > 0) {
    EMS_HIP(hipMemcpyAsync(ss->coef.p, ss->h_coef.p, ss->coef.bytes, hipMemcpyHostToDevice, ss->stream));
    push_items(ss, 9, naxp);
    launch_axpy_list(ditem(ss, 9), naxp, N, ss->stream);
  }
  if (nscl > 0) {
    push_items(ss, 8, nscl);
    launch_copy_list(ditem(ss, 8), nscl, N, ss->stream);
  }
  ss->launched = false;
  return finished;
}

}  // namespace emsurf

namespace {

template <typename F>
emsurf_status sguard(F&& f) {
  return guarded_call(std::forward<F>(f));
}

void check_session_opts(emsurf_plan plan, const emsurf_solve_opts* o, int max_slots) {
  EMS_CHECK_ARG(plan != nullptr && o != nullptr, "plan and opts must be non-NULL");
  EMS_CHECK_ARG(max_slots >= 1 && max_slots <= plan->d.max_rhs, "max_slots must be in [1, plan max_rhs]");
  EMS_CHECK_ARG(std::isfinite(o->tol) && o->tol > 0, "tol must be > 0");
  EMS_CHECK_ARG(o->restart >= 1 && o->restart <= 64, "restart must be in [1, 64]");
  EMS_CHECK_ARG(o->max_iter >= 1, "max_iter must be >= 1");
  EMS_CHECK_ARG(o->prec == EMSURF_FP64 || o->prec == EMSURF_FP32 || o->prec == EMSURF_FP32_IR, "bad prec");
  if (o->prec == EMSURF_FP32_IR)
    EMS_CHECK_ARG(std::isfinite(o->inner_tol) && o->inner_tol > 0 && o->inner_tol < 1, "inner_tol must be in (0, 1)");
  const bool need64 = o->prec != EMSURF_FP32, need32 = o->prec != EMSURF_FP64;
  if ((need64 && !plan->that64.p) || (need32 && !plan->that32.p)) {
    set_error("plan lacks the Fourier-domain store this precision needs");
    throw Err{EMSURF_ERR_UNSUPPORTED};
  }
}

}  // namespace

extern "C" {

size_t emsurf_session_bytes(emsurf_plan plan, int32_t max_slots, const emsurf_solve_opts* opts) {
  if (!plan || !opts || max_slots < 1 || opts->restart < 1) return 0;
  return session_bytes(plan->d, max_slots, opts->restart);
}

emsurf_status emsurf_session_create(emsurf_plan plan, int32_t max_slots, const emsurf_solve_opts* opts, void* stream,
                                    emsurf_session* out) {
  emsurf_session ss = nullptr;
  emsurf_status st = sguard([&] {
    EMS_CHECK_ARG(out != nullptr, "out is NULL");
    check_session_opts(plan, opts, max_slots);
    ss = new emsurf_session_s();
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool own = false;
    if (!s) {
      EMS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      own = true;
    }
    ss->stream = s;
    ss->own_stream = own;
    session_init(ss, plan, max_slots, *opts, s, own);
  });
  if (st != EMSURF_OK) {
    delete ss;
    return st;
  }
  *out = ss;
  return EMSURF_OK;
}

emsurf_status emsurf_session_submit(emsurf_session ss, const void* b_dev, int64_t tag, int32_t* slot) {
  return sguard([&] {
    EMS_CHECK_ARG(ss != nullptr && b_dev != nullptr, "session and b must be non-NULL");
    // a free slot that already holds its vectors first, else any free slot
    int s = -1;
    for (int i = 0; i < ss->S && s < 0; ++i)
      if (ss->slot[i].ph == SessionSlot::FREE && ss->mem[i].p) s = i;
    for (int i = 0; i < ss->S && s < 0; ++i)
      if (ss->slot[i].ph == SessionSlot::FREE) s = i;
    if (s < 0) {
      set_error("no free slot");
      throw Err{EMSURF_ERR_BUSY};
    }
    if (!ss->mem[s].p) ss->mem[s].alloc((size_t)(ss->m + 4) * ss->N * 16);
    EMS_HIP(hipMemcpyAsync(sb(ss, s), b_dev, (size_t)ss->N * 16, hipMemcpyDeviceToDevice, ss->stream));
    EMS_HIP(hipMemsetAsync(sx(ss, s), 0, (size_t)ss->N * 16, ss->stream));
    SessionSlot q;
    q.ph = SessionSlot::INIT;
    q.tag = tag;
    q.t_submit = now_ms();
    ss->slot[s] = q;
    if (slot) *slot = s;
  });
}

emsurf_status emsurf_session_step(emsurf_session ss, int32_t* n_finished) {
  return sguard([&] {
    EMS_CHECK_ARG(ss != nullptr, "session is NULL");
    session_launch(ss);
    const int f = session_finish(ss);
    if (n_finished) *n_finished = f;
  });
}

emsurf_status emsurf_session_finished(emsurf_session ss, int32_t* slots, int64_t* tags, int32_t cap,
                                      int32_t* count) {
  return sguard([&] {
    EMS_CHECK_ARG(ss != nullptr && count != nullptr, "session and count must be non-NULL");
    int c = 0;
    for (int s = 0; s < ss->S; ++s)
      if (ss->slot[s].ph == SessionSlot::DONE) {
        if (c < cap) {
          if (slots) slots[c] = s;
          if (tags) tags[c] = ss->slot[s].tag;
        }
        ++c;
      }
    *count = c;
  });
}

emsurf_status emsurf_session_active(emsurf_session ss, int32_t* busy_slots) {
  return sguard([&] {
    EMS_CHECK_ARG(ss != nullptr && busy_slots != nullptr, "session and busy_slots must be non-NULL");
    int c = 0;
    for (auto& q : ss->slot) c += q.ph != SessionSlot::FREE;
    *busy_slots = c;
  });
}

emsurf_status emsurf_session_collect(emsurf_session ss, int32_t slot, void* x_dev, emsurf_solve_info* info) {
  return sguard([&] {
    EMS_CHECK_ARG(ss != nullptr, "session is NULL");
    EMS_CHECK_ARG(slot >= 0 && slot < ss->S, "slot out of range");
    SessionSlot& q = ss->slot[slot];
    EMS_CHECK_ARG(q.ph == SessionSlot::DONE, "slot has not finished");
    if (x_dev) {
      EMS_HIP(hipMemcpyAsync(x_dev, sx(ss, slot), (size_t)ss->N * 16, hipMemcpyDeviceToDevice, ss->stream));
      EMS_HIP(hipStreamSynchronize(ss->stream));
    }
    if (info) {
      info->iters = q.iters;
      info->outer_iters = q.cycles;
      info->converged = q.converged ? 1 : 0;
      info->rel_res_true = q.rel;
      info->ms = q.t_done - q.t_submit;
    }
    const bool bad = q.bad;
    q = SessionSlot{};
    if (bad) {
      set_error("right-hand side had a non-finite entry");
      throw Err{EMSURF_ERR_ARG};
    }
  });
}

void emsurf_session_destroy(emsurf_session ss) { delete ss; }

}  // extern "C"
