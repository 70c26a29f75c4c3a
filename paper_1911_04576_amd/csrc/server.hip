// Serving loop: requests for different surfaces (lattice, n_eq, macromodels)
// arrive at any time; each surface's plan (its Fourier-domain blocks) stays
// resident in HBM and is shared by every request on that surface; requests
// are admitted when their plan fits the HBM budget (idle plans are evicted
// least-recently-used first) and their session has free slots; every step
// runs one batched GMRES iteration on every busy session, each session on its
// own stream so that work on different plans overlaps on the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "internal.h"
#include "session.h"

namespace emsurf {
namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  uint64_t key = 0;
  emsurf_plan_desc desc{};
  std::vector<double> rho, area, tan;
  double pitch = 0, k = 0;
  std::vector<double> S;        // interleaved complex
  std::vector<int32_t> types;
  int nrhs = 0;
  std::vector<double> b;        // interleaved complex [nrhs][N]
  enum { QUEUED, ACTIVE, DONE } state = QUEUED;
  std::vector<int> slots;
  std::vector<double> x;        // result [nrhs][N]
  std::vector<emsurf_solve_info> info;
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool bad = false;
};

struct PlanEntry {
  emsurf_plan plan = nullptr;
  emsurf_session session = nullptr;
  hipStream_t stream = nullptr;
  size_t bytes = 0;        // plan, session staging and reductions, host staging vector
  size_t slot_bytes = 0;   // vectors and Krylov basis of one slot
  size_t held = 0;         // slot buffers the session holds now
  double last_used = 0;
  int active = 0;
  DevBuf staging;   // one right-hand side, for host -> slot copies
};

}  // namespace
}  // namespace emsurf

struct emsurf_server_s {
  emsurf_server_desc d{};
  std::map<uint64_t, std::unique_ptr<emsurf::PlanEntry>> plans;
  std::deque<std::unique_ptr<emsurf::Request>> queue;
  std::map<int64_t, std::unique_ptr<emsurf::Request>> active, done;
  std::deque<int64_t> completed;
  int64_t next_id = 1;
  size_t used = 0;
  int64_t evictions = 0, plans_built = 0;
  double admit_ms = 0, step_ms = 0;
  ~emsurf_server_s() {
    for (auto& kv : plans) {
      if (kv.second->session) emsurf_session_destroy(kv.second->session);
      if (kv.second->plan) emsurf_plan_destroy(kv.second->plan);
      if (kv.second->stream) (void)hipStreamDestroy(kv.second->stream);
    }
  }
};

using namespace emsurf;

namespace {

void destroy_entry(emsurf_server sv, std::map<uint64_t, std::unique_ptr<PlanEntry>>::iterator it) {
  PlanEntry& e = *it->second;
  if (e.session) emsurf_session_destroy(e.session);
  if (e.plan) emsurf_plan_destroy(e.plan);
  if (e.stream) (void)hipStreamDestroy(e.stream);
  sv->used -= e.bytes + e.held;
  sv->plans.erase(it);
}

emsurf_plan_desc server_desc(emsurf_server sv, emsurf_plan_desc pd) {
  pd.max_rhs = sv->d.max_slots;
  pd.store = sv->d.store;
  return pd;
}

// Device bytes a resident surface holds with no busy right-hand side: the plan
// (its stores and the apply workspace of its stream, which the session on the
// same stream shares), the session's batch staging and reductions, and one
// staging vector.  Each busy slot adds entry_slot_bytes.
size_t entry_bytes(emsurf_server sv, emsurf_plan_desc pd) {
  pd = server_desc(sv, pd);
  const size_t pb = emsurf_plan_bytes(&pd);
  if (pb == 0) return 0;
  return pb + session_fixed_bytes(pd, sv->d.max_slots, sv->d.opts.restart) + (size_t)pd.nx * pd.ny * pd.n_eq * 16;
}

size_t entry_slot_bytes(emsurf_server sv, emsurf_plan_desc pd) {
  return session_slot_bytes(server_desc(sv, pd), sv->d.opts.restart);
}

// Account for the slot buffers the entry's session holds now.
void refresh_held(emsurf_server sv, PlanEntry& e) {
  const size_t h = session_held_bytes(e.session);
  sv->used = sv->used - e.held + h;
  e.held = h;
}

// Make room for `need` more bytes: first release the buffers of free slots
// (cheap to allocate again), then evict idle plans (neither active nor queued,
// least recently used first).  Nothing is released unless the need can be met.
bool make_room(emsurf_server sv, size_t need, const std::map<uint64_t, int>& protect) {
  const size_t budget = sv->d.budget_bytes;
  if (sv->used + need <= budget) return true;
  auto idle = [&](const PlanEntry& e, uint64_t key) { return e.active == 0 && protect.count(key) == 0; };
  size_t releasable = 0;
  for (auto& kv : sv->plans) {
    PlanEntry& e = *kv.second;
    releasable += idle(e, kv.first) ? e.bytes + e.held
                                    : (size_t)session_free_held(e.session) * e.slot_bytes;
  }
  if (sv->used - releasable + need > budget) return false;   // wait; release nothing
  for (auto& kv : sv->plans) {
    if (sv->used + need <= budget) return true;
    (void)session_trim(kv.second->session);
    refresh_held(sv, *kv.second);
  }
  while (sv->used + need > budget) {
    auto victim = sv->plans.end();
    for (auto p = sv->plans.begin(); p != sv->plans.end(); ++p)
      if (idle(*p->second, p->first) &&
          (victim == sv->plans.end() || p->second->last_used < victim->second->last_used))
        victim = p;
    if (victim == sv->plans.end()) return false;
    destroy_entry(sv, victim);
    ++sv->evictions;
  }
  return true;
}

// Make the plan of request rq resident (building it if needed) with room for
// the request's slots.  Returns null when it does not fit the budget yet.
PlanEntry* resident(emsurf_server sv, Request& rq, const std::map<uint64_t, int>& queued_keys) {
  auto it = sv->plans.find(rq.key);
  if (it != sv->plans.end()) return it->second.get();
  const emsurf_plan_desc pd = server_desc(sv, rq.desc);
  const size_t fixed = entry_bytes(sv, pd);
  const size_t slot = entry_slot_bytes(sv, pd);
  const size_t need = fixed + (size_t)rq.nrhs * slot;
  if (fixed == 0 || need > sv->d.budget_bytes) {   // invalid, or can never be admitted
    rq.bad = true;
    return nullptr;
  }
  if (!make_room(sv, need, queued_keys)) return nullptr;
  auto e = std::make_unique<PlanEntry>();
  EMS_HIP(hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking));
  emsurf_geom g{(int32_t)rq.area.size(), rq.rho.data(), rq.area.data(), rq.tan.data(), rq.pitch, rq.k};
  emsurf_status st = emsurf_plan_create_green(&pd, &g, rq.S.data(), rq.types.data(), e->stream, &e->plan);
  if (st != EMSURF_OK) {
    (void)hipStreamDestroy(e->stream);
    throw Err{st};
  }
  st = emsurf_session_create(e->plan, sv->d.max_slots, &sv->d.opts, e->stream, &e->session);
  if (st != EMSURF_OK) {
    emsurf_plan_destroy(e->plan);
    (void)hipStreamDestroy(e->stream);
    throw Err{st};
  }
  e->staging.alloc((size_t)pd.nx * pd.ny * pd.n_eq * 16);
  e->bytes = fixed;
  e->slot_bytes = slot;
  e->last_used = now_ms();
  sv->used += fixed;
  ++sv->plans_built;
  PlanEntry* raw = e.get();
  sv->plans[rq.key] = std::move(e);
  return raw;
}

int free_slots(emsurf_session ss) {
  int c = 0;
  for (auto& q : ss->slot) c += q.ph == SessionSlot::FREE;
  return c;
}

void place(emsurf_server sv, Request& rq, PlanEntry* e) {
  const size_t N = (size_t)rq.desc.nx * rq.desc.ny * rq.desc.n_eq;
  rq.slots.resize(rq.nrhs);
  for (int r = 0; r < rq.nrhs; ++r) {
    EMS_HIP(hipMemcpyAsync(e->staging.p, rq.b.data() + 2 * N * r, N * 16, hipMemcpyHostToDevice, e->stream));
    int32_t slot = -1;
    emsurf_status st = emsurf_session_submit(e->session, e->staging.p, rq.id, &slot);
    if (st != EMSURF_OK) throw Err{st};
    rq.slots[r] = slot;
  }
  EMS_HIP(hipStreamSynchronize(e->stream));
  refresh_held(sv, *e);
  e->active += 1;
  e->last_used = now_ms();
  rq.state = Request::ACTIVE;
  rq.t_admit = now_ms();
  rq.b.clear();
  rq.b.shrink_to_fit();
}

// Admission: first every queued request whose plan is resident and has free
// slots (in arrival order); then, for the oldest waiting requests whose plan is
// not resident, build plans as long as they fit after evicting idle plans.
void admit(emsurf_server sv) {
  auto take = [&](std::deque<std::unique_ptr<Request>>::iterator it) {
    const int64_t id = (*it)->id;
    sv->active[id] = std::move(*it);
    return sv->queue.erase(it);
  };
  std::map<uint64_t, int> queued_keys;
  for (auto& q : sv->queue) queued_keys[q->key] += 1;
  for (auto it = sv->queue.begin(); it != sv->queue.end();) {
    Request& rq = **it;
    auto pe = sv->plans.find(rq.key);
    bool placed = false;
    if (pe != sv->plans.end() && free_slots(pe->second->session) >= rq.nrhs) {
      PlanEntry& e = *pe->second;
      const int fresh = std::max(0, rq.nrhs - session_free_held(e.session));
      if (make_room(sv, (size_t)fresh * e.slot_bytes, queued_keys)) {
        place(sv, rq, &e);
        placed = true;
      }
    }
    if (placed) {
      if (--queued_keys[rq.key] == 0) queued_keys.erase(rq.key);
      it = take(it);
    } else {
      ++it;
    }
  }
  for (auto it = sv->queue.begin(); it != sv->queue.end();) {
    Request& rq = **it;
    if (sv->plans.count(rq.key)) { ++it; continue; }
    // the request's own key does not protect plans from eviction, other queued keys do
    auto mine = queued_keys.find(rq.key);
    std::map<uint64_t, int> others = queued_keys;
    others.erase(rq.key);
    (void)mine;
    PlanEntry* e = resident(sv, rq, others);
    if (rq.bad) {
      rq.state = Request::DONE;
      rq.t_done = now_ms();
      sv->completed.push_back(rq.id);
      const int64_t id = rq.id;
      sv->done[id] = std::move(*it);
      it = sv->queue.erase(it);
      continue;
    }
    if (e && free_slots(e->session) >= rq.nrhs) {
      place(sv, rq, e);
      if (--queued_keys[rq.key] == 0) queued_keys.erase(rq.key);
      it = take(it);
      continue;
    }
    ++it;
  }
}

void harvest(emsurf_server sv) {
  std::vector<int64_t> finished;
  for (auto& kv : sv->active) {
    Request& rq = *kv.second;
    PlanEntry& e = *sv->plans.at(rq.key);
    bool all = true;
    for (int s : rq.slots) all = all && e.session->slot[s].ph == SessionSlot::DONE;
    if (!all) continue;
    const size_t N = (size_t)rq.desc.nx * rq.desc.ny * rq.desc.n_eq;
    rq.x.assign(2 * N * rq.nrhs, 0.0);
    rq.info.resize(rq.nrhs);
    for (int r = 0; r < rq.nrhs; ++r) {
      emsurf_status st = emsurf_session_collect(e.session, rq.slots[r], e.staging.p, &rq.info[r]);
      if (st == EMSURF_ERR_ARG) rq.bad = true;
      else if (st != EMSURF_OK) throw Err{st};
      EMS_HIP(hipMemcpy(rq.x.data() + 2 * N * r, e.staging.p, N * 16, hipMemcpyDeviceToHost));
    }
    e.active -= 1;
    e.last_used = now_ms();
    rq.state = Request::DONE;
    rq.t_done = now_ms();
    finished.push_back(kv.first);
  }
  for (int64_t id : finished) {
    sv->done[id] = std::move(sv->active[id]);
    sv->active.erase(id);
    sv->completed.push_back(id);
  }
}

template <typename F>
emsurf_status vguard(F&& f) {
  return guarded_call(std::forward<F>(f));
}

}  // namespace

extern "C" {

emsurf_status emsurf_server_create(const emsurf_server_desc* desc, emsurf_server* out) {
  return vguard([&] {
    EMS_CHECK_ARG(desc != nullptr && out != nullptr, "desc and out must be non-NULL");
    EMS_CHECK_ARG(desc->budget_bytes > 0, "budget must be > 0");
    EMS_CHECK_ARG(desc->max_slots >= 1 && desc->max_slots <= 64, "max_slots must be in [1, 64]");
    EMS_CHECK_ARG(desc->opts.restart >= 1 && desc->opts.restart <= 64 && desc->opts.tol > 0, "bad solve options");
    EMS_CHECK_ARG(desc->store != 0, "store must be non-zero");
    auto* sv = new emsurf_server_s();
    sv->d = *desc;
    *out = sv;
  });
}

emsurf_status emsurf_server_submit(emsurf_server sv, uint64_t key, const emsurf_plan_desc* desc,
                                   const emsurf_geom* geom, const void* S_types, const int32_t* elem_type,
                                   int32_t nrhs, const void* b_host, int64_t* req_id) {
  return vguard([&] {
    EMS_CHECK_ARG(sv && desc && geom && S_types && elem_type && b_host, "arguments must be non-NULL");
    EMS_CHECK_ARG(nrhs >= 1 && nrhs <= sv->d.max_slots, "nrhs must be in [1, max_slots]");
    EMS_CHECK_ARG(desc->nx >= 1 && desc->ny >= 1 && desc->nx <= 512 && desc->ny <= 512, "bad lattice");
    EMS_CHECK_ARG(desc->n_eq == 4 * geom->n_patch && desc->n_types >= 1, "n_eq must equal 4 * n_patch");
    auto rq = std::make_unique<Request>();
    rq->id = sv->next_id++;
    rq->key = key;
    rq->desc = *desc;
    const int P = geom->n_patch;
    rq->rho.assign(geom->rho, geom->rho + 3 * P);
    rq->area.assign(geom->area, geom->area + P);
    rq->tan.assign(geom->tan, geom->tan + 6 * P);
    rq->pitch = geom->pitch;
    rq->k = geom->k;
    const size_t nS = (size_t)desc->n_types * desc->n_eq * desc->n_eq * 2;
    rq->S.assign(static_cast<const double*>(S_types), static_cast<const double*>(S_types) + nS);
    rq->types.assign(elem_type, elem_type + (size_t)desc->nx * desc->ny);
    for (int32_t t : rq->types) EMS_CHECK_ARG(t >= 0 && t < desc->n_types, "elem_type entry out of range");
    const size_t N = (size_t)desc->nx * desc->ny * desc->n_eq;
    rq->nrhs = nrhs;
    rq->b.assign(static_cast<const double*>(b_host), static_cast<const double*>(b_host) + 2 * N * nrhs);
    rq->t_submit = now_ms();
    if (req_id) *req_id = rq->id;
    sv->queue.push_back(std::move(rq));
  });
}

emsurf_status emsurf_server_step(emsurf_server sv, int32_t* n_completed) {
  return vguard([&] {
    EMS_CHECK_ARG(sv != nullptr, "server is NULL");
    const size_t before = sv->completed.size();
    const double t0 = now_ms();
    admit(sv);
    const double t1 = now_ms();
    std::vector<emsurf_session> busy;
    for (auto& kv : sv->plans)
      if (kv.second->active > 0) busy.push_back(kv.second->session);
    // launch every session's step first (each on its own stream), then wait
    for (auto* ss : busy) session_launch(ss);
    for (auto* ss : busy) session_finish(ss);
    harvest(sv);
    sv->admit_ms += t1 - t0;
    sv->step_ms += now_ms() - t1;
    if (n_completed) *n_completed = (int32_t)(sv->completed.size() - before);
  });
}

emsurf_status emsurf_server_next_completed(emsurf_server sv, int64_t* req_id, int32_t* nrhs, int64_t* n_unknowns) {
  return vguard([&] {
    EMS_CHECK_ARG(sv && req_id, "server and req_id must be non-NULL");
    *req_id = -1;
    if (sv->completed.empty()) return;
    const int64_t id = sv->completed.front();
    sv->completed.pop_front();
    Request& rq = *sv->done.at(id);
    *req_id = id;
    if (nrhs) *nrhs = rq.nrhs;
    if (n_unknowns) *n_unknowns = (int64_t)rq.desc.nx * rq.desc.ny * rq.desc.n_eq;
  });
}

emsurf_status emsurf_server_fetch(emsurf_server sv, int64_t req_id, void* x_host, emsurf_solve_info* info,
                                  double* times_ms) {
  return vguard([&] {
    EMS_CHECK_ARG(sv != nullptr, "server is NULL");
    auto it = sv->done.find(req_id);
    EMS_CHECK_ARG(it != sv->done.end(), "unknown or not finished request id");
    Request& rq = *it->second;
    if (x_host && !rq.x.empty()) std::memcpy(x_host, rq.x.data(), rq.x.size() * sizeof(double));
    if (info)
      for (int r = 0; r < (int)rq.info.size(); ++r) info[r] = rq.info[r];
    if (times_ms) {
      times_ms[0] = rq.t_admit - rq.t_submit;
      times_ms[1] = rq.t_done - rq.t_submit;
    }
    const bool bad = rq.bad;
    sv->done.erase(it);
    if (bad) {
      set_error("request could not be solved (invalid plan or non-finite right-hand side)");
      throw Err{EMSURF_ERR_ARG};
    }
  });
}

emsurf_status emsurf_server_query(emsurf_server sv, emsurf_server_stats* out) {
  return vguard([&] {
    EMS_CHECK_ARG(sv && out, "server and out must be non-NULL");
    out->queued = (int32_t)sv->queue.size();
    out->active = (int32_t)sv->active.size();
    out->resident_plans = (int32_t)sv->plans.size();
    out->bytes_used = sv->used;
    out->plans_built = sv->plans_built;
    out->evictions = sv->evictions;
    out->admit_ms = sv->admit_ms;
    out->step_ms = sv->step_ms;
  });
}

size_t emsurf_server_entry_bytes(emsurf_server sv, const emsurf_plan_desc* desc) {
  if (!sv || !desc) return 0;
  try {
    return entry_bytes(sv, *desc);
  } catch (...) {
    return 0;
  }
}

size_t emsurf_server_slot_bytes(emsurf_server sv, const emsurf_plan_desc* desc) {
  if (!sv || !desc) return 0;
  try {
    return entry_bytes(sv, *desc) ? entry_slot_bytes(sv, *desc) : 0;
  } catch (...) {
    return 0;
  }
}

void emsurf_server_destroy(emsurf_server sv) { delete sv; }

}  // extern "C"
