// Continuous-batching session state (session.hip) shared with the server.
#pragma once
#include <complex>
#include <vector>

#include "internal.h"

namespace emsurf {

struct SessionSlot {
  enum Phase { FREE, INIT, RESID, ARNOLDI, DONE };
  Phase ph = FREE;
  int64_t tag = 0;
  double bnorm = 0, beta = 0, target = 0, rel = 0;
  int j = 0, kend = 0, iters = 0, cycles = 0;
  bool converged = false, bad = false;
  double t_submit = 0, t_done = 0;
  std::vector<std::complex<double>> H, g, sn;
  std::vector<double> cs;
};

// Device bytes of a session: the part held for its lifetime (batch staging,
// reductions, item lists), the vectors of one slot ([b | x | r | V_0..V_m],
// allocated when a slot is first used), and the total with every slot
// allocated plus the apply workspace of its stream.
size_t session_fixed_bytes(const emsurf_plan_desc& d, int max_slots, int restart);
size_t session_slot_bytes(const emsurf_plan_desc& d, int restart);
size_t session_bytes(const emsurf_plan_desc& d, int max_slots, int restart);
void session_launch(emsurf_session ss);
int session_finish(emsurf_session ss);
// bytes of the slot buffers the session holds, and the number of free slots
// that hold one
size_t session_held_bytes(emsurf_session ss);
int session_free_held(emsurf_session ss);
// release the buffers of free slots; returns the bytes released
size_t session_trim(emsurf_session ss);

}  // namespace emsurf

struct emsurf_session_s {
  emsurf_plan plan = nullptr;
  emsurf_solve_opts opts{};
  int S = 0, m = 0;
  long long N = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev = nullptr;
  emsurf::DevBuf xin, wout, partial, red, coef, items;
  std::vector<emsurf::DevBuf> mem;   // per slot: [b | x | r | V_0 .. V_m] (N values each), or empty
  emsurf::PinnedBuf h_red, h_coef, h_items;
  int nblk = 0, ns = 0, rstride = 0, variant32 = 0;
  bool launched = false;
  std::vector<emsurf::SessionSlot> slot;
  std::vector<int> q_norm, q_arn;
  ~emsurf_session_s();
};

namespace emsurf {
void session_init(emsurf_session ss, emsurf_plan plan, int max_slots, const emsurf_solve_opts& o, hipStream_t s,
                  bool own);
}
