// Plans and operator applies of the C ABI: circulant embedding and kernel FFT
// at plan time, then y = T x (Sec. IV-B), y = S x (Sec. III-A) and
// y = x - S T x per apply.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>

#include "internal.h"

namespace emsurf {

namespace {
thread_local std::string g_last_error;

void validate_desc(const emsurf_plan_desc* d) {
  EMS_CHECK_ARG(d != nullptr, "plan descriptor is NULL");
  EMS_CHECK_ARG(d->nx >= 1 && d->ny >= 1, "lattice sizes nx, ny must be >= 1");
  EMS_CHECK_ARG(d->nx <= 512 && d->ny <= 512, "lattice sizes above 512 are not supported");
  EMS_CHECK_ARG(d->n_eq >= 1 && d->n_eq <= 512, "n_eq must be in [1, 512]");
  EMS_CHECK_ARG(d->n_types >= 1, "n_types must be >= 1");
  EMS_CHECK_ARG(d->max_rhs >= 1 && d->max_rhs <= 64, "max_rhs must be in [1, 64]");
  const uint32_t all = EMSURF_STORE_FP64 | EMSURF_STORE_FP32 | EMSURF_STORE_BF16;
  EMS_CHECK_ARG(d->store != 0 && (d->store & ~all) == 0,
                "store must be a non-empty mask of EMSURF_STORE_FP64 | EMSURF_STORE_FP32 | EMSURF_STORE_BF16");
  EMS_CHECK_ARG(d->form == EMSURF_T_DENSE || d->form == EMSURF_T_LK, "form must be EMSURF_T_DENSE or EMSURF_T_LK");
  if (d->form == EMSURF_T_LK) {
    EMS_CHECK_ARG(d->n_eq % 2 == 0, "EMSURF_T_LK needs an even n_eq (J and M halves)");
    for (double c : d->coef) EMS_CHECK_ARG(std::isfinite(c), "EMSURF_T_LK coefficients must be finite");
  }
  EMS_CHECK_ARG(d->recip == 0 || d->recip == 1, "recip must be 0 or 1");
  EMS_CHECK_ARG(d->recip == 0 || d->form == EMSURF_T_DENSE || d->n_eq <= 416,
                "reciprocal storage of the structured form supports n_eq <= 416");
  if (d->store & EMSURF_STORE_BF16) {
    EMS_CHECK_ARG(d->form == EMSURF_T_DENSE && d->recip == 0,
                  "the split-BF16 store needs a dense plan that stores every frequency (recip 0)");
    EMS_CHECK_ARG(block_bf16_supported(d->n_eq), "the split-BF16 store needs n_eq a multiple of 32 in [32, 480]");
  }
  // The pass along y of a full-width apply spans Lx Ly max_rhs n_eq complex
  // values, addressed with 32-bit offsets inside the FFT kernels: refuse such
  // plans here rather than at their first apply.
  const int64_t Lx = fft_length_at_least(2 * d->nx - 1), Ly = fft_length_at_least(2 * d->ny - 1);
  const int64_t B = (int64_t)d->max_rhs * d->n_eq;
  EMS_CHECK_ARG(Lx * Ly * B + B + 1024 < (1LL << 31),
                "padded lattice x max_rhs x n_eq exceeds the 2^31 values one FFT pass addresses; "
                "lower max_rhs (or n_eq)");
}

// complex entries of one stored block of a reciprocal plan (tile padding included)
int64_t recip_block_entries(const emsurf_plan_desc& d) {
  return d.form == EMSURF_T_LK ? lkpair_block_entries(d.n_eq / 2) : pair_block_entries(d.n_eq);
}

// stored blocks: every frequency, or one per pair {k, -k} (a length L has one
// self-paired index, 0, when odd and two, 0 and L/2, when even)
int64_t stored_blocks(int Lx, int Ly, bool recip) {
  const int64_t P = (int64_t)Lx * Ly;
  if (!recip) return P;
  const int64_t self = (Lx % 2 == 0 ? 2 : 1) * (Ly % 2 == 0 ? 2 : 1);
  return (P + self) / 2;
}

struct Sizes {
  int Lx, Ly;
  int64_t P, Ps, M, n, nn;
  size_t that64, that32, that16, S, tiles, ws;
};

Sizes sizes_of(const emsurf_plan_desc* d) {
  Sizes z{};
  z.Lx = fft_length_at_least(2 * d->nx - 1);
  z.Ly = fft_length_at_least(2 * d->ny - 1);
  z.P = (int64_t)z.Lx * z.Ly;
  z.Ps = stored_blocks(z.Lx, z.Ly, d->recip == 1);
  z.M = (int64_t)d->nx * d->ny;
  z.n = d->n_eq;
  z.nn = z.n * z.n;
  const int64_t kc = kernel_cols(*d);
  const int64_t kc64 = d->recip ? recip_block_entries(*d) : kc;
  const int64_t kc32 = kc64;
  z.that64 = (d->store & EMSURF_STORE_FP64) ? (size_t)(z.Ps * kc64) * 16 : 0;
  z.that32 = (d->store & EMSURF_STORE_FP32) ? (size_t)(z.Ps * kc32) * 8 : 0;
  z.that16 = (d->store & EMSURF_STORE_BF16) ? (size_t)(z.P * z.nn) * 8 : 0;
  z.S = (size_t)d->n_types * z.nn * (16 + 8) + packed_S_reals(z.n, d->n_types) * (8 + 4);
  z.tiles = (size_t)z.M * 4 + (size_t)(z.M + d->n_types) * 12;
  if (d->recip) z.tiles += (size_t)z.Ps * 8 + (size_t)z.n * 24;  // pair list and weights
  const int64_t B = (int64_t)d->max_rhs * z.n;
  z.ws = (size_t)(d->ny * (int64_t)z.Lx * B) * 16 + 2 * (size_t)(z.P * B) * 16 + (size_t)(B * z.M) * 16;
  return z;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

emsurf_status current_exception_status() {
  try {
    throw;
  } catch (const Err& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return EMSURF_ERR_OOM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return EMSURF_ERR_DEVICE;
  } catch (...) {
    set_error("unknown error");
    return EMSURF_ERR_DEVICE;
  }
}
const char* last_error() { return g_last_error.c_str(); }

// Workspaces: one per stream, sized for max_rhs at FP64 width.
Workspace& workspace(emsurf_plan p, hipStream_t s) {
  std::lock_guard<std::mutex> lk(p->mu);
  auto it = p->ws.find(s);
  if (it != p->ws.end()) return *it->second;
  const int64_t B = (int64_t)p->d.max_rhs * p->d.n_eq;
  auto w = std::make_unique<Workspace>();
  w->W.alloc((size_t)(p->d.ny * (int64_t)p->Lx * B) * 16);
  w->X.alloc((size_t)(p->P * B) * 16);
  w->Y.alloc((size_t)(p->P * B) * 16);
  w->t.alloc((size_t)(B * p->M) * 16);
  Workspace* raw = w.release();
  p->ws[s] = raw;
  return *raw;
}

void timer_begin(emsurf_plan p, int phase, hipStream_t s, hipEvent_t* end_out) {
  *end_out = nullptr;
  if (!p->timer.enabled) return;
  auto& T = p->timer;
  if (T.used[phase] == T.ev[phase].size()) {
    hipEvent_t a, b;
    EMS_HIP(hipEventCreate(&a));
    EMS_HIP(hipEventCreate(&b));
    T.ev[phase].push_back({a, b});
  }
  auto& pr = T.ev[phase][T.used[phase]++];
  EMS_HIP(hipEventRecord(pr.first, s));
  *end_out = pr.second;
}

void timer_end(hipEvent_t e, hipStream_t s) {
  if (e) EMS_HIP(hipEventRecord(e, s));
}

void apply_T_typed(emsurf_plan p, Cx tin, Cx tc, Cx tout, int nrhs, const void* x, void* y, hipStream_t s,
                   int variant, int split) {
  Workspace& w = workspace(p, s);
  const ApplyBufs b{w.W.p, w.X.p, w.Y.p, twiddle_table(p->Lx, tc), twiddle_table(p->Ly, tc)};
  apply_T_bufs(p, tin, tc, tout, nrhs, x, y, b, s, variant, split, true);
}

void apply_T_bufs(emsurf_plan p, Cx tin, Cx tc, Cx tout, int nrhs, const void* x, void* y, const ApplyBufs& bufs,
                  hipStream_t s, int variant, int split, bool timed) {
  EMS_CHECK_ARG(split == 0 || (tc == Cx::C64 && (split == 1 || split == 3)), "internal: bad split-BF16 request");
  const void* That = split ? p->that16.p : (tc == Cx::C128) ? p->that64.p : p->that32.p;
  if (!That) {
    set_error(split ? "plan has no split-BF16 Fourier-domain store"
              : tc == Cx::C128 ? "plan has no FP64 Fourier-domain store" : "plan has no FP32 Fourier-domain store");
    throw Err{EMSURF_ERR_UNSUPPORTED};
  }
  struct Bufs {
    void *W, *X, *Y;
  } w{bufs.W, bufs.X, bufs.Y};
  const int n = p->d.n_eq, Nx = p->d.nx, Ny = p->d.ny, Lx = p->Lx, Ly = p->Ly;
  const int64_t M = p->M;
  const int64_t B = (int64_t)nrhs * n;
  const void* twx = bufs.twx;
  const void* twy = bufs.twy;
  hipEvent_t e;
  // phase events only on timed applies
  auto timer_begin = [&](emsurf_plan pp, int phase, hipStream_t ss, hipEvent_t* end_out) {
    *end_out = nullptr;
    if (timed) ::emsurf::timer_begin(pp, phase, ss, end_out);
  };

  // forward along x: lines (r, iy); x[r][iy][ix][u] -> W[iy][kx][r][u]
  FftPass fx;
  fx.L = Lx; fx.n_in = Nx; fx.n_out = Lx; fx.batch = n;
  fx.n_lines = nrhs * Ny; fx.nl0 = Ny;
  fx.in_s1 = M * n; fx.in_s0 = (int64_t)Nx * n; fx.in_pt = n;
  fx.out_s1 = n; fx.out_s0 = (int64_t)Lx * B; fx.out_pt = B;
  fx.sign = -1;
  timer_begin(p, 0, s, &e);
  launch_fft_pass(fx, tin, tc, tc, x, w.W, twx, s);
  timer_end(e, s);

  // forward along y: lines kx; W[iy][kx][b] -> X[ky][kx][b]
  FftPass fy;
  fy.L = Ly; fy.n_in = Ny; fy.n_out = Ly; fy.batch = (int)B;
  fy.n_lines = Lx; fy.nl0 = Lx;
  fy.in_s0 = B; fy.in_pt = (int64_t)Lx * B;
  fy.out_s0 = B; fy.out_pt = (int64_t)Lx * B;
  fy.sign = -1;
  timer_begin(p, 1, s, &e);
  launch_fft_pass(fy, tc, tc, tc, w.W, w.X, twy, s);
  timer_end(e, s);

  // Fourier-domain block products
  timer_begin(p, 2, s, &e);
  const int v = tc == Cx::C64 && !p->d.recip && !split ? (variant >= 0 ? variant : choose_variant(p, nrhs))
                                                       : BP_GEMV;
  if (split)
    launch_block_bf16(split, That, w.X, w.Y, n, nrhs, p->P, s);
  else if (p->d.recip && p->d.form == EMSURF_T_LK)
    launch_block_product_pair_lk(tc, That, p->pairs.p, tc == Cx::C128 ? p->w64.p : p->w32.p,
                                 tc == Cx::C128 ? p->winv64.p : p->winv32.p, w.X, w.Y, n / 2, nrhs, p->Ps,
                                 p->d.coef, s);
  else if (p->d.recip)
    launch_block_product_pair(tc, That, p->pairs.p, tc == Cx::C128 ? p->w64.p : p->w32.p,
                              tc == Cx::C128 ? p->winv64.p : p->winv32.p, w.X, w.Y, n, nrhs, p->Ps, s);
  else if (p->d.form == EMSURF_T_LK)
    launch_block_product_lk(tc, v, That, w.X, w.Y, n / 2, nrhs, p->P, p->d.coef, s);
  else
    launch_block_product_variant(tc, v, That, w.X, w.Y, n, nrhs, p->P, s);
  timer_end(e, s);

  // inverse along y, keep rows iy < Ny
  FftPass iy = fy;
  iy.n_in = Ly; iy.n_out = Ny; iy.sign = +1;
  timer_begin(p, 3, s, &e);
  launch_fft_pass(iy, tc, tc, tc, w.Y, w.W, twy, s);
  timer_end(e, s);

  // inverse along x, keep ix < Nx, scale 1/(Lx Ly)
  FftPass ix;
  ix.L = Lx; ix.n_in = Lx; ix.n_out = Nx; ix.batch = n;
  ix.n_lines = nrhs * Ny; ix.nl0 = Ny;
  ix.in_s1 = n; ix.in_s0 = (int64_t)Lx * B; ix.in_pt = B;
  ix.out_s1 = M * n; ix.out_s0 = (int64_t)Nx * n; ix.out_pt = n;
  ix.sign = +1;
  ix.scale = 1.0 / ((double)Lx * (double)Ly);
  timer_begin(p, 4, s, &e);
  launch_fft_pass(ix, tc, tc, tout, w.W, y, twx, s);
  timer_end(e, s);
}

void apply_A_typed(emsurf_plan p, Cx tx, Cx tc, Cx ty, int nrhs, const void* x, void* y, hipStream_t s,
                   int variant, int split) {
  Workspace& w = workspace(p, s);
  apply_T_typed(p, tx, tc, tc, nrhs, x, w.t.p, s, variant, split);
  apply_S_plan(p, tc, ty, nrhs, w.t.p, x, y, s);
}

void apply_S_plan(emsurf_plan p, Cx tc, Cx ty, int nrhs, const void* t, const void* x_axpy, void* y, hipStream_t s) {
  const void* Sp = (tc == Cx::C128) ? p->SP64.p : p->SP32.p;
  launch_apply_S_packed(tc, ty, Sp, p->tiles, p->d.n_eq, p->M, nrhs, t, x_axpy, y, s);
}

bool boxes_touch(const emsurf_geom* g) {
  const int P = g->n_patch;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      if (dx == 0 && dy == 0) continue;
      for (int p = 0; p < P; ++p)
        for (int q = 0; q < P; ++q) {
          const double ex = g->rho[3 * p] - g->rho[3 * q] + g->pitch * dx;
          const double ey = g->rho[3 * p + 1] - g->rho[3 * q + 1] + g->pitch * dy;
          const double ez = g->rho[3 * p + 2] - g->rho[3 * q + 2];
          if (ex * ex + ey * ey + ez * ez <= 1e-18 * g->area[q]) return true;
        }
    }
  return false;
}

void upload_geom(const emsurf_geom* g, GreenGeomDev& d) {
  EMS_CHECK_ARG(g != nullptr && g->rho && g->area && g->tan, "geometry pointers must be non-NULL");
  EMS_CHECK_ARG(g->n_patch >= 1, "n_patch must be >= 1");
  EMS_CHECK_ARG(std::isfinite(g->pitch) && g->pitch > 0 && std::isfinite(g->k), "pitch must be > 0, k finite");
  const int P = g->n_patch;
  for (int i = 0; i < P; ++i) EMS_CHECK_ARG(g->area[i] > 0 && std::isfinite(g->area[i]), "patch areas must be > 0");
  d.n_patch = P;
  d.pitch = g->pitch;
  d.k = g->k;
  d.rho.alloc((size_t)P * 3 * 8);
  d.area.alloc((size_t)P * 8);
  d.tan.alloc((size_t)P * 6 * 8);
  EMS_HIP(hipMemcpy(d.rho.p, g->rho, (size_t)P * 3 * 8, hipMemcpyHostToDevice));
  EMS_HIP(hipMemcpy(d.area.p, g->area, (size_t)P * 8, hipMemcpyHostToDevice));
  EMS_HIP(hipMemcpy(d.tan.p, g->tan, (size_t)P * 6 * 8, hipMemcpyHostToDevice));
}

}  // namespace emsurf

emsurf_plan_s::~emsurf_plan_s() {
  for (auto& kv : ws) delete kv.second;
  for (auto& kv : solve_ws) emsurf::destroy_solve_work(kv.second);
  for (int ph = 0; ph < 5; ++ph)
    for (auto& pr : timer.ev[ph]) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
}

using namespace emsurf;

namespace {

template <typename F>
emsurf_status guarded(F&& f) {
  return guarded_call(std::forward<F>(f));
}

void build_tiles(emsurf_plan p, const int32_t* elem_type, hipStream_t s) {
  const int M = p->M;
  const int nt = p->d.n_types;
  std::vector<int> order(M);
  for (int m = 0; m < M; ++m) {
    EMS_CHECK_ARG(elem_type[m] >= 0 && elem_type[m] < nt, "elem_type entry out of [0, n_types)");
    order[m] = m;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return elem_type[a] < elem_type[b]; });
  const int TC = 32;
  std::vector<int> tiles;
  int i = 0;
  while (i < M) {
    const int t = elem_type[order[i]];
    int j = i;
    while (j < M && elem_type[order[j]] == t) ++j;
    for (int a = i; a < j; a += TC) {
      tiles.push_back(t);
      tiles.push_back(a);
      tiles.push_back(std::min(TC, j - a));
    }
    i = j;
  }
  p->tiles.n_tiles = (int)(tiles.size() / 3);
  p->tiles.elem_sorted.alloc(order.size() * sizeof(int));
  p->tiles.tiles.alloc(tiles.size() * sizeof(int));
  EMS_HIP(hipMemcpyAsync(p->tiles.elem_sorted.p, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, s));
  EMS_HIP(hipMemcpyAsync(p->tiles.tiles.p, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, s));
  EMS_HIP(hipStreamSynchronize(s));
}

void upload_S(emsurf_plan p, const void* S_types, hipStream_t s) {
  const size_t cnt = (size_t)p->d.n_types * p->d.n_eq * p->d.n_eq;
  const double* h = static_cast<const double*>(S_types);
  for (size_t i = 0; i < 2 * cnt; ++i) EMS_CHECK_ARG(std::isfinite(h[i]), "S_types has a non-finite entry");
  p->S64.alloc(cnt * 16);
  p->S32.alloc(cnt * 8);
  EMS_HIP(hipMemcpyAsync(p->S64.p, S_types, cnt * 16, hipMemcpyHostToDevice, s));
  launch_convert(Cx::C128, Cx::C64, p->S64.p, p->S32.p, (int64_t)cnt, s);
  const size_t pk = packed_S_reals(p->d.n_eq, p->d.n_types);
  p->SP64.alloc(pk * 8);
  p->SP32.alloc(pk * 4);
  launch_pack_S(Cx::C128, p->S64.p, p->SP64.p, p->d.n_eq, p->d.n_types, s);
  launch_pack_S(Cx::C64, p->S64.p, p->SP32.p, p->d.n_eq, p->d.n_types, s);
  EMS_HIP(hipStreamSynchronize(s));
}

// Kernel FFT of the padded blocks, in column chunks, into the resident stores.
// gen: dense point-sampled plans generate the entries inside the first pass of
// the kernel transform (no fill chunk written and read back); else `fill`
// writes each chunk
template <typename FillChunk>
void build_that(emsurf_plan p, hipStream_t s, FillChunk&& fill, const GreenGeomDev* gen = nullptr) {
  const int64_t nn = kernel_cols(p->d);
  const int64_t P = p->P;
  const int n = p->d.n_eq;
  const int64_t kc64 = p->d.recip ? recip_block_entries(p->d) : nn;
  const int64_t kc32 = kc64;
  if (p->d.store & EMSURF_STORE_FP64) p->that64.alloc((size_t)(p->Ps * kc64) * 16);
  if (p->d.store & EMSURF_STORE_FP32) p->that32.alloc((size_t)(p->Ps * kc32) * 8);
  if (p->d.store & EMSURF_STORE_BF16) p->that16.alloc((size_t)(P * nn) * 8);
  // the padding rows of the last panel of a reciprocal store stay zero
  if (p->d.recip && kc64 != nn && p->that64.p) EMS_HIP(hipMemsetAsync(p->that64.p, 0, p->that64.bytes, s));
  if (p->d.recip && kc32 != nn && p->that32.p) EMS_HIP(hipMemsetAsync(p->that32.p, 0, p->that32.bytes, s));
  // reciprocal plans keep the representative of each pair {k, -k}
  DevBuf slot_dev;
  if (p->d.recip) {
    std::vector<int> pairs, slot_of;
    spectrum_pairs(p->Lx, p->Ly, pairs, slot_of);
    EMS_CHECK_ARG((int64_t)pairs.size() == 2 * p->Ps, "internal: pair count mismatch");
    p->pairs.alloc(pairs.size() * sizeof(int));
    slot_dev.alloc(slot_of.size() * sizeof(int));
    EMS_HIP(hipMemcpyAsync(p->pairs.p, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice, s));
    EMS_HIP(hipMemcpyAsync(slot_dev.p, slot_of.data(), slot_of.size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  // two chunk buffers of at most ~512 MB each.  A dense reciprocal store fills
  // its columns in the pair_fill_v order, in chunks of whole multiples of
  // 4 n_eq columns (buffers of up to 1 GiB), so that each chunk writes whole
  // 16-byte pieces of the paired tiles instead of scattered values
  int64_t nc = (int64_t)((512ull << 20) / ((size_t)P * 16));
  // Point-sampled dense plans (gen) generate their entries inside the kernel
  // transform, with rows in the green_fill_u order, on the same whole-column
  // chunks; plans too large for such chunks fill chunk by chunk instead.
  const int64_t grp = 4 * (int64_t)n;
  const bool wide = (size_t)P * grp * 16 <= (1ull << 30);
  const int vperm = p->d.recip && p->d.form != EMSURF_T_LK && wide ? 1 : 0;
  if (!wide) gen = nullptr;
  if (vperm || gen) nc = std::max<int64_t>(1, nc / grp) * grp;
  nc = std::max<int64_t>(1, std::min<int64_t>(nc, nn));
  nc = std::min<int64_t>(nc, 0x7fffffff);
  DevBuf K((size_t)(P * nc) * 16), tmp((size_t)(P * nc) * 16);
  const void* twx = twiddle_table(p->Lx, Cx::C128);
  const void* twy = twiddle_table(p->Ly, Cx::C128);
  for (int64_t c0 = 0; c0 < nn; c0 += nc) {
    const int64_t cnt = std::min(nc, nn - c0);
    FftPass fx;
    fx.L = p->Lx; fx.n_in = p->Lx; fx.n_out = p->Lx; fx.batch = (int)cnt;
    fx.n_lines = p->Ly; fx.nl0 = p->Ly;
    fx.in_s0 = (int64_t)p->Lx * cnt; fx.in_pt = cnt;
    fx.out_s0 = (int64_t)p->Lx * cnt; fx.out_pt = cnt;
    fx.sign = -1;
    if (gen) {
      launch_fft_pass_green(fx, *gen, p->d.nx, p->d.ny, p->Ly, c0, n, vperm, tmp.p, twx, s);
    } else {
      fill(c0, cnt, K.p, vperm);
      launch_fft_pass(fx, Cx::C128, Cx::C128, Cx::C128, K.p, tmp.p, twx, s);
    }
    FftPass fy;
    fy.L = p->Ly; fy.n_in = p->Ly; fy.n_out = p->Ly; fy.batch = (int)cnt;
    fy.n_lines = p->Lx; fy.nl0 = p->Lx;
    fy.in_s0 = cnt; fy.in_pt = (int64_t)p->Lx * cnt;
    fy.out_s0 = cnt; fy.out_pt = (int64_t)p->Lx * cnt;
    fy.sign = -1;
    launch_fft_pass(fy, Cx::C128, Cx::C128, Cx::C128, tmp.p, K.p, twy, s);
    launch_store_chunk(K.p, P, nn, c0, cnt, slot_dev.as<const int>(), p->pairs.as<const int>(), p->Ps, n,
                       p->d.form == EMSURF_T_LK ? n / 2 : 0, vperm, gen ? 1 : 0,
                       p->that64.p, p->that32.p, p->that16.p, s);
  }
  EMS_HIP(hipStreamSynchronize(s));
}

// Workspace of the creating stream and every twiddle table the applies need are
// made now, so no apply (or graph capture) allocates or copies on first use.
void finish_plan(emsurf_plan p, hipStream_t s) {
  (void)workspace(p, s);
  for (Cx t : {Cx::C128, Cx::C64}) {
    (void)twiddle_table(p->Lx, t);
    (void)twiddle_table(p->Ly, t);
  }
  EMS_HIP(hipStreamSynchronize(s));
}

emsurf_plan new_plan(const emsurf_plan_desc* desc) {
  validate_desc(desc);
  auto z = sizes_of(desc);
  emsurf_plan p = new emsurf_plan_s();
  p->d = *desc;
  p->Lx = z.Lx;
  p->Ly = z.Ly;
  p->P = z.P;
  p->Ps = z.Ps;
  p->M = (int)z.M;
  return p;
}

// Reciprocity weights of the unknowns (host, n values): checked and kept on
// the device in both precisions with their inverses.
void set_weights(emsurf_plan p, const std::vector<double>& w, hipStream_t s) {
  const int n = p->d.n_eq;
  std::vector<double> inv(n);
  std::vector<float> w32(n), inv32(n);
  for (int u = 0; u < n; ++u) {
    EMS_CHECK_ARG(std::isfinite(w[u]) && w[u] != 0.0 && std::isfinite(1.0 / w[u]),
                  "reciprocity weights must be finite and non-zero");
    inv[u] = 1.0 / w[u];
    w32[u] = (float)w[u];
    inv32[u] = (float)inv[u];
  }
  p->w64.alloc((size_t)n * 8);
  p->winv64.alloc((size_t)n * 8);
  p->w32.alloc((size_t)n * 4);
  p->winv32.alloc((size_t)n * 4);
  EMS_HIP(hipMemcpyAsync(p->w64.p, w.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
  EMS_HIP(hipMemcpyAsync(p->winv64.p, inv.data(), (size_t)n * 8, hipMemcpyHostToDevice, s));
  EMS_HIP(hipMemcpyAsync(p->w32.p, w32.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
  EMS_HIP(hipMemcpyAsync(p->winv32.p, inv32.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
  EMS_HIP(hipStreamSynchronize(s));
}

}  // namespace

namespace emsurf {
ApplyPrec apply_prec(emsurf_prec prec) {
  switch (prec) {
    case EMSURF_FP64: return {Cx::C128, 0};
    case EMSURF_FP32: return {Cx::C64, 0};
    case EMSURF_BF16X3: return {Cx::C64, 3};
    case EMSURF_BF16: return {Cx::C64, 1};
    default: break;
  }
  set_error("apply precision must be EMSURF_FP64, EMSURF_FP32, EMSURF_BF16X3 or EMSURF_BF16");
  throw Err{EMSURF_ERR_ARG};
}
}  // namespace emsurf

namespace {

void check_apply(emsurf_plan plan, int32_t nrhs, const void* x, const void* y) {
  EMS_CHECK_ARG(plan != nullptr, "plan is NULL");
  EMS_CHECK_ARG(x != nullptr && y != nullptr, "x and y must be non-NULL device pointers");
  EMS_CHECK_ARG(nrhs >= 1 && nrhs <= plan->d.max_rhs, "nrhs must be in [1, max_rhs]");
}

}  // namespace

extern "C" {

size_t emsurf_plan_bytes(const emsurf_plan_desc* desc) {
  size_t out = 0;
  if (guarded([&] {
        validate_desc(desc);
        auto z = sizes_of(desc);
        out = z.that64 + z.that32 + z.that16 + z.S + z.tiles + z.ws;
      }) != EMSURF_OK)
    return 0;
  return out;
}

}  // extern "C"

namespace {

emsurf_status create_from_blocks(const emsurf_plan_desc* desc, const void* T_blocks, int32_t T_is_device,
                                 const double* weights, const void* S_types, const int32_t* elem_type, void* stream,
                                 emsurf_plan* out) {
  emsurf_plan p = nullptr;
  emsurf_status st = guarded([&] {
    EMS_CHECK_ARG(out != nullptr, "out is NULL");
    EMS_CHECK_ARG(T_blocks && S_types && elem_type, "T_blocks, S_types and elem_type must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    p = new_plan(desc);
    const int nx = desc->nx, ny = desc->ny, n = desc->n_eq;
    const bool lk = desc->form == EMSURF_T_LK;
    const int nb = lk ? n / 2 : n, parts = lk ? 2 : 1;
    const size_t tb_bytes = (size_t)(2 * ny - 1) * (2 * nx - 1) * parts * nb * nb * 16;
    DevBuf Tdev;
    const void* Tb = T_blocks;
    if (!T_is_device) {
      Tdev.alloc(tb_bytes);
      EMS_HIP(hipMemcpyAsync(Tdev.p, T_blocks, tb_bytes, hipMemcpyHostToDevice, s));
      Tb = Tdev.p;
    }
    if (desc->recip) {
      // n weights for dense blocks; n / 2 for the structured form (the weights
      // of L and K, stored twice so that both halves have theirs)
      std::vector<double> w(n, 1.0);
      if (weights) {
        for (int u = 0; u < n; ++u) w[u] = weights[u % nb];
      }
      set_weights(p, w, s);
      DevBuf res(2 * sizeof(double));
      launch_recip_check(Tb, nx, ny, nb, parts, p->w64.as<const double>(), res.as<double>(), s);
      double h[2];
      EMS_HIP(hipMemcpyAsync(h, res.p, sizeof(h), hipMemcpyDeviceToHost, s));
      EMS_HIP(hipStreamSynchronize(s));
      if (!(h[0] <= 1e-9 * h[1])) {
        set_error("T_blocks are not reciprocal under the given weights: max |T(-d) - W^-1 T(d)^T W| = " +
                  std::to_string(h[0]) + ", max |T(d)| = " + std::to_string(h[1]));
        throw Err{EMSURF_ERR_ARG};
      }
    }
    build_that(p, s, [&](int64_t c0, int64_t cnt, void* K, int vperm) {
      launch_pad_blocks(Tb, nx, ny, nb, parts, p->Lx, p->Ly, c0, cnt, vperm, K, s);
    });
    upload_S(p, S_types, s);
    build_tiles(p, elem_type, s);
    finish_plan(p, s);
  });
  if (st != EMSURF_OK) {
    delete p;
    return st;
  }
  *out = p;
  return EMSURF_OK;
}

}  // namespace

extern "C" {

emsurf_status emsurf_plan_create(const emsurf_plan_desc* desc, const void* T_blocks, int32_t T_is_device,
                                 const void* S_types, const int32_t* elem_type, void* stream, emsurf_plan* out) {
  return create_from_blocks(desc, T_blocks, T_is_device, nullptr, S_types, elem_type, stream, out);
}

emsurf_status emsurf_plan_create_reciprocal(const emsurf_plan_desc* desc, const void* T_blocks, int32_t T_is_device,
                                            const double* weights, const void* S_types, const int32_t* elem_type,
                                            void* stream, emsurf_plan* out) {
  if (desc && desc->recip != 1) {
    set_error("emsurf_plan_create_reciprocal needs desc->recip = 1");
    return EMSURF_ERR_ARG;
  }
  return create_from_blocks(desc, T_blocks, T_is_device, weights, S_types, elem_type, stream, out);
}

emsurf_status emsurf_spectrum_pairs(int32_t Lx, int32_t Ly, int32_t* pairs, int64_t* count) {
  return guarded([&] {
    EMS_CHECK_ARG(count != nullptr, "count is NULL");
    EMS_CHECK_ARG(Lx >= 1 && Ly >= 1 && (int64_t)Lx * Ly <= (1LL << 30), "Lx, Ly must be >= 1 with Lx Ly <= 2^30");
    EMS_CHECK_ARG(*count >= 0 && (*count == 0 || pairs != nullptr), "pairs is NULL with a non-zero capacity");
    std::vector<int> pr, slot_of;
    spectrum_pairs(Lx, Ly, pr, slot_of);
    const int64_t total = (int64_t)pr.size() / 2;
    const int64_t m = std::min(*count, total);
    for (int64_t i = 0; i < 2 * m; ++i) pairs[i] = pr[(size_t)i];
    *count = total;
  });
}

emsurf_status emsurf_plan_create_green(const emsurf_plan_desc* desc, const emsurf_geom* geom, const void* S_types,
                                       const int32_t* elem_type, void* stream, emsurf_plan* out) {
  emsurf_plan p = nullptr;
  emsurf_status st = guarded([&] {
    EMS_CHECK_ARG(out != nullptr, "out is NULL");
    EMS_CHECK_ARG(S_types && elem_type, "S_types and elem_type must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    validate_desc(desc);
    EMS_CHECK_ARG(geom != nullptr && desc->n_eq == 4 * geom->n_patch, "n_eq must equal 4 * geom->n_patch");
    EMS_CHECK_ARG(desc->form != EMSURF_T_LK || geom->k > 0, "the structured fill needs a wavenumber k > 0");
    GreenGeomDev g;
    upload_geom(geom, g);
    EMS_CHECK_ARG(desc->form != EMSURF_T_LK || !boxes_touch(geom),
                  "the structured fill needs boxes that do not touch (its gradient terms are singular there)");
    p = new_plan(desc);
    if (desc->recip) {
      // the fill weights each source by its patch area: W = that area per unknown
      const int P2 = 2 * geom->n_patch;
      std::vector<double> w(desc->n_eq);
      for (int u = 0; u < desc->n_eq; ++u) w[u] = geom->area[(u % P2) / 2];
      set_weights(p, w, s);
    }
    build_that(p, s, [&](int64_t c0, int64_t cnt, void* K, int vperm) {
      if (desc->form == EMSURF_T_LK)
        launch_lk_padded(g, desc->nx, desc->ny, p->Lx, p->Ly, c0, cnt, K, s);
      else
        launch_green_padded(g, desc->nx, desc->ny, p->Lx, p->Ly, c0, cnt, vperm, K, s);
    }, desc->form == EMSURF_T_LK ? nullptr : &g);
    upload_S(p, S_types, s);
    build_tiles(p, elem_type, s);
    finish_plan(p, s);
  });
  if (st != EMSURF_OK) {
    delete p;
    return st;
  }
  *out = p;
  return EMSURF_OK;
}

emsurf_status emsurf_fill_T_point_green(const emsurf_geom* geom, int32_t nx, int32_t ny, void* T_blocks_dev,
                                        void* stream) {
  return guarded([&] {
    EMS_CHECK_ARG(T_blocks_dev != nullptr, "T_blocks_dev is NULL");
    EMS_CHECK_ARG(nx >= 1 && ny >= 1 && nx <= 512 && ny <= 512, "lattice sizes must be in [1, 512]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    GreenGeomDev g;
    upload_geom(geom, g);
    launch_green_blocks(g, nx, ny, T_blocks_dev, s);
    // the geometry buffers are freed on return: finish using them first
    EMS_HIP(hipStreamSynchronize(s));
  });
}

emsurf_status emsurf_fill_LK_point_green(const emsurf_geom* geom, int32_t nx, int32_t ny, void* LK_blocks_dev,
                                         void* stream) {
  return guarded([&] {
    EMS_CHECK_ARG(LK_blocks_dev != nullptr, "LK_blocks_dev is NULL");
    EMS_CHECK_ARG(geom != nullptr && geom->k > 0, "the structured fill needs a wavenumber k > 0");
    EMS_CHECK_ARG(nx >= 1 && ny >= 1 && nx <= 512 && ny <= 512, "lattice sizes must be in [1, 512]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    GreenGeomDev g;
    upload_geom(geom, g);
    EMS_CHECK_ARG(!boxes_touch(geom),
                  "the structured fill needs boxes that do not touch (its gradient terms are singular there)");
    launch_lk_blocks(g, nx, ny, LK_blocks_dev, s);
    EMS_HIP(hipStreamSynchronize(s));
  });
}

emsurf_status emsurf_apply_T(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev, void* y_dev,
                             void* stream) {
  return guarded([&] {
    check_apply(plan, nrhs, x_dev, y_dev);
    EMS_CHECK_ARG(x_dev != y_dev, "apply_T needs distinct x and y buffers");
    const ApplyPrec ap = apply_prec(prec);
    apply_T_typed(plan, ap.t, ap.t, ap.t, nrhs, x_dev, y_dev, static_cast<hipStream_t>(stream), -1, ap.split);
  });
}

emsurf_status emsurf_apply_S(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev, void* y_dev,
                             void* stream) {
  return guarded([&] {
    check_apply(plan, nrhs, x_dev, y_dev);
    const Cx t = apply_prec(prec).t;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const void* src = x_dev;
    if (x_dev == y_dev) {
      Workspace& w = workspace(plan, s);
      const size_t bytes = (size_t)nrhs * plan->M * plan->d.n_eq * cx_bytes(t);
      EMS_HIP(hipMemcpyAsync(w.t.p, x_dev, bytes, hipMemcpyDeviceToDevice, s));
      src = w.t.p;
    }
    apply_S_plan(plan, t, t, nrhs, src, nullptr, y_dev, s);
  });
}

emsurf_status emsurf_apply_A(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev, void* y_dev,
                             void* stream) {
  return guarded([&] {
    check_apply(plan, nrhs, x_dev, y_dev);
    EMS_CHECK_ARG(x_dev != y_dev, "apply_A needs distinct x and y buffers");
    const ApplyPrec ap = apply_prec(prec);
    apply_A_typed(plan, ap.t, ap.t, ap.t, nrhs, x_dev, y_dev, static_cast<hipStream_t>(stream), -1, ap.split);
  });
}

emsurf_status emsurf_plan_query(emsurf_plan plan, emsurf_plan_stats* out) {
  return guarded([&] {
    EMS_CHECK_ARG(plan != nullptr && out != nullptr, "plan and out must be non-NULL");
    out->Lx = plan->Lx;
    out->Ly = plan->Ly;
    out->n_freq = plan->P;
    out->bytes_that64 = plan->that64.bytes;
    out->bytes_that32 = plan->that32.bytes;
    out->n_stored = plan->Ps;
    out->bytes_that16 = plan->that16.bytes;
    size_t tot = plan->that64.bytes + plan->that32.bytes + plan->that16.bytes + plan->S64.bytes + plan->S32.bytes +
                 plan->SP64.bytes + plan->SP32.bytes +
                 plan->tiles.elem_sorted.bytes + plan->tiles.tiles.bytes + plan->pairs.bytes + plan->w64.bytes +
                 plan->winv64.bytes + plan->w32.bytes + plan->winv32.bytes;
    std::lock_guard<std::mutex> lk(plan->mu);
    for (auto& kv : plan->ws) tot += kv.second->W.bytes + kv.second->X.bytes + kv.second->Y.bytes + kv.second->t.bytes;
    for (auto& kv : plan->solve_ws) tot += emsurf::solve_work_bytes(kv.second);
    out->bytes_total = tot;
  });
}

emsurf_status emsurf_kernel_timing(emsurf_plan plan, int32_t enable) {
  return guarded([&] {
    EMS_CHECK_ARG(plan != nullptr, "plan is NULL");
    plan->timer.enabled = enable != 0;
  });
}

emsurf_status emsurf_kernel_times(emsurf_plan plan, double* ms, int64_t* count) {
  return guarded([&] {
    EMS_CHECK_ARG(plan != nullptr && ms != nullptr && count != nullptr, "plan, ms and count must be non-NULL");
    auto& T = plan->timer;
    for (int ph = 0; ph < 5; ++ph) {
      double acc = 0;
      for (size_t i = 0; i < T.used[ph]; ++i) {
        EMS_HIP(hipEventSynchronize(T.ev[ph][i].second));
        float f = 0;
        EMS_HIP(hipEventElapsedTime(&f, T.ev[ph][i].first, T.ev[ph][i].second));
        acc += f;
      }
      ms[ph] = acc;
      count[ph] = (int64_t)T.used[ph];
      T.used[ph] = 0;
    }
  });
}

void emsurf_plan_destroy(emsurf_plan plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  delete plan;
}

const char* emsurf_status_str(emsurf_status s) {
  switch (s) {
    case EMSURF_OK: return "ok";
    case EMSURF_ERR_ARG: return "invalid argument";
    case EMSURF_ERR_OOM: return "out of memory";
    case EMSURF_ERR_DEVICE: return "device error";
    case EMSURF_ERR_NOT_CONVERGED: return "not converged";
    case EMSURF_ERR_BUSY: return "busy";
    case EMSURF_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* emsurf_last_error(void) { return emsurf::last_error(); }

}  // extern "C"
