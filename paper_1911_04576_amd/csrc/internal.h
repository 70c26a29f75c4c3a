// Internal declarations of the emsurf library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/emsurf.h"

namespace emsurf {

// ----------------------------------------------------------------------------- errors
void set_error(const std::string& msg);
const char* last_error();

struct Err {
  emsurf_status st;
};
// Status of the exception being handled (call only inside a catch block): the
// library's own errors carry their status, host allocation failures map to
// EMSURF_ERR_OOM and anything else to EMSURF_ERR_DEVICE, so that no exception
// crosses the C interface.
emsurf_status current_exception_status();
template <typename F>
emsurf_status guarded_call(F&& f) {
  try {
    f();
    return EMSURF_OK;
  } catch (...) {
    return current_exception_status();
  }
}

#define EMS_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      ::emsurf::set_error(std::string(#call) + ": " + hipGetErrorString(e_));              \
      throw ::emsurf::Err{e_ == hipErrorOutOfMemory ? EMSURF_ERR_OOM : EMSURF_ERR_DEVICE}; \
    }                                                                                      \
  } while (0)

#define EMS_CHECK_ARG(cond, msg)                 \
  do {                                           \
    if (!(cond)) {                               \
      ::emsurf::set_error(msg);                  \
      throw ::emsurf::Err{EMSURF_ERR_ARG};       \
    }                                            \
  } while (0)

#define EMS_LAUNCH_CHECK() EMS_HIP(hipGetLastError())

// ----------------------------------------------------------------------------- device buffer
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    EMS_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // keep the buffer if it already holds n bytes, else reallocate
  void reserve(size_t n) {
    if (n > bytes) alloc(n);
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() { if (p) (void)hipHostFree(p); }
  void alloc(size_t n) {
    if (p) (void)hipHostFree(p);
    p = nullptr; bytes = 0;
    if (n == 0) return;
    EMS_HIP(hipHostMalloc(&p, n, hipHostMallocDefault));
    bytes = n;
  }
  void reserve(size_t n) {
    if (n > bytes) alloc(n);
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ----------------------------------------------------------------------------- FFT
// One pass of a batched 1-D FFT along one lattice axis.  A "line" is one 1-D
// transform over L points for a contiguous set of batch columns; line l is
// split as (l1, l0) = (l / nl0, l % nl0) to form its base offsets.
struct FftPass {
  int L = 0;           // transform length: 2^a in [2, 1024] or 3 * 2^a in [24, 768]
  int n_in = 0;        // points read; points >= n_in are zero
  int n_out = 0;       // points written (crop)
  int batch = 0;       // batch columns per line (contiguous, stride 1)
  int n_lines = 0;
  int nl0 = 1;
  int64_t in_s0 = 0, in_s1 = 0, out_s0 = 0, out_s1 = 0;   // line strides (elements)
  int64_t in_pt = 0, out_pt = 0;                          // point strides (elements)
  int sign = -1;       // -1 forward, +1 inverse
  double scale = 1.0;  // applied to outputs
};

enum class Cx { C64, C128 };

bool fft_length_supported(int L);
// smallest supported FFT length >= v (the circulant embedding needs >= 2N - 1)
int fft_length_at_least(int v);

// Launch a pass. tin/tcomp/tout select element types of input, arithmetic and output.
void launch_fft_pass(const FftPass& p, Cx tin, Cx tcomp, Cx tout, const void* in, void* out,
                     const void* twiddles, hipStream_t s);
struct GreenGeomDev;
// x pass of the kernel transform (FP64) whose inputs are the point-sampled
// coupling entries of columns [c0, c0 + p.batch), generated in the first stage
// instead of loaded (lines = the Ly slots along y)
void launch_fft_pass_green(const FftPass& p, const GreenGeomDev& geo, int nx, int ny, int Ly, int64_t c0, int n,
                           int vperm, void* out, const void* twiddles, hipStream_t s);
// Twiddle table exp(-2 pi i j / L), j < L, in FP64 (computed on the host with
// long-double arithmetic) and FP32 (rounded from it).  Device memory, cached.
const void* twiddle_table(int L, Cx t);

// ----------------------------------------------------------------------------- block products
// yh[k][r][u] = sum_v That[k](u, v) xh[k][r][v]; yh and xh must not overlap.
// That layout: [k][v][u] (column-major n x n blocks).
void launch_block_product(Cx t, const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P,
                          hipStream_t s);
// Kernel variants of the FP32 product (FP64 always uses the lane-per-row GEMV):
// BP_GEMV = lane-per-row streaming GEMV; BP_MFMA_Tk = MFMA GEMM with k row
// tiles of 32 per wavefront (n_eq a multiple of 32, ceil(n_eq/32/k) <= 4),
// 4 K steps of block columns in flight; BP_MFMA_TkD the same with 6 or 8.
enum BpVariant {
  BP_GEMV = 0, BP_MFMA_T1 = 1, BP_MFMA_T2 = 2, BP_MFMA_T3 = 3, BP_MFMA_T4 = 4,
  BP_MFMA_T1D = 5, BP_MFMA_T2D = 6, BP_MFMA_T3D = 7, BP_MFMA_T4D = 8, BP_NVARIANTS = 9
};
bool block_mfma_supported(int n, int nrhs);
// variant runnable for this n_eq (MFMA: n_eq % 32 == 0, <= 480, at most 4 wavefronts)
bool block_variant_supported(int variant, int n, int nrhs);
void launch_block_product_variant(Cx t, int variant, const void* That, const void* xh, void* yh, int n, int nrhs,
                                  int64_t P, hipStream_t s);
// Block layout of the reciprocal store (FP64 and FP32 alike, padding zero):
// 16 x 16 tiles (nt = ceil(n / 16) per side), 256 complex entries per tile,
// in the order the four wavefronts of the paired product visit them: u tile t
// belongs to wavefront w = t % 4, which walks v tiles outer (v tile q at step
// (q - w) mod nt) and its own u tiles inner, so tile (t, q) sits at
// base(w) + ((q - w) mod nt) ntw(w) + t / 4, with ntw(w) = (nt - w + 3) / 4
// and base(w) = nt sum_{w' < w} ntw(w').  Within a
// tile, real and imaginary parts apart: the first product's A operand on the
// matrix cores holds part p of tile entry (a, b) in lane L = a + 16 p +
// 32 (b % 2), register r = b / 2.  With ch = 16 / (bytes of a real) values per
// 16-byte chunk (4 in FP32, 2 in FP64) the tile stores chunk r / ch of every
// lane in turn: value offset (r / ch) 64 ch + L ch + r % ch, so that each
// 16-byte load instruction of a wavefront reads 1024 contiguous bytes.
constexpr int PAIR_TILE = 16;
__host__ __device__ inline int pair_tiles(int n) { return (n + PAIR_TILE - 1) / PAIR_TILE; }
// complex entries (= reals / 2) of one stored block
__host__ __device__ inline int64_t pair_block_entries(int n) {
  return (int64_t)pair_tiles(n) * pair_tiles(n) * PAIR_TILE * PAIR_TILE;
}
// u tiles of wavefront w, and the first tile position of wavefront w
__host__ __device__ inline int pair_wave_tiles(int nt, int w) { return (nt - w + 3) / 4; }
__host__ __device__ inline int pair_wave_base(int nt, int w) {
  int b = 0;
  for (int x = 0; x < w; ++x) b += pair_wave_tiles(nt, x) * nt;
  return b;
}
// tile position of (u tile t, v tile q) within a block
__host__ __device__ inline int pair_tile_pos(int nt, int t, int q) {
  const int w = t % 4;   // < nt, as t < nt
  return pair_wave_base(nt, w) + ((q - w + nt) % nt) * pair_wave_tiles(nt, w) + t / 4;
}
// in-tile real-value offset of part p of tile entry (a, b) (row a, column b
// of a 16 x 16 tile): lane a + 16 p + 32 (b % 2), register b / 2 of the
// first operand of v_mfma_*_16x16x4, chunk by chunk (ch reals per 16 bytes)
__host__ __device__ inline int tile_value_offset(int a, int b, int p, int ch) {
  const int L = a + 16 * p + 32 * (b % 2), r = b / 2;
  return (r / ch) * 64 * ch + L * ch + r % ch;
}
// real-value offset of part p (0 real, 1 imaginary) of entry (u, v) within a
// block; ch = 4 for FP32, 2 for FP64
__host__ __device__ inline int64_t pair_value_offset(int n, int u, int v, int p, int ch) {
  return (int64_t)pair_tile_pos(pair_tiles(n), u / PAIR_TILE, v / PAIR_TILE) * (2 * PAIR_TILE * PAIR_TILE) +
         tile_value_offset(u % PAIR_TILE, v % PAIR_TILE, p, ch);
}
// Reciprocal structured plans (EMSURF_T_LK): per stored pair the n_h x 2 n_h
// matrix [L | K] in 16 x 16 tiles, ntr = ceil(n_h / 16) row tiles and 2 ntr
// column tiles (L in column tiles q < ntr, K in q >= ntr, each half padded to
// whole tiles), in the order the four wavefronts visit them: column tile q
// with wavefront q % 4, its row tiles inner, so tile (t, q) sits at
// base(q % 4) + (q / 4) ntr + t with base(w) = ntr sum_{w' < w} nqw(w'),
// nqw(w) = (2 ntr - w + 3) / 4 column tiles of wavefront w.
__host__ __device__ inline int64_t lkpair_block_entries(int nh) {
  return (int64_t)pair_tiles(nh) * 2 * pair_tiles(nh) * PAIR_TILE * PAIR_TILE;
}
__host__ __device__ inline int lkpair_tile_pos(int ntr, int t, int q) {
  const int w = q % 4, ntc = 2 * ntr;
  int base = 0;
  for (int x = 0; x < w; ++x) base += (ntc - x + 3) / 4 * ntr;
  return base + (q / 4) * ntr + t;
}
// real-value offset of part p of entry (u, v) of L (half 0) or K (half 1)
__host__ __device__ inline int64_t lkpair_value_offset(int nh, int u, int v, int half, int p, int ch) {
  const int ntr = pair_tiles(nh);
  const int q = half * ntr + v / PAIR_TILE;
  return (int64_t)lkpair_tile_pos(ntr, u / PAIR_TILE, q) * (2 * PAIR_TILE * PAIR_TILE) +
         tile_value_offset(u % PAIR_TILE, v % PAIR_TILE, p, ch);
}
// Paired products of a reciprocal structured plan: with L(-d) = D^-1 L(d)^T D
// and K(-d) = D^-1 K(d)^T D (D = w, n_h weights),
//   yh[k]  = [[a L, b K], [c K, e L]] xh[k],
//   yh[-k] = [[a D^-1 L^T D, b D^-1 K^T D], [c D^-1 K^T D, e D^-1 L^T D]] xh[-k].
void launch_block_product_pair_lk(Cx t, const void* That, const void* pairs, const void* w, const void* winv,
                                  const void* xh, void* yh, int nh, int nrhs, int64_t Ps, const double* coef,
                                  hipStream_t s);
// Reciprocal plans: one block per frequency pair {k, -k}; pairs = int [Ps][2]
// (k, -k), w / winv the per-unknown weights and their inverses in the compute
// precision.  yh[k] = That[s] xh[k], yh[-k] = W^-1 That[s]^T W xh[-k].
void launch_block_product_pair(Cx t, const void* That, const void* pairs, const void* w, const void* winv,
                               const void* xh, void* yh, int n, int nrhs, int64_t Ps, hipStream_t s);
// pairs (k, -k) with k <= -k in increasing k, flattened; slot_of[k] = pair index or -1
void spectrum_pairs(int Lx, int Ly, std::vector<int>& pairs, std::vector<int>& slot_of);

// Structured outer operator (EMSURF_T_LK): That per frequency holds the
// stacked n x n_h matrix [L; K] column-major ([k][v][L|K][u]);
//   yh[k][r][u] = a L xJ + b K xM (u < n_h),  yh[k][r][n_h + u] = c K xJ + e L xM,
// xJ = xh[k][r][0:n_h], xM = xh[k][r][n_h:2 n_h]; coef = (a, b, c, e) as (re, im).
// variant: BP_GEMV (lane-per-row stream, FP32 or FP64) or an FP32 MFMA variant
// (as for dense blocks, two operand blocks per step); FP64 always streams.
void launch_block_product_lk(Cx t, int variant, const void* That, const void* xh, void* yh, int nh, int nrhs,
                             int64_t P, const double* coef, hipStream_t s);
bool block_variant_supported_lk(int variant, int n, int nrhs);
void launch_block_mfma_lk(int variant, const void* That, const void* xh, void* yh, int nh, int nrhs, int64_t P,
                          const double* coef, hipStream_t s);
// FP32 MFMA variants only (blockprod_mfma.hip); ERR_ARG for a variant that
// block_variant_supported rejects
void launch_block_mfma(int variant, const void* That, const void* xh, void* yh, int n, int nrhs, int64_t P,
                       hipStream_t s);
// Split-BF16 products (blockprod_bf16.hip): split = 3 runs a_hi b_hi + a_hi b_lo
// + a_lo b_hi, split = 1 a_hi b_hi alone; FP32 spectral input and output.
// Tb: per frequency a hi plane then a lo plane, entry (u, v) part p at bf16
// index ((v / 4) n + u) 8 + (v % 4) 2 + p of its plane (bf16_offset).
bool block_bf16_supported(int n);
void launch_block_bf16(int split, const void* Tb, const void* xh, void* yh, int n, int nrhs, int64_t P,
                       hipStream_t s);
__host__ __device__ inline int64_t bf16_offset(int n, int u, int v, int p) {
  return ((int64_t)(v / 4) * n + u) * 8 + (v % 4) * 2 + p;
}

// ----------------------------------------------------------------------------- S apply
struct TypeTiles {
  DevBuf elem_sorted;   // int32 [M] elements sorted by type
  DevBuf tiles;         // int32 [n_tiles][3] = (type, start in elem_sorted, count)
  int n_tiles = 0;
};
// y[r][m] = (axpy ? x_axpy[r][m] - : ) S_{type(m)} t[r][m]
// types: S store type; t type; x_axpy and y types (FP64 or FP32 per ty/tx).
void launch_apply_S(Cx ts, Cx tt, Cx txy, const void* S, const TypeTiles& tiles, int n, int M, int nrhs,
                    const void* t, const void* x_axpy, void* y, hipStream_t s);
// The same on the matrix cores, from macromodels packed by launch_pack_S
// (FP64 or FP32 reals, packed_S_reals of them, from the FP64 [type][n][n]
// macromodels); compute type tc for S and t, x_axpy and y of type txy.
size_t packed_S_reals(int n, int n_types);
void launch_pack_S(Cx t, const void* S64, void* out, int n, int n_types, hipStream_t s);
void launch_apply_S_packed(Cx tc, Cx txy, const void* Sp, const TypeTiles& tiles, int n, int M, int nrhs,
                           const void* t, const void* x_axpy, void* y, hipStream_t s);

// ----------------------------------------------------------------------------- fill
// Write padded kernel K[sy][sx][v][u] (columns cols [c0, c0+nc) of the n*n batch
// only, as a dense [Ly][Lx][nc] array) from blocks or from the Green fill.
struct GreenGeomDev {
  DevBuf rho, area, tan;   // double [P][3], [P], [P][2][3]
  int n_patch = 0;
  double pitch = 0, k = 0;
};
// validate a box geometry (finite pitch > 0, areas > 0) and copy it to the device
void upload_geom(const emsurf_geom* g, GreenGeomDev& d);
// a patch centre of one box coincides with one of an adjacent box (touching boxes)
bool boxes_touch(const emsurf_geom* g);
// caller blocks: `parts` row-major nb x nb matrices per offset (1 x n_eq dense; 2 x n_h for L, K)
// vperm: columns in the pair_fill_v order (dense blocks only)
void launch_pad_blocks(const void* T_blocks_dev, int nx, int ny, int nb, int parts, int Lx, int Ly, int64_t c0,
                       int64_t nc, int vperm, void* K, hipStream_t s);
// structured (L, K) fill into the padded layout / into [2ny-1][2nx-1][2][n_h][n_h]
void launch_lk_padded(const GreenGeomDev& g, int nx, int ny, int Lx, int Ly, int64_t c0, int64_t nc, void* K,
                      hipStream_t s);
void launch_lk_blocks(const GreenGeomDev& g, int nx, int ny, void* LK_blocks, hipStream_t s);
void launch_green_padded(const GreenGeomDev& g, int nx, int ny, int Lx, int Ly, int64_t c0, int64_t nc, int vperm,
                         void* K, hipStream_t s);
void launch_green_blocks(const GreenGeomDev& g, int nx, int ny, void* T_blocks, hipStream_t s);
// Scatter a [P][nc] chunk into the [P][n*n] store at column offset c0 (FP64 and/or FP32 rounded).
// slot_of (device int [P], or NULL for the identity) maps a frequency to its
// stored block, -1 for frequencies that are not stored; with slot_of the
// blocks (n x n, kernel column v n + u) go to the row-panel layout of the
// reciprocal store, else to [k][v][u].
// that16 (or NULL): the split-BF16 store of a full dense plan (slot_of NULL),
// split from the FP32-rounded entry.
// nh > 0: the columns are those of a structured record (v (2 n_h) + half n_h
// + u) and a reciprocal store takes the [L | K] pair layout.
// pairs / Ps: the pair list (k, -k) per stored slot, used by the pair-order store
// uperm: rows in the green_fill_u order (point-sampled dense plans)
void launch_store_chunk(const void* Kc, int64_t P, int64_t nn, int64_t c0, int64_t nc, const int* slot_of,
                        const int* pairs, int64_t Ps, int n, int nh, int vperm, int uperm, void* that64,
                        void* that32, void* that16, hipStream_t s);
// max |T(-d)[u][v] - T(d)[v][u] w[v] / w[u]| and max |T(d)| over dense caller
// blocks [2ny-1][2nx-1][n][n] (device), written to out (device double [2]).
// parts = 2 for structured blocks [..][2][n][n] (L and K, each checked with w).
void launch_recip_check(const void* T_blocks_dev, int nx, int ny, int n, int parts, const double* w_dev, double* out,
                        hipStream_t s);

// ----------------------------------------------------------------------------- dense elimination
// Partial elimination of the leading K x K block of T row-major N x N FP64
// complex matrices (A + b N^2), partial pivoting among the leading rows: the
// trailing block becomes A22 - A21 A11^-1 A12.  piv: int [T][K] work space;
// info[b] (zeroed by the caller) receives 1 + the first column whose pivot
// candidates are all zero.
void schur_eliminate(double2* A, int N, int K, int T, int* piv, int* info, hipStream_t s);

// ----------------------------------------------------------------------------- vector ops (GMRES)
void launch_convert(Cx tin, Cx tout, const void* in, void* out, int64_t n, hipStream_t s);

// ----------------------------------------------------------------------------- plan
struct Workspace {
  DevBuf W;     // half-transformed [Ny][Lx][B]
  DevBuf X;     // spectral input [Ly][Lx][B]
  DevBuf Y;     // spectral output [Ly][Lx][B]
  DevBuf t;     // T x result for A-apply [nrhs][M][n] (widest type)
};

// GMRES workspace of emsurf_solve (csrc/solver.hip), kept per stream in the plan
struct SolveWork;
void destroy_solve_work(SolveWork* w);
size_t solve_work_bytes(const SolveWork* w);

struct KernelTimer {
  bool enabled = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[5];
  size_t used[5] = {0, 0, 0, 0, 0};
  double ms_acc[5] = {0, 0, 0, 0, 0};
  int64_t cnt[5] = {0, 0, 0, 0, 0};
};

}  // namespace emsurf

struct emsurf_plan_s {
  emsurf_plan_desc d{};
  int Lx = 0, Ly = 0;
  int64_t P = 0;
  int M = 0;
  emsurf::DevBuf that64, that32;  // [Ps][v][u]
  emsurf::DevBuf that16;          // split-BF16 store: [P][hi | lo plane], bf16_offset order
  int64_t Ps = 0;                 // stored blocks: P, or the pair count of a reciprocal plan
  emsurf::DevBuf pairs;           // reciprocal plans: int [Ps][2]
  emsurf::DevBuf w64, winv64, w32, winv32;  // reciprocal weights and inverses [n]
  emsurf::DevBuf S64, S32;        // [n_types][n][n] row-major
  emsurf::DevBuf SP64, SP32;      // the same packed for the matrix-core apply
  emsurf::TypeTiles tiles;
  std::mutex mu;
  std::map<hipStream_t, emsurf::Workspace*> ws;
  std::map<hipStream_t, emsurf::SolveWork*> solve_ws;  // created by the first solve on a stream
  emsurf::KernelTimer timer;
  hipStream_t timer_stream = nullptr;
  int bp_variant[65];             // FP32 block-product variant per nrhs, -1 = automatic
  emsurf_plan_s() { for (int& v : bp_variant) v = -1; }
  ~emsurf_plan_s();
};

namespace emsurf {
// x = P^-1 y with a near-field preconditioner (precond.hip); FP64 c128
// [nrhs][M][n_eq], x != y
void precond_apply(emsurf_precond pc, int nrhs, const void* y, void* x, hipStream_t s);
emsurf_plan precond_plan(emsurf_precond pc);
Workspace& workspace(emsurf_plan p, hipStream_t s);
// FP32 block-product variant for this plan and nrhs: explicit choice, else the
// persisted autotuning cache, else a heuristic.
int choose_variant(emsurf_plan p, int nrhs);
// apply_T with explicit element types: input tin, compute/that type tc, output tout.
// variant: FP32 block-product variant, -1 = the plan's choice for nrhs.
// split: 0 = products on the tc store; 1 or 3 = split-BF16 products (tc must
// be C64) with one or three matrix-core products per entry.
void apply_T_typed(emsurf_plan p, Cx tin, Cx tc, Cx tout, int nrhs, const void* x, void* y, hipStream_t s,
                   int variant = -1, int split = 0);
// The same apply on caller-supplied intermediates: W (half-transformed, Ny Lx
// nrhs n_eq values), X and Y (spectra, Lx Ly nrhs n_eq values each) in the
// compute type, and the twiddle tables of Lx and Ly.  timed: record the
// plan's phase events when kernel timing is on.
struct ApplyBufs {
  void* W;
  void* X;
  void* Y;
  const void* twx;
  const void* twy;
};
void apply_T_bufs(emsurf_plan p, Cx tin, Cx tc, Cx tout, int nrhs, const void* x, void* y, const ApplyBufs& b,
                  hipStream_t s, int variant, int split, bool timed);
// values (complex, compute type) of W and of each of X, Y for nrhs right-hand sides
inline int64_t apply_W_values(emsurf_plan p, int nrhs);
inline int64_t apply_X_values(emsurf_plan p, int nrhs);
// apply_A with explicit types: x (tx) -> y (ty) = x - S T x, arithmetic in tc.
void apply_A_typed(emsurf_plan p, Cx tx, Cx tc, Cx ty, int nrhs, const void* x, void* y, hipStream_t s,
                   int variant = -1, int split = 0);
// y = (x_axpy ? x_axpy - : ) S t with the plan's macromodels (matrix cores),
// compute type tc for t, type ty for x_axpy and y
void apply_S_plan(emsurf_plan p, Cx tc, Cx ty, int nrhs, const void* t, const void* x_axpy, void* y, hipStream_t s);
// element type and split of an apply precision (EMSURF_FP64, EMSURF_FP32,
// EMSURF_BF16X3, EMSURF_BF16); ERR_ARG for any other
struct ApplyPrec {
  Cx t;
  int split;
};
ApplyPrec apply_prec(emsurf_prec prec);
inline int64_t apply_W_values(emsurf_plan p, int nrhs) { return (int64_t)p->d.ny * p->Lx * nrhs * p->d.n_eq; }
inline int64_t apply_X_values(emsurf_plan p, int nrhs) { return p->P * nrhs * p->d.n_eq; }
// twiddle table if it exists already (no allocation), else NULL
const void* twiddle_lookup(int L, Cx t);
inline size_t cx_bytes(Cx t) { return t == Cx::C128 ? 16 : 8; }
// kernel columns (complex entries) of one frequency's Fourier-domain record:
// n_eq^2 for dense blocks, 2 (n_eq/2)^2 for the L and K operators
// Column order of the chunked kernel fill of a dense reciprocal plan: column
// c holds entry (u, v) with u = c % n_eq and v = pair_fill_v(c / n_eq); in each
// group of 8 consecutive v the even ones come first.  Then v, v + 2, v + 4,
// v + 6 (the values of one 16-byte chunk of the paired tile layout, in FP32;
// v, v + 2 in FP64) are 4 consecutive column groups, and a chunk of whole
// multiples of 4 n_eq columns writes whole 16-byte pieces of the store.
__host__ __device__ inline int pair_fill_v(int vp, int n) {
  const int g = vp & ~7, w = vp & 7;
  const int m = n - g < 8 ? n - g : 8;   // members of this group
  const int e = (m + 1) >> 1;            // of which even
  return g + (w < e ? 2 * w : 2 * (w - e) + 1);
}
// Row order of the point-sampled (Green) kernel columns: position up of a
// column holds row u = green_fill_u(up), ordering each current type's rows
// by tangent index a before patch p (u = 2 P hu + 2 p + a, up = 2 P hu + P a + p),
// so that neighbouring lanes of the generating transform share a tangent and
// with it which entries vanish.  green_fill_up is the inverse.
__host__ __device__ inline int green_fill_u(int up, int P) {
  const int hu = up / (2 * P), r = up - hu * 2 * P;
  const int a = r / P, p = r - a * P;
  return hu * 2 * P + 2 * p + a;
}
__host__ __device__ inline int green_fill_up(int u, int P) {
  const int hu = u / (2 * P), r = u - hu * 2 * P;
  return hu * 2 * P + (r & 1) * P + (r >> 1);
}
inline int64_t kernel_cols(const emsurf_plan_desc& d) {
  const int64_t n = d.n_eq;
  return d.form == EMSURF_T_LK ? 2 * (n / 2) * (n / 2) : n * n;
}
}  // namespace emsurf
