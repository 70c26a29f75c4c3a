/*
 * emsurf -- FFT-coupled macromodel solver for lattices of fictitious boxes on
 * one AMD Instinct MI355X (gfx950).
 *
 * The operator solved is  A x = (I - S T) x = b  where
 *   S  is block-diagonal: one dense n_eq x n_eq macromodel per lattice element,
 *      shared by all elements of a cell type (paper Sec. III-A, eq.
 *      (Zmacromodel_Array); Sec. II-D: macromodels for unique cells only);
 *   T  is the block-Toeplitz free-space coupling between elements (Sec. III-B,
 *      eqs. (out) and (blockZo); Toeplitz by Sec. IV-A), applied by circulant
 *      embedding and 2-D FFTs over the lattice with the local-basis products
 *      accumulated in the Fourier domain (Sec. IV-B, eqs. (LJV3)-(LJV5) and the
 *      2-D generalisation at the end of Sec. IV-B);
 * and the solve is restarted GMRES (Sec. IV-A).  The form (I - S T) follows
 * from the summed system (Z_eq + Z_o) Y = V of Sec. III-C by splitting Z_o into
 * its per-element self blocks and its mutual blocks and left-multiplying by
 * the inverse of the block-diagonal part: S = -(Z_eq + Z_o^self)^-1, T = Z_o^mut.
 *
 * Conventions shared by every entry point
 *  - Complex numbers are interleaved (re, im): c128 = two doubles, c64 = two
 *    floats; layout-compatible with torch.complex128 / complex64 and C99
 *    _Complex.
 *  - Vectors are laid out x[r][iy][ix][u]: right-hand side r, lattice row iy,
 *    column ix, local unknown u (element m = iy*nx + ix, the element-major
 *    stacking of Sec. III-A; J unknowns before M unknowns on each box).
 *  - Coupling blocks are T(d) with d = (dy, dx) = (test element) - (source
 *    element), the index convention of the 1-D example of Sec. IV-B, stored
 *    as c128 [2ny-1][2nx-1][n_eq][n_eq] at [dy+ny-1][dx+nx-1], row = test
 *    unknown, column = source unknown.
 *  - Pointers named *_dev are HIP device pointers (e.g. tensor.data_ptr());
 *    all other pointers are host pointers.  `stream` is a hipStream_t (NULL =
 *    the null stream).
 *  - Every call returns a status; on error nothing is allocated, out-params
 *    and plan state are unchanged, and emsurf_last_error() describes the cause
 *    for the calling thread.  No C++ exception crosses this interface.
 *  - apply_* calls are asynchronous on `stream`; solve blocks the host.
 *  - A plan is immutable after creation; applies on different streams may run
 *    concurrently on one plan (each apply uses a per-stream workspace taken
 *    from the plan under a lock).  Solves on one plan use internal workspaces
 *    and must not overlap each other.
 */
#ifndef EMSURF_H
#define EMSURF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EMSURF_OK = 0,
  EMSURF_ERR_ARG = 1,            /* invalid argument (null pointer, size, non-finite b, ...) */
  EMSURF_ERR_OOM = 2,            /* device or pinned host allocation failed */
  EMSURF_ERR_DEVICE = 3,         /* a HIP runtime call failed */
  EMSURF_ERR_NOT_CONVERGED = 4,  /* solve stopped at max_iter / max_outer; best iterate returned */
  EMSURF_ERR_BUSY = 5,           /* session has no free slot */
  EMSURF_ERR_UNSUPPORTED = 6     /* precision not resident in this plan, or size beyond the kernels */
} emsurf_status;

typedef enum {
  EMSURF_FP64 = 0,     /* FP64 FFTs and products on the FP64 Fourier-domain store */
  EMSURF_FP32 = 1,     /* FP32 FFTs and products on the FP32 store (rounded from FP64) */
  EMSURF_FP32_IR = 2   /* solve only: FP32 inner GMRES, FP64 residual refinement */
} emsurf_prec;

/* bit mask of Fourier-domain block stores kept resident in a plan */
#define EMSURF_STORE_FP64 1u
#define EMSURF_STORE_FP32 2u

typedef struct emsurf_plan_s* emsurf_plan;

typedef struct {
  int32_t nx, ny;      /* lattice size, 1..512 each */
  int32_t n_eq;        /* unknowns per element, 1 <= n_eq <= 512 */
  int32_t n_types;     /* number of macromodel cell types, >= 1 */
  int32_t max_rhs;     /* largest nrhs any apply or solve on this plan uses, 1..64 */
  uint32_t store;      /* EMSURF_STORE_* mask, non-zero */
} emsurf_plan_desc;

/* Geometry of one box for the synthetic point-sampled coupling fill: the
 * Green's function exp(-jkR)/(4 pi R) between patch centres of distinct boxes,
 * weighted by the source patch area, J coupling to J and M to M through the
 * dot product of the patch tangents; T(0) = 0.  Unknown order on a box:
 * u = tau*(2*n_patch) + 2*p + alpha (tau 0 = J, 1 = M; alpha = tangent). */
typedef struct {
  int32_t n_patch;      /* n_eq = 4 * n_patch */
  const double* rho;    /* host [n_patch][3] patch centres relative to the box centre */
  const double* area;   /* host [n_patch] patch areas */
  const double* tan;    /* host [n_patch][2][3] unit tangents */
  double pitch;         /* lattice pitch (element (ix, iy) sits at pitch*(ix, iy, 0)) */
  double k;             /* free-space wavenumber */
} emsurf_geom;

typedef struct {
  emsurf_prec prec;     /* EMSURF_FP64, EMSURF_FP32 or EMSURF_FP32_IR */
  double tol;           /* stop when ||b - A x|| / ||b|| <= tol (FP64 operator for FP64/IR) */
  int32_t restart;      /* GMRES cycle length m, 1..64 (default 30) */
  int32_t max_iter;     /* total Arnoldi steps per RHS (inner steps summed for IR) */
  int32_t use_x0;       /* 1: start from the x passed in; 0: start from x = 0 */
  double inner_tol;     /* IR only: floor of the inner relative tolerance; inner solve k aims at
                           max(inner_tol, tol * ||b|| / (2 ||r_k||)) (default 1e-6) */
  int32_t max_outer;    /* IR only: refinement steps (default 10) */
} emsurf_solve_opts;

typedef struct {
  int32_t iters;          /* Arnoldi steps (matrix-vector products with A) */
  int32_t outer_iters;    /* refinement steps (IR) or GMRES cycles (FP64/FP32) */
  int32_t converged;      /* 1 if the true relative residual met tol */
  double rel_res_true;    /* ||b - A x|| / ||b|| with the FP64 operator (FP32 operator for EMSURF_FP32) */
  double ms;              /* host wall time of the whole solve */
} emsurf_solve_info;

typedef struct {
  int32_t Lx, Ly;           /* padded FFT lengths (>= 2n-1, powers of two) */
  int64_t n_freq;           /* Lx * Ly */
  size_t bytes_that64;      /* FP64 Fourier-domain store, 0 if absent */
  size_t bytes_that32;      /* FP32 store, 0 if absent */
  size_t bytes_total;       /* all device memory the plan holds */
} emsurf_plan_stats;

/* Device bytes a plan with this descriptor will hold (Fourier-domain stores,
 * macromodels, index lists and apply workspaces for max_rhs), for admission
 * control.  Returns 0 for an invalid descriptor. */
size_t emsurf_plan_bytes(const emsurf_plan_desc* desc);

/* Build a plan from caller-supplied coupling blocks (Sec. IV-B: circulant
 * embedding of every block, kernel FFT, products later in the Fourier domain).
 *   T_blocks    c128 [2ny-1][2nx-1][n_eq][n_eq] (layout above); host memory if
 *               T_is_device == 0, device memory otherwise.  Read during the
 *               call only; the caller keeps ownership.
 *   S_types     host c128 [n_types][n_eq][n_eq], row-major, y_u = sum_v S[u][v] x_v.
 *   elem_type   host int32 [ny][nx], each in [0, n_types).
 * The call synchronises `stream` before returning.  *out receives the plan. */
emsurf_status emsurf_plan_create(const emsurf_plan_desc* desc, const void* T_blocks, int32_t T_is_device,
                                 const void* S_types, const int32_t* elem_type, void* stream,
                                 emsurf_plan* out);

/* Build a plan whose coupling blocks are the synthetic point-sampled fill of
 * `geom`, computed on the device straight into the padded kernel layout (no
 * [2ny-1][2nx-1] intermediate).  desc->n_eq must equal 4 * geom->n_patch. */
emsurf_status emsurf_plan_create_green(const emsurf_plan_desc* desc, const emsurf_geom* geom,
                                       const void* S_types, const int32_t* elem_type, void* stream,
                                       emsurf_plan* out);

/* Write the synthetic point-sampled blocks of `geom` for an nx x ny lattice
 * into T_blocks_dev (c128 [2ny-1][2nx-1][n_eq][n_eq], caller-allocated, device). */
emsurf_status emsurf_fill_T_point_green(const emsurf_geom* geom, int32_t nx, int32_t ny,
                                        void* T_blocks_dev, void* stream);

/* y = T x over nrhs right-hand sides (1 <= nrhs <= max_rhs).  x_dev and y_dev
 * are c128 for EMSURF_FP64 and c64 for EMSURF_FP32, [nrhs][ny][nx][n_eq]; they
 * must not overlap.  Requires the matching store in the plan. */
emsurf_status emsurf_apply_T(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                             void* y_dev, void* stream);

/* y = S x (block-diagonal macromodel apply).  Same types and layout as apply_T;
 * x_dev and y_dev may be the same buffer only if they are identical pointers
 * (then the call is out-of-place internally). */
emsurf_status emsurf_apply_S(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                             void* y_dev, void* stream);

/* y = x - S T x.  Same types and layout as apply_T; x_dev and y_dev must not overlap. */
emsurf_status emsurf_apply_A(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                             void* y_dev, void* stream);

/* Solve A x = b for nrhs independent right-hand sides with restarted GMRES
 * (Sec. IV-A).  b_dev, x_dev: c128 [nrhs][ny][nx][n_eq] device.  With use_x0
 * the solve starts from x_dev's content.  info_host: nrhs entries (may be
 * NULL).  Blocks until done.  Returns EMSURF_ERR_NOT_CONVERGED (x holds the
 * best iterate, info filled) if any RHS missed tol; EMSURF_ERR_ARG if b has a
 * non-finite entry.  A zero RHS returns x = 0, converged, 0 iterations. */
emsurf_status emsurf_solve(emsurf_plan plan, const emsurf_solve_opts* opts, int32_t nrhs,
                           const void* b_dev, void* x_dev, emsurf_solve_info* info_host, void* stream);

/* Plan facts (padded sizes and memory). */
emsurf_status emsurf_plan_query(emsurf_plan plan, emsurf_plan_stats* out);

/* Per-kernel timing of apply_T.  While enabled, every apply_T on the plan
 * brackets each of its kernel launches with HIP events recorded on the apply's
 * stream.  emsurf_kernel_times() synchronises those events and writes, for
 * each phase (0 forward FFT along x, 1 forward FFT along y, 2 Fourier-domain
 * block product, 3 inverse FFT along y, 4 inverse FFT along x), the summed
 * milliseconds into ms[5] and the number of launches into count[5], then
 * clears the record.  Timing costs a few microseconds per launch. */
emsurf_status emsurf_kernel_timing(emsurf_plan plan, int32_t enable);
emsurf_status emsurf_kernel_times(emsurf_plan plan, double* ms, int64_t* count);

void emsurf_plan_destroy(emsurf_plan plan);
const char* emsurf_status_str(emsurf_status s);
const char* emsurf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EMSURF_H */
