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
  EMSURF_FP32_IR = 2,  /* solve only: FP32 inner GMRES, FP64 residual refinement */
  EMSURF_BF16X3 = 3,   /* applies only: FP32 FFTs, block products on the split-BF16 store with
                          three matrix-core products per entry, a b ~ a_hi b_hi + a_hi b_lo +
                          a_lo b_hi accumulated in FP32 (a = a_hi + a_lo, both bfloat16 rounded
                          to nearest even, a_lo = bf16(a - a_hi); the FP32 spectral input is
                          split the same way); per-product error about 3 * 2^-16 |a||b| */
  EMSURF_BF16 = 4      /* applies only: as EMSURF_BF16X3 with a_hi b_hi alone, reading half the
                          store; per-product error about 2^-7 |a||b| */
} emsurf_prec;

/* bit mask of Fourier-domain block stores kept resident in a plan */
#define EMSURF_STORE_FP64 1u
#define EMSURF_STORE_FP32 2u
/* split-BF16 store (for EMSURF_BF16X3 / EMSURF_BF16): per frequency a hi plane
 * then a lo plane of the FP32-rounded block, 8 n_eq^2 bytes in all.  Dense,
 * non-reciprocal plans with n_eq a multiple of 32 in [32, 480] only. */
#define EMSURF_STORE_BF16 4u

typedef struct emsurf_plan_s* emsurf_plan;

/* Form of the coupling operator a plan holds.
 *  EMSURF_T_DENSE: opaque dense n_eq x n_eq blocks T(d).
 *  EMSURF_T_LK:    the outer operator in the paper's structured form (eq.
 *                  (blockZo) with eqs. (SIE_TEFIE1_Outer)/(SIE_TMFIE1_Outer)):
 *                  T(d) = [[a L(d), b K(d)], [c K(d), e L(d)]] with the
 *                  discretised L and K operators (n_h x n_h, n_h = n_eq / 2,
 *                  J unknowns first) shared by the four quadrants; the plan
 *                  stores the Fourier transforms of L and K only, the storage
 *                  of Sec. IV-C (half the bytes of dense blocks). */
#define EMSURF_T_DENSE 0
#define EMSURF_T_LK 1

typedef struct {
  int32_t nx, ny;      /* lattice size, 1..512 each */
  int32_t n_eq;        /* unknowns per element, 1 <= n_eq <= 512 (even for EMSURF_T_LK) */
  int32_t n_types;     /* number of macromodel cell types, >= 1 */
  int32_t max_rhs;     /* largest nrhs any apply or solve on this plan uses, 1..64 */
  uint32_t store;      /* EMSURF_STORE_* mask, non-zero */
  int32_t form;        /* EMSURF_T_DENSE (0) or EMSURF_T_LK (1) */
  int32_t recip;       /* 1: reciprocal operator, store one Fourier-domain block per
                          frequency pair {k, -k} (see emsurf_plan_create_reciprocal);
                          EMSURF_T_LK with n_eq <= 416; 0: store every frequency */
  double coef[8];      /* EMSURF_T_LK: a, b, c, e as (re, im) pairs, finite; ignored for dense */
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
  int32_t Lx, Ly;           /* padded FFT lengths (>= 2n-1, of the form 2^a or 3 * 2^a) */
  int64_t n_freq;           /* Lx * Ly */
  size_t bytes_that64;      /* FP64 Fourier-domain store, 0 if absent */
  size_t bytes_that32;      /* FP32 store, 0 if absent */
  size_t bytes_total;       /* all device memory the plan holds */
  int64_t n_stored;         /* Fourier-domain blocks per store: n_freq, or the pair count of a reciprocal plan */
  size_t bytes_that16;      /* split-BF16 store (hi and lo planes), 0 if absent */
} emsurf_plan_stats;

/* Device bytes a plan with this descriptor will hold (Fourier-domain stores,
 * macromodels, index lists and apply workspaces for max_rhs), for admission
 * control.  Returns 0 for an invalid descriptor. */
size_t emsurf_plan_bytes(const emsurf_plan_desc* desc);

/* Build a plan from caller-supplied coupling blocks (Sec. IV-B: circulant
 * embedding of every block, kernel FFT, products later in the Fourier domain).
 *   T_blocks    EMSURF_T_DENSE: c128 [2ny-1][2nx-1][n_eq][n_eq] (layout above);
 *               EMSURF_T_LK: c128 [2ny-1][2nx-1][2][n_h][n_h], L(d) then K(d)
 *               for each offset, row = test, column = source.  Host memory if
 *               T_is_device == 0, device memory otherwise.  Read during the
 *               call only; the caller keeps ownership.
 *   S_types     host c128 [n_types][n_eq][n_eq], row-major, y_u = sum_v S[u][v] x_v.
 *   elem_type   host int32 [ny][nx], each in [0, n_types).
 * The call synchronises `stream` before returning.  *out receives the plan. */
emsurf_status emsurf_plan_create(const emsurf_plan_desc* desc, const void* T_blocks, int32_t T_is_device,
                                 const void* S_types, const int32_t* elem_type, void* stream,
                                 emsurf_plan* out);

/* Reciprocal plans (desc->recip = 1).  Reciprocity of the
 * Green's function (Sec. II: a source and a test point may trade places) makes
 * the blocks of Sec. IV-A satisfy T(-d) = W^-1 T(d)^T W for a diagonal W of
 * per-unknown weights (the source patch areas of the point-sampled fill); the
 * circulant embedding of Sec. IV-B turns this into That[-k] = W^-1 That[k]^T W.
 * A reciprocal plan stores one block per frequency pair {k, -k} (about half the
 * bytes) and its block products read each stored block once for both
 * frequencies.  Results equal those of a full plan up to rounding.
 *   weights  host double [n_eq], finite and non-zero; NULL means all ones
 *            (T(-d) = T(d)^T).
 * EMSURF_T_LK: L and K are reciprocal one by one, X(-d) = D^-1 X(d)^T D for
 * X = L, K with the n_eq / 2 weights D (`weights` then holds n_eq / 2 values);
 * a plan stores [L | K] of one frequency per pair and forms
 * yJ[-k] = D^-1 (a L^T D xJ + b K^T D xM), yM[-k] = D^-1 (c K^T D xJ + e L^T D xM)
 * from it (a quarter of the dense bytes).  The check covers both L and K.
 * The blocks are checked before the transform: the call fails with
 * EMSURF_ERR_ARG if max |T(-d) - W^-1 T(d)^T W| exceeds 1e-9 max |T(d)|, or if
 * desc->recip != 1.  Other arguments as for emsurf_plan_create (which itself
 * treats desc->recip = 1 as weights = NULL).  emsurf_plan_create_green with
 * desc->recip = 1 takes W from the geometry (the source patch area of each
 * unknown); its fill is reciprocal by construction. */
emsurf_status emsurf_plan_create_reciprocal(const emsurf_plan_desc* desc, const void* T_blocks,
                                            int32_t T_is_device, const double* weights,
                                            const void* S_types, const int32_t* elem_type, void* stream,
                                            emsurf_plan* out);

/* Stored frequencies of a reciprocal plan with padded lengths Lx, Ly: pair s
 * of the store holds That[pairs[2s]] and serves k = pairs[2s] and
 * -k = pairs[2s + 1] (k = ky * Lx + kx, -k = ((Ly - ky) % Ly) * Lx + (Lx - kx) % Lx,
 * k <= -k; the two are equal for self-paired frequencies).  Pure host
 * function: writes min(*count, total) pairs into `pairs` (host int32
 * [2 * capacity], may be NULL with *count = 0) and sets *count to the total,
 * (Lx Ly + s) / 2 with s the number of self-paired frequencies. */
emsurf_status emsurf_spectrum_pairs(int32_t Lx, int32_t Ly, int32_t* pairs, int64_t* count);

/* Build a plan whose coupling blocks are the synthetic point-sampled fill of
 * `geom`, computed on the device straight into the padded kernel layout (no
 * [2ny-1][2nx-1] intermediate).  desc->n_eq must equal 4 * geom->n_patch.
 * EMSURF_T_DENSE uses the scalar fill described at emsurf_geom; EMSURF_T_LK
 * the structured fill described at emsurf_fill_LK_point_green. */
emsurf_status emsurf_plan_create_green(const emsurf_plan_desc* desc, const emsurf_geom* geom,
                                       const void* S_types, const int32_t* elem_type, void* stream,
                                       emsurf_plan* out);

/* Write the synthetic point-sampled blocks of `geom` for an nx x ny lattice
 * into T_blocks_dev (c128 [2ny-1][2nx-1][n_eq][n_eq], caller-allocated, device). */
emsurf_status emsurf_fill_T_point_green(const emsurf_geom* geom, int32_t nx, int32_t ny,
                                        void* T_blocks_dev, void* stream);

/* Write the synthetic structured blocks of `geom` (outer operator of Sec.
 * III-B, point-matched at the test patch centre, one-point quadrature over
 * the source patch, R = rho_p - rho_q + pitch (dx, dy, 0), g = exp(-jkR)/(4 pi R)):
 *     L(d)[(p,a),(q,b)] = A_q t_pa . (I + grad grad / k^2) g(R) . t_qb
 *     K(d)[(p,a),(q,b)] = A_q t_pa . (grad g(R) x t_qb),   L(0) = K(0) = 0,
 * local index 2p + a, into LK_blocks_dev (c128 [2ny-1][2nx-1][2][n_h][n_h],
 * n_h = 2 * n_patch, caller-allocated, device). */
emsurf_status emsurf_fill_LK_point_green(const emsurf_geom* geom, int32_t nx, int32_t ny,
                                         void* LK_blocks_dev, void* stream);

/* Macromodel generation for unique cells (Sec. II-D, eq. (Zmacromodel)): for
 * every cell type t the interior unknowns are eliminated with the Schur
 * complement (LU with partial pivoting of Z_int,int),
 *     Z~_t = Z_eq,eq - Z_eq,int Z_int,int^-1 Z_int,eq,
 * and the element operator of the solve (block-Jacobi form of Sec. III-C) is
 *     S_t = -(Z~_t + Z_self)^-1.
 *   Z_dev      c128 [n_types][N][N], N = n_eq + n_int, row-major, the reduced
 *              cell system [[Z_eq,eq, Z_eq,int], [Z_int,eq, Z_int,int]]
 *              (equivalent-surface unknowns first); read only.
 *   Zself_dev  c128 [n_eq][n_eq], the box self block of the outer operator,
 *              shared by all types; NULL means zero.
 *   S_dev      c128 [n_types][n_eq][n_eq] output, row-major (the S_types
 *              layout of emsurf_plan_create once copied to the host).
 *   Zt_dev     c128 [n_types][n_eq][n_eq] output of Z~, or NULL.
 * 1 <= n_types <= 4096, 1 <= n_eq <= 512, 0 <= n_int <= 4096.  Workspaces of
 * n_types ((n_eq + n_int)^2 + 4 n_eq^2) complex values are allocated for the
 * call.  Part of the elimination runs on a second stream that the library
 * creates once per device (default priority) and joins back into `stream`;
 * the call blocks until `stream` is done.  A singular Z_int,int or Z~ + Z_self (a zero
 * pivot column) returns EMSURF_ERR_ARG naming the cell type, with the outputs
 * unspecified. */
emsurf_status emsurf_macromodels(int32_t n_types, int32_t n_eq, int32_t n_int, const void* Z_dev,
                                 const void* Zself_dev, void* S_dev, void* Zt_dev, void* stream);

/* Far field radiated by the equivalent currents of every box (Sec. II-A:
 * the equivalent J and M on each fictitious surface radiate the exterior
 * field; Sec. III: they are the solved unknowns), with the point-sampled
 * currents of the coupling fill (patch q of element (ix, iy) carries
 * J = sum_a x_J[q, a] t_qa at rho_q + pitch (ix, iy, 0), M likewise) and
 * eta = 1, common factor -jk e^{-jkr} / (4 pi r) dropped:
 *     E_theta = N . theta^ + L . phi^,   E_phi = N . phi^ - L . theta^,
 *     N = sum A_q J e^{jk rhat . r'},    L = sum A_q M e^{jk rhat . r'}.
 * Directions are the bins of an Lu x Lv lattice DFT: bin (q, p) has direction
 * cosines u = 2 pi p' / (Lu k pitch), v = 2 pi q' / (Lv k pitch), with p', q'
 * the signed bin indices (p' = p for p < Lu/2, else p - Lu), w = cos(theta) =
 * sqrt(1 - u^2 - v^2) >= 0 (upper half space, phi = 0 at the zenith).
 *   x_dev   c128 [nrhs][ny][nx][n_eq], n_eq = 4 * geom->n_patch (J unknowns first).
 *   E_dev   c128 [nrhs][Lv][Lu][2] output (E_theta, E_phi) per bin; bins with
 *           u^2 + v^2 >= 1 (no real direction) are set to zero.
 * Lu >= nx and Lv >= ny must be supported FFT lengths (2^a <= 1024 or
 * 3 * 2^a <= 768); larger ones sample the pattern more finely.  Workspaces of
 * nrhs * n_eq * Lu * (ny + Lv) complex values are allocated for the call,
 * which synchronises `stream` before returning. */
emsurf_status emsurf_far_field(const emsurf_geom* geom, int32_t nx, int32_t ny, int32_t nrhs, int32_t Lu,
                               int32_t Lv, const void* x_dev, void* E_dev, void* stream);

/* Directivity of the same currents (Sec. V shows it in the phi = 0, 45 and 90
 * degree cuts): D = 4 pi U / P_rad with U = |E_theta|^2 + |E_phi|^2 (the
 * dropped common factor cancels).  The paper does not state how it integrates
 * the radiated power; here P_rad is the midpoint rule in direction cosines
 * over the lattice-DFT bins of both half spaces, dOmega = du dv / |w|, with
 * du = 2 pi / (Lu k pitch), dv = 2 pi / (Lv k pitch): finer bins (larger Lu,
 * Lv) integrate more accurately.
 *   D_dev      double [nrhs][2][Lv][Lu]: half space 0 (w >= 0) then 1 (w < 0);
 *              zero at bins outside the visible region.
 *   prad_host  double [nrhs] (may be NULL): P_rad in units of U.
 * Other arguments as for emsurf_far_field.  EMSURF_ERR_ARG if a right-hand
 * side radiates no power.  Synchronises `stream`. */
emsurf_status emsurf_directivity(const emsurf_geom* geom, int32_t nx, int32_t ny, int32_t nrhs, int32_t Lu,
                                 int32_t Lv, const void* x_dev, void* D_dev, double* prad_host, void* stream);

/* y = T x over nrhs right-hand sides (1 <= nrhs <= max_rhs).  x_dev and y_dev
 * are c128 for EMSURF_FP64 and c64 for EMSURF_FP32, EMSURF_BF16X3 and
 * EMSURF_BF16, [nrhs][ny][nx][n_eq]; they must not overlap.  Requires the
 * matching store in the plan (EMSURF_STORE_BF16 for the split-BF16 forms,
 * which run the FFTs in FP32).  EMSURF_FP32_IR is rejected (EMSURF_ERR_ARG). */
emsurf_status emsurf_apply_T(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                             void* y_dev, void* stream);

/* y = S x (block-diagonal macromodel apply).  Same types and layout as apply_T
 * (the split-BF16 precisions apply S in FP32); x_dev and y_dev may be the same
 * buffer only if they are identical pointers (then the call is out-of-place
 * internally). */
emsurf_status emsurf_apply_S(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                             void* y_dev, void* stream);

/* y = x - S T x.  Same types and layout as apply_T; x_dev and y_dev must not overlap. */
emsurf_status emsurf_apply_A(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                             void* y_dev, void* stream);

/* y = T x exactly as emsurf_apply_T (same kernels, same results), for callers
 * that cannot allocate device memory: code under HIP-graph capture, serving
 * loops, harnesses that forbid hipMalloc.  The call allocates nothing; its
 * intermediates (Ny Lx + 2 Lx Ly values of nrhs n_eq complex numbers in the
 * precision's type, each part rounded up to 256 bytes) live in one static
 * device workspace of emsurf_apply_T_noalloc_limit() bytes (64 MiB) per GPU,
 * held until the process ends.  Larger requests return EMSURF_ERR_ARG.  Every
 * call on one GPU shares that workspace: calls that overlap on a GPU race
 * (serialise them on one stream).  Arguments, layouts and the other errors as
 * for emsurf_apply_T; the plan's own workspaces are not touched. */
emsurf_status emsurf_apply_T_noalloc(emsurf_plan plan, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                                     void* y_dev, void* stream);
size_t emsurf_apply_T_noalloc_limit(void);

/* Solve A x = b for nrhs independent right-hand sides with restarted GMRES
 * (Sec. IV-A).  b_dev, x_dev: c128 [nrhs][ny][nx][n_eq] device.  With use_x0
 * the solve starts from x_dev's content.  info_host: nrhs entries (may be
 * NULL).  Blocks until done.  Returns EMSURF_ERR_NOT_CONVERGED (x holds the
 * best iterate, info filled) if any RHS missed tol; EMSURF_ERR_ARG if b has a
 * non-finite entry.  A zero RHS returns x = 0, converged, 0 iterations.
 * The GMRES workspace ((restart + 1) nrhs basis vectors of c128 and a few
 * vectors more) is kept in the plan for the stream after the first solve on
 * it, grows to the largest nrhs and restart used, is reused by later solves
 * on that stream and freed with the plan (counted in emsurf_plan_query's
 * bytes_total); concurrent solves on one plan must use distinct streams. */
emsurf_status emsurf_solve(emsurf_plan plan, const emsurf_solve_opts* opts, int32_t nrhs,
                           const void* b_dev, void* x_dev, emsurf_solve_info* info_host, void* stream);

/* ---- Near-field right preconditioner (Sec. IV-A, eq. (final_precond)) ----
 * The paper preconditions on the right with P, the entries of the system
 * matrix that couple basis functions closer than Delta_NF (lambda/10 to
 * lambda/6), and applies P^-1 through an LU factorisation.  In the form solved
 * here, A = I - S T, this is
 *     P = I - S T_NF,  T_NF(d)[u][v] = T(d)[u][v] where |r_u - r_v + pitch (dx, dy, 0)| < delta_nf, else 0,
 * r_u the centre of the patch of unknown u (geom->rho; u = tau 2 n_patch +
 * 2 p + alpha).  Each element's own block stays whole in S (the exact inverse
 * of its self block).  delta_nf may reach adjacent elements only (ERR_ARG
 * otherwise).  P is factored on the device per tile of tile_x x tile_y
 * elements (1 <= tile_x tile_y <= 64; tiles from element (0, 0), ragged at
 * the far edges): couplings between tiles are dropped, and a tile that covers
 * the lattice gives the paper's P exactly.
 * T_near: host c128 [3][3][n_eq][n_eq], block [dy + 1][dx + 1] = T(d) row-major
 * [test u][source v] (the plan's own blocks at the 8 neighbour offsets; the
 * centre block is ignored), or NULL to take the point-sampled fill of geom
 * (as emsurf_plan_create_green).  Dense-form plans with an FP64 macromodel
 * copy only.  The preconditioner keeps a pointer to the plan (destroy it
 * first) and owns its device memory (per tile a |Q|^2 c128 matrix, |Q| the
 * tile's unknowns with a near partner in another element of the tile, and a
 * max_rhs vector workspace).  ERR_ARG if a tile's block is singular.  Calls
 * on one preconditioner must not overlap. */
typedef struct emsurf_precond_s* emsurf_precond;
typedef struct {
  int32_t n_tiles, nq_max;    /* tiles, largest near-field unknown set of a tile */
  int64_t near_entries;       /* (u, v, d) triples within delta_nf over the 8 offsets */
  size_t bytes;               /* device bytes held */
  double build_ms;            /* host time of emsurf_precond_create */
} emsurf_precond_stats;
emsurf_status emsurf_precond_create(emsurf_plan plan, const emsurf_geom* geom, double delta_nf, int32_t tile_x,
                                    int32_t tile_y, const void* T_near, void* stream, emsurf_precond* out);
/* x = P^-1 y, c128 [nrhs][ny][nx][n_eq] device, distinct buffers; async on stream. */
emsurf_status emsurf_precond_apply(emsurf_precond pc, int32_t nrhs, const void* y_dev, void* x_dev, void* stream);
emsurf_status emsurf_precond_query(emsurf_precond pc, emsurf_precond_stats* out);
void emsurf_precond_destroy(emsurf_precond pc);
/* emsurf_solve on the right-preconditioned system A P^-1 y = b, x = P^-1 y
 * (the Arnoldi process runs on A P^-1, every cycle ends with x += P^-1 V y,
 * residuals and tol are those of A x = b).  pc must belong to plan.  With
 * EMSURF_FP32_IR the inner solves are preconditioned (P^-1 in FP64). */
emsurf_status emsurf_solve_precond(emsurf_plan plan, emsurf_precond pc, const emsurf_solve_opts* opts, int32_t nrhs,
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

/* ---- Fourier-domain block-product variants and autotuning (FP32 applies) ----
 * EMSURF_BP_GEMV streams each frequency's block with one lane per row (best for
 * few right-hand sides); EMSURF_BP_MFMA_T1..T4 run the per-frequency complex
 * product as a real MFMA GEMM with 1..4 row tiles of 32 per wavefront and 16
 * right-hand sides per pass (n_eq a multiple of 32, at most 480, and at most
 * 4 wavefronts: ceil(n_eq / 32 / k) <= 4; best for many right-hand sides),
 * keeping 4 pairs of block columns in flight per wavefront; the _DEEP forms
 * keep 6 (n_eq a multiple of 96) or 8 (more registers, longer latency cover).  FP64 applies always use the
 * GEMV form. */
#define EMSURF_BP_AUTO (-1)
#define EMSURF_BP_GEMV 0
#define EMSURF_BP_MFMA_T1 1
#define EMSURF_BP_MFMA_T2 2
#define EMSURF_BP_MFMA_T3 3
#define EMSURF_BP_MFMA_T4 4
#define EMSURF_BP_MFMA_T1_DEEP 5
#define EMSURF_BP_MFMA_T2_DEEP 6
#define EMSURF_BP_MFMA_T3_DEEP 7
#define EMSURF_BP_MFMA_T4_DEEP 8
#define EMSURF_BP_NVARIANTS 9

/* Time every FP32 block-product variant for `nrhs` right-hand sides on this
 * plan's blocks (HIP events, 3 launches each after a warm-up; the workspace
 * spectra of `stream` are used as scratch), keep the fastest as the plan's
 * choice for that nrhs and, if the environment variable EMSURF_TUNE_CACHE names
 * a file, record it there ("n_eq nrhs variant" lines) for later processes.
 * ms_out (may be NULL): EMSURF_BP_NVARIANTS entries, -1 for unsupported
 * variants.  best_out (may be NULL) receives the chosen variant.  A reciprocal
 * plan has one kernel, the paired product, timed as variant 0 (no cache
 * entry).  Blocks. */
emsurf_status emsurf_plan_autotune(emsurf_plan plan, int32_t nrhs, double* ms_out, int32_t* best_out,
                                   void* stream);

/* Force the FP32 block-product variant used for `nrhs` right-hand sides
 * (EMSURF_BP_AUTO restores: tuned cache entry, else for nrhs >= 8 the deep
 * MFMA variant with the fewest row tiles that fits, else GEMV).
 * EMSURF_ERR_UNSUPPORTED for an MFMA variant this n_eq cannot run, and for
 * any MFMA variant on a reciprocal plan. */
emsurf_status emsurf_plan_set_variant(emsurf_plan plan, int32_t nrhs, int32_t variant);

/* ---- HIP-graph capture of an apply ----
 * Records the kernels of one apply (op EMSURF_OP_T: y = T x, EMSURF_OP_S:
 * y = S x, EMSURF_OP_A: y = x - S T x) with fixed buffers into a HIP graph on
 * `stream` (must not be the null stream) and instantiates it.  Launching the
 * graph on any stream then recomputes y from the current content of x.  The
 * graph uses the workspace belonging to `stream`: do not overlap a graph
 * launch with other applies issued on that stream.  prec: EMSURF_FP64,
 * EMSURF_FP32, EMSURF_BF16X3 or EMSURF_BF16, as for the applies. */
typedef struct emsurf_graph_s* emsurf_graph;
#define EMSURF_OP_T 0
#define EMSURF_OP_S 1
#define EMSURF_OP_A 2
emsurf_status emsurf_graph_create(emsurf_plan plan, int32_t op, emsurf_prec prec, int32_t nrhs, const void* x_dev,
                                  void* y_dev, void* stream, emsurf_graph* out);
emsurf_status emsurf_graph_launch(emsurf_graph graph, void* stream);
void emsurf_graph_destroy(emsurf_graph graph);

/* ---- Touching fictitious surfaces (Sec. III-D, eqs. (connections_IUI), (final)) ----
 * When the lattice pitch equals the box edge, adjacent boxes share faces and
 * the shared faces' currents are expanded twice.  The paper keeps one set of
 * unknowns through the sparse incidence U_o (Y = U_o Y~) and solves
 * U_o^T [Z_eq + Z_o] U_o Y~ = U_o^T V.  Readings for the point-sampled
 * patches: a patch of element (ix + 1, iy) or (ix, iy + 1) whose centre
 * coincides with a patch of (ix, iy) is a duplicate, with currents
 * x' = -sum_a (t'_b . t_a) x_a for both J and M (continuous tangential fields,
 * opposite outward normals), the face staying with the lower-index element;
 * with ground_plane = 1 the bottom face of every box (the patches with the
 * lowest centres and horizontal tangents) lies on PEC and its M unknowns
 * leave the system.  U_o's columns are the remaining unknowns in increasing
 * full index m n_eq + u.  The coupling fill of such plans evaluates
 * coincident test and source points with the square-patch average of the
 * Green's function (emsurf_plan_create_green).  Z_eq + Z_o is D + T with
 * D = -S^-1 per cell type (the block-Jacobi form), so the reduced operator is
 *     y~ = U_o^T (T U_o x~ - S^-1 U_o x~).
 * The handle keeps a pointer to the plan (destroy the handle first), S^-1 of
 * every type (ERR_ARG if a macromodel is singular) and three max_rhs
 * full-length vectors.  FP64 c128 throughout; calls on one handle must not
 * overlap. */
typedef struct emsurf_overlap_s* emsurf_overlap;
emsurf_status emsurf_overlap_create(emsurf_plan plan, const emsurf_geom* geom, int32_t ground_plane, void* stream,
                                    emsurf_overlap* out);
/* sizes: full unknowns M n_eq, unique unknowns N~, device bytes (each may be NULL) */
emsurf_status emsurf_overlap_query(emsurf_overlap ov, int64_t* n_full, int64_t* n_unique, size_t* bytes);
/* x = U_o x~: x~ c128 [nrhs][N~] -> x c128 [nrhs][M n_eq] (async on stream) */
emsurf_status emsurf_overlap_expand(emsurf_overlap ov, int32_t nrhs, const void* xt_dev, void* x_dev, void* stream);
/* y~ = U_o^T y: y c128 [nrhs][M n_eq] -> y~ c128 [nrhs][N~] (async on stream) */
emsurf_status emsurf_overlap_reduce(emsurf_overlap ov, int32_t nrhs, const void* y_dev, void* yt_dev, void* stream);
/* y~ = U_o^T (D + T) U_o x~, nrhs <= the plan's max_rhs (async on stream) */
emsurf_status emsurf_apply_reduced(emsurf_overlap ov, int32_t nrhs, const void* xt_dev, void* yt_dev, void* stream);
void emsurf_overlap_destroy(emsurf_overlap ov);

/* ---- Continuous-batching sessions (serving) ----
 * A session holds max_slots right-hand-side slots on one plan and its own
 * stream.  emsurf_session_submit places one right-hand side (c128
 * [ny][nx][n_eq], device, copied) into a free slot; emsurf_session_step runs
 * one batched GMRES iteration for every busy slot: slots join and leave at
 * iteration granularity and run at their own Arnoldi index (same algorithm and
 * stopping rule as emsurf_solve; opts.prec EMSURF_FP32_IR runs each cycle's
 * Arnoldi steps with the FP32 operator and every cycle's starting residual
 * with the FP64 operator, aiming each cycle at max(inner_tol * ||r||,
 * tol * ||b|| / 2)).  A slot's numbers never depend on the other slots, so a
 * result is bitwise the same alone and in a mix.  Finished slots keep their
 * solution until emsurf_session_collect copies it out and frees the slot.
 * Calls on one session must not overlap; different sessions may run
 * concurrently (each on its own stream).  The bitwise statement holds for every
 * plan form: dense and structured, full and reciprocal stores. */
typedef struct emsurf_session_s* emsurf_session;
/* device bytes a session with these parameters allocates with every slot in
 * use (slot vectors and Krylov bases, batch staging, reduction buffers) plus
 * an apply workspace for its stream (none is added when the session shares a
 * stream that already has one in the plan).  A slot's vectors and Krylov basis,
 * (restart + 4) unknown vectors, are allocated when the slot is first used and
 * kept for reuse. */
size_t emsurf_session_bytes(emsurf_plan plan, int32_t max_slots, const emsurf_solve_opts* opts);
/* stream NULL: the session creates (and later destroys) its own non-blocking stream. */
emsurf_status emsurf_session_create(emsurf_plan plan, int32_t max_slots, const emsurf_solve_opts* opts, void* stream,
                                    emsurf_session* out);
/* EMSURF_ERR_BUSY if no slot is free.  *slot receives the slot index. */
emsurf_status emsurf_session_submit(emsurf_session session, const void* b_dev, int64_t tag, int32_t* slot);
/* one batched iteration; blocks until its reductions are on the host */
emsurf_status emsurf_session_step(emsurf_session session, int32_t* n_finished);
/* finished, not yet collected slots (up to cap) and their tags; *count = total */
emsurf_status emsurf_session_finished(emsurf_session session, int32_t* slots, int64_t* tags, int32_t cap,
                                      int32_t* count);
emsurf_status emsurf_session_active(emsurf_session session, int32_t* busy_slots);
/* copy the slot's x (c128, may be NULL) and info out, free the slot; EMSURF_ERR_ARG
 * if its right-hand side was not finite.  info->ms = submit-to-finish host time. */
emsurf_status emsurf_session_collect(emsurf_session session, int32_t slot, void* x_dev, emsurf_solve_info* info);
void emsurf_session_destroy(emsurf_session session);

/* ---- Serving loop over many surfaces ----
 * A server accepts solve requests for any number of surfaces.  A surface is
 * identified by a caller key; requests with the same key must describe the
 * same surface (lattice, geometry, macromodels, type map).  Each resident
 * surface has a plan (synthetic point-sampled coupling, FP64 and/or FP32
 * stores per desc.store) and a session with max_slots slots on its own stream.
 * emsurf_server_step admits queued requests whose plan and busy slots fit
 * budget_bytes and whose session has nrhs free slots.  To make room it first
 * releases the vectors of free slots, then evicts idle plans (no active or
 * queued request) least-recently-used first.  Then it runs one batched
 * iteration on every busy session
 * (launching all sessions before waiting for any, so they overlap on the
 * device), and moves finished requests to the completion queue.  All host
 * inputs are copied at submit. */
typedef struct emsurf_server_s* emsurf_server;
typedef struct {
  size_t budget_bytes;        /* device bytes plans + sessions may hold */
  int32_t max_slots;          /* slots per session = largest nrhs of a request, 1..64 */
  uint32_t store;             /* EMSURF_STORE_* of every plan */
  emsurf_solve_opts opts;     /* solve options of every request */
} emsurf_server_desc;
typedef struct {
  int32_t queued, active, resident_plans;
  size_t bytes_used;
  int64_t plans_built, evictions;
  double admit_ms;            /* host time spent admitting (building plans, evicting, uploading b) */
  double step_ms;             /* host time spent in batched iterations (launch to reductions back) */
} emsurf_server_stats;
emsurf_status emsurf_server_create(const emsurf_server_desc* desc, emsurf_server* out);
/* desc: nx, ny, n_eq (= 4 geom->n_patch), n_types (max_rhs, store ignored);
 * S_types, elem_type as for emsurf_plan_create (host); b_host c128
 * [nrhs][ny][nx][n_eq] (host).  *req_id receives the request id. */
emsurf_status emsurf_server_submit(emsurf_server server, uint64_t key, const emsurf_plan_desc* desc,
                                   const emsurf_geom* geom, const void* S_types, const int32_t* elem_type,
                                   int32_t nrhs, const void* b_host, int64_t* req_id);
emsurf_status emsurf_server_step(emsurf_server server, int32_t* n_completed);
/* pop the oldest completed request (*req_id = -1 if none); nrhs and unknowns per RHS */
emsurf_status emsurf_server_next_completed(emsurf_server server, int64_t* req_id, int32_t* nrhs,
                                           int64_t* n_unknowns);
/* copy a completed request's solution (c128 [nrhs][N], host, may be NULL), per-RHS
 * info and times_ms[2] = {submit->admit, submit->done} (may be NULL), then forget it.
 * EMSURF_ERR_ARG if the request could not be solved. */
emsurf_status emsurf_server_fetch(emsurf_server server, int64_t req_id, void* x_host, emsurf_solve_info* info,
                                  double* times_ms);
emsurf_status emsurf_server_query(emsurf_server server, emsurf_server_stats* out);
/* device bytes a resident surface with this desc (nx, ny, n_eq, n_types) holds on
 * this server with no busy right-hand side (plan with its stream's apply
 * workspace, which its session shares, the session's batch staging and
 * reductions, one staging vector), as used for admission; 0 if invalid */
size_t emsurf_server_entry_bytes(emsurf_server server, const emsurf_plan_desc* desc);
/* device bytes each busy right-hand side adds on that surface (its slot's
 * vectors and Krylov basis); 0 if invalid */
size_t emsurf_server_slot_bytes(emsurf_server server, const emsurf_plan_desc* desc);
void emsurf_server_destroy(emsurf_server server);

void emsurf_plan_destroy(emsurf_plan plan);
const char* emsurf_status_str(emsurf_status s);
const char* emsurf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EMSURF_H */
