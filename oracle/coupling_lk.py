"""Oracle (test infrastructure only): the outer operator in the paper's own
structured form, discretised L and K operators shared by the four quadrants.

Paper passages followed (Patel, Triverio, Hum):
* Sec. III-B, eqs. (SIE_TEFIE1_Outer)/(SIE_TMFIE1_Outer): the outer EFIE and
  MFIE couple the equivalent currents through the free-space L and K
  operators; eq. (blockZo): the coupling block of two boxes is
  [[L^E, K^E], [K^H, L^H]], rows tested on box m, columns sourced on box m'.
* Sec. IV-B: Z_o x is evaluated by multiplying the discretised L and K
  operators, scaled by constants, with blocks of x; both are Toeplitz.
* Sec. IV-C: the method stores 2^{d+1} N_eq^2 M numbers, i.e. the two N_eq x
  N_eq operators L and K per padded lattice offset, not the four quadrants.

Synthetic content (the paper's are Galerkin RWG integrals that need its
meshes; this stand-in point-matches at the test patch centre with one-point
quadrature over the source patch, as the dense stand-in in coupling.py does):

    L(d)[(p,a),(q,b)] = A_q  t_pa . (I + grad grad / k^2) g(R) . t_qb
    K(d)[(p,a),(q,b)] = A_q  t_pa . (grad g(R) x t_qb)

with R = rho_p - rho_q + pitch (dx, dy, 0) (test minus source), grad acting on
the test point, g(R) = exp(-jkR)/(4 pi R), and L(0) = K(0) = 0.  The coupling
block is T(d) = [[a L, b K], [c K, e L]] with J rows/columns first; the
EFIE/MFIE constants with eta = 1 are a = -jk, b = 1, c = -1, e = jk.

Pins (tests/test_oracle_lk.py): finite-difference derivatives of the scalar
Green's function, the far-field (transverse) limit, the reciprocity identities
L(-d)^T = D L(d) D^-1 and K(-d)^T = D K(d) D^-1 (D = source-area diagonal),
K = 0 between parallel tangents along the separation, and T(0) = 0.  The
physical accuracy of the point-sampled stand-in is "parity unpinned".
"""
from __future__ import annotations

import numpy as np


def green_radial(R: np.ndarray, k: float):
    """g, dg/dR and d2g/dR2 of g(R) = exp(-jkR)/(4 pi R)."""
    g = np.exp(-1j * k * R) / (4.0 * np.pi * R)
    a = 1j * k + 1.0 / R
    return g, -a * g, (a * a + 1.0 / (R * R)) * g


def paper_coefficients(k: float):
    """(a, b, c, e) of T = [[a L, b K], [c K, e L]] from the outer EFIE and MFIE
    with eta = 1 (Sec. III-B): -j omega mu0 = -jk, +K, -K, +j omega eps0 = jk."""
    return (-1j * k, 1.0 + 0j, -1.0 + 0j, 1j * k)


def lk_blocks_at(rho, area, tan, offsets, pitch: float, k: float):
    """L(d) and K(d) for every offset d = (dy, dx) in `offsets`: two complex128
    arrays [n_off][n_h][n_h], n_h = 2 n_patch, local index 2p + a."""
    offsets = np.asarray(offsets, dtype=np.int64).reshape(-1, 2)
    P = rho.shape[0]
    nh = 2 * P
    shift = np.zeros((offsets.shape[0], 3))
    shift[:, 0] = pitch * offsets[:, 1]
    shift[:, 1] = pitch * offsets[:, 0]
    disp = rho[None, :, None, :] - rho[None, None, :, :] + shift[:, None, None, :]   # [o][p][q][3]
    R = np.sqrt(np.sum(disp * disp, axis=-1))
    self_mask = (offsets[:, 0] == 0) & (offsets[:, 1] == 0)
    R[self_mask] = 1.0                                   # values discarded below
    Rhat = disp / R[..., None]
    g, g1, g2 = green_radial(R, k)
    iso = g + g1 / (k * k * R)                           # coefficient of I
    rad = (g2 - g1 / R) / (k * k)                        # coefficient of Rhat Rhat
    tt = np.einsum("pai,qbi->paqb", tan, tan)                    # t_pa . t_qb
    tR_test = np.einsum("pai,opqi->opqa", tan, Rhat)              # t_pa . Rhat
    tR_src = np.einsum("qbi,opqi->opqb", tan, Rhat)               # t_qb . Rhat
    L = (iso[:, :, None, :, None] * tt[None]
         + rad[:, :, None, :, None] * np.einsum("opqa,opqb->opaqb", tR_test, tR_src))
    L = L * area[None, None, None, :, None]
    # grad g = g'(R) Rhat; entry t_pa . (Rhat x t_qb)
    Rxt = np.cross(Rhat[:, :, :, None, :], tan[None, None, :, :, :])      # [o][p][q][b][3]
    K = np.einsum("pai,opqbi->opaqb", tan, Rxt) * g1[:, :, None, :, None] * area[None, None, None, :, None]
    L = L.reshape(offsets.shape[0], nh, nh)
    K = K.reshape(offsets.shape[0], nh, nh)
    L[self_mask] = 0.0
    K[self_mask] = 0.0
    return L, K


def lk_blocks(rho, area, tan, nx: int, ny: int, pitch: float, k: float):
    """All offsets, [2ny-1][2nx-1][n_h][n_h] each, indexed [dy+ny-1][dx+nx-1]."""
    from .coupling import all_offsets
    nh = 2 * rho.shape[0]
    L, K = lk_blocks_at(rho, area, tan, all_offsets(nx, ny), pitch, k)
    return L.reshape(2 * ny - 1, 2 * nx - 1, nh, nh), K.reshape(2 * ny - 1, 2 * nx - 1, nh, nh)


def lk_assemble(L: np.ndarray, K: np.ndarray, coef) -> np.ndarray:
    """Dense coupling blocks T = [[a L, b K], [c K, e L]] (eq. (blockZo)),
    same leading offset axes as L and K, n_eq = 2 n_h."""
    a, b, c, e = coef
    top = np.concatenate([a * L, b * K], axis=-1)
    bot = np.concatenate([c * K, e * L], axis=-1)
    return np.concatenate([top, bot], axis=-2)


def apply_T_elements_lk(rho, area, tan, pitch: float, k: float, coef, x: np.ndarray, elems, chunk_rows: int = 1):
    """Rows of y = T x at sampled output elements, every L and K block of the
    row generated on the fly and assembled into [[a L, b K], [c K, e L]]:
    y[m] = sum_{m'} T(m - m') x[m'].  x: [nrhs][ny][nx][n_eq]; returns
    complex128 [len(elems)][nrhs][n_eq]."""
    nrhs, ny, nx, n = x.shape
    out = np.zeros((len(elems), nrhs, n), dtype=np.complex128)
    jx = np.arange(nx)
    for e, (iy, ix) in enumerate(elems):
        acc = np.zeros((nrhs, n), dtype=np.complex128)
        for jy0 in range(0, ny, chunk_rows):
            jys = np.arange(jy0, min(ny, jy0 + chunk_rows))
            offs = np.stack(np.broadcast_arrays((iy - jys)[:, None], (ix - jx)[None, :]), axis=-1).reshape(-1, 2)
            L, K = lk_blocks_at(rho, area, tan, offs, pitch, k)
            blk = lk_assemble(L, K, coef)                                  # [o][n][n]
            src = x[:, jys, :, :].reshape(nrhs, -1, n)                     # [r][o][n]
            acc += np.einsum("ouv,rov->ru", blk, src)
        out[e] = acc
    return out
