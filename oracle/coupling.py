"""Oracle: the free-space coupling operator T between the fictitious boxes.

Paper passages followed (Patel, Triverio, Hum):
* Sec. III-B, eqs. (out)/(blockZo): the outer problem couples every pair of
  boxes (m, m') with a dense block whose rows are tested on box m and whose
  columns are sources on box m'.
* Sec. IV-A/IV-B: identical meshes on every box, constant lattice pitch and a
  translation-invariant Green's function make this block depend only on the
  lattice offset d = (test element) - (source element); the whole matrix is
  block-Toeplitz.  The index convention L_mn = (test m, source n) of the 1-D
  example in Sec. IV-B fixes the sign of d.

Synthetic block content (the paper's blocks are Galerkin RWG reaction
integrals, which need its meshes; this implementation uses a point-sampled stand-in):

    T(d)[(tau,p,a),(tau',q,b)] = delta(tau,tau') (t_pa . t_qb) A_q g(R),
    R = | rho_p - rho_q + pitch (dx, dy, 0) |,  g(R) = exp(-j k R) / (4 pi R),

tested at the centre of patch p on the test box, one-point quadrature over
source patch q; J couples to J and M to M only; T(0) = 0 (the self term of a
box belongs to its macromodel).  When boxes touch (Sec. III-D: pitch equal
to the box edge), patches of a shared face coincide (R = 0); there A_q g(R)
is replaced by its average over a square source patch of the same area,
    (4 a ln(1 + sqrt 2) - j k a^2) / (4 pi),   a = sqrt(A_q),
the integral of 1/(4 pi R) over the square about its centre plus the first
term of (exp(-jkR) - 1) / (4 pi R).

Parity: pinned by closed-form entries (facing patches across the 0.05 gap,
patch pairs at exactly one pitch), reciprocity of the Green's function, the
Toeplitz shift invariance, the paper's 1-D circulant example rebuilt with a
library FFT, and a library 2-D FFT convolution (tests/test_oracle_coupling.py).
The physical accuracy of the point-sampled stand-in itself is "parity
unpinned": no published values exist for it.
"""
from __future__ import annotations

import numpy as np


def green(R: np.ndarray, k: float) -> np.ndarray:
    """Scalar free-space Green's function exp(-jkR)/(4 pi R) (e^{+jwt} convention)."""
    return np.exp(-1j * k * R) / (4.0 * np.pi * R)


def coincident_patch_term(A, k: float):
    """A g(R) for a test point at the centre of its own (square) source patch of
    area A: (4 a ln(1 + sqrt 2) - j k a^2) / (4 pi), a = sqrt(A)."""
    a = np.sqrt(A)
    return (4.0 * a * np.log(1.0 + np.sqrt(2.0)) - 1j * k * a * a) / (4.0 * np.pi)


def tangent_products(tan: np.ndarray) -> np.ndarray:
    """(t_pa . t_qb) as a [2P][2P] matrix over local indices 2p+a."""
    P = tan.shape[0]
    tt = np.einsum("pai,qbi->paqb", tan, tan)
    return tt.reshape(2 * P, 2 * P)


def coupling_blocks_at(rho, area, tan, offsets, pitch: float, k: float) -> np.ndarray:
    """T(d) for every offset d = (dy, dx) in `offsets` ([n_off][2] ints).

    Returns complex128 [n_off][n_eq][n_eq] with n_eq = 4 * n_patch; the block
    for d = (0, 0) is zero."""
    offsets = np.asarray(offsets, dtype=np.int64).reshape(-1, 2)
    P = rho.shape[0]
    n = 4 * P
    shift = np.zeros((offsets.shape[0], 3))
    shift[:, 0] = pitch * offsets[:, 1]
    shift[:, 1] = pitch * offsets[:, 0]
    disp = rho[None, :, None, :] - rho[None, None, :, :] + shift[:, None, None, :]   # [o][p][q][3]
    R = np.sqrt(np.sum(disp * disp, axis=-1))
    self_mask = (offsets[:, 0] == 0) & (offsets[:, 1] == 0)
    R[self_mask] = 1.0                      # value discarded below
    touch = R <= 1e-9 * np.sqrt(area)[None, None, :]
    G = green(np.where(touch, 1.0, R), k) * area[None, None, :]   # [o][p][q], weighted by the source area
    G = np.where(touch, coincident_patch_term(area, k)[None, None, :], G)
    G[self_mask] = 0.0
    tt = tangent_products(tan)              # [2P][2P]
    half = G[:, :, None, :, None] * tt.reshape(P, 2, P, 2)[None]   # [o][p][a][q][b]
    half = half.reshape(offsets.shape[0], 2 * P, 2 * P)
    out = np.zeros((offsets.shape[0], n, n), dtype=np.complex128)
    out[:, : 2 * P, : 2 * P] = half         # J <- J
    out[:, 2 * P :, 2 * P :] = half         # M <- M
    return out


def coupling_block(rho, area, tan, dy: int, dx: int, pitch: float, k: float) -> np.ndarray:
    return coupling_blocks_at(rho, area, tan, [(dy, dx)], pitch, k)[0]


def all_offsets(nx: int, ny: int) -> np.ndarray:
    """Every lattice offset, ordered [dy + ny - 1][dx + nx - 1]."""
    dy, dx = np.meshgrid(np.arange(-(ny - 1), ny), np.arange(-(nx - 1), nx), indexing="ij")
    return np.stack([dy.ravel(), dx.ravel()], axis=1)


def coupling_blocks(rho, area, tan, nx: int, ny: int, pitch: float, k: float) -> np.ndarray:
    """All blocks, complex128 [2ny-1][2nx-1][n_eq][n_eq] indexed [dy+ny-1][dx+nx-1]."""
    n = 4 * rho.shape[0]
    blk = coupling_blocks_at(rho, area, tan, all_offsets(nx, ny), pitch, k)
    return blk.reshape(2 * ny - 1, 2 * nx - 1, n, n)


def dense_T(blocks: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """Assemble the dense M n_eq x M n_eq matrix: block (m, m') = T(m - m'),
    m = iy*nx + ix (Sec. III-B; Toeplitz by Sec. IV-A)."""
    n = blocks.shape[-1]
    M = nx * ny
    T = np.zeros((M * n, M * n), dtype=np.complex128)
    for iy in range(ny):
        for ix in range(nx):
            m = iy * nx + ix
            for jy in range(ny):
                for jx in range(nx):
                    mp = jy * nx + jx
                    T[m * n:(m + 1) * n, mp * n:(mp + 1) * n] = blocks[iy - jy + ny - 1, ix - jx + nx - 1]
    return T


def apply_T_dense(blocks: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = T x with T formed densely.  x, y: [nrhs][ny][nx][n_eq]."""
    nrhs, ny, nx, n = x.shape
    T = dense_T(blocks, nx, ny)
    y = x.reshape(nrhs, -1) @ T.T
    return y.reshape(x.shape)


def apply_T_direct(block_of, x: np.ndarray) -> np.ndarray:
    """y = T x as a direct sum over lattice offsets, never forming T:
    y[m] += T(d) x[m - d] for every offset d and every element m whose source
    m - d lies inside the lattice.  `block_of(dy, dx)` returns T(d)."""
    nrhs, ny, nx, n = x.shape
    y = np.zeros_like(x, dtype=np.complex128)
    for dy in range(-(ny - 1), ny):
        ty0, ty1 = max(0, dy), min(ny, ny + dy)
        for dx in range(-(nx - 1), nx):
            tx0, tx1 = max(0, dx), min(nx, nx + dx)
            blk = block_of(dy, dx)
            src = x[:, ty0 - dy:ty1 - dy, tx0 - dx:tx1 - dx, :]
            y[:, ty0:ty1, tx0:tx1, :] += src @ blk.T
    return y


def apply_T_elements(rho, area, tan, pitch: float, k: float, x: np.ndarray, elems, chunk_rows: int = 1):
    """Rows of y = T x for a sample of output elements only, with the blocks
    generated on the fly: y[m] = sum_{m'} T(m - m') x[m'].

    `elems` is a list of (iy, ix).  Returns complex128 [len(elems)][nrhs][n_eq].
    Cost per element: M blocks of n_eq^2 (fill + multiply)."""
    nrhs, ny, nx, n = x.shape
    out = np.zeros((len(elems), nrhs, n), dtype=np.complex128)
    jx = np.arange(nx)
    for e, (iy, ix) in enumerate(elems):
        acc = np.zeros((nrhs, n), dtype=np.complex128)
        for jy0 in range(0, ny, chunk_rows):
            jys = np.arange(jy0, min(ny, jy0 + chunk_rows))
            offs = np.stack(np.broadcast_arrays((iy - jys)[:, None], (ix - jx)[None, :]), axis=-1).reshape(-1, 2)
            blk = coupling_blocks_at(rho, area, tan, offs, pitch, k)           # [o][n][n]
            src = x[:, jys, :, :].reshape(nrhs, -1, n)                         # [r][o][n]
            acc += np.einsum("ouv,rov->ru", blk, src)
        out[e] = acc
    return out


def apply_T_elements_from_blocks(blocks: np.ndarray, x: np.ndarray, elems):
    """Same as apply_T_elements, reading T(d) from a stored block array."""
    nrhs, ny, nx, n = x.shape
    out = np.zeros((len(elems), nrhs, n), dtype=np.complex128)
    for e, (iy, ix) in enumerate(elems):
        for jy in range(ny):
            for jx in range(nx):
                out[e] += x[:, jy, jx, :] @ blocks[iy - jy + ny - 1, ix - jx + nx - 1].T
    return out
