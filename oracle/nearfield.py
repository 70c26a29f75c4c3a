"""Oracle (test infrastructure only): the near-field right preconditioner of
Sec. IV-A, eq. (final_precond), in the block-Jacobi form of the solve.

The paper preconditions its final system on the right with P, the part of the
system matrix whose entries couple basis functions closer than Delta_NF
(lambda/10 to lambda/6), and applies P^-1 through an LU factorisation.  In the
form solved here, A = I - S T with S = -(Z_eq + Z_o^self)^-1 the per-element
macromodels and T the mutual coupling (T(0) = 0), the same construction reads

    P = I - S T_NF,    T_NF(d)[u][v] = T(d)[u][v]  if |r_u - r_v - pitch d| < Delta_NF,
                                       0            otherwise,

with r_u the centre of the patch carrying unknown u (both tangents and both
currents of a patch share it).  The element's own block is kept whole: S holds
the exact inverse of the element's self block, which contains every near-field
entry of that block.  The right-preconditioned system is A P^-1 y = b, x = P^-1 y.

The paper factors P over the whole surface.  Here P may also be factored per
tile of tile_x x tile_y elements (block Jacobi over the tiles of P: the
near-field couplings between different tiles are dropped); a tile that covers
the lattice is exactly the paper's P.  P^-1 is applied tile by tile as the
dense LU solve of that tile's block (LAPACK zgesv), its plain definition.

Pins (tests/test_oracle_nearfield.py): the count of near pairs at lambda/10 on
the synthetic box in closed form; mask(-d) = mask(d)^T; Delta_NF = 0 gives
P = I and the unpreconditioned iterates; a Delta_NF that reaches every pair of
a 2-element or 2 x 2 lattice gives P = A, so preconditioned GMRES stops after
one step with the LU solution; the block structure of the tiled P^-1; and
unchanged solutions against LU.
"""
from __future__ import annotations

import numpy as np

from . import macromodel as MM

OFFSETS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def unknown_patch(n_patch: int) -> np.ndarray:
    """Patch index of each local unknown u = tau (2 P) + 2 p + alpha."""
    u = np.arange(4 * n_patch)
    return (u % (2 * n_patch)) // 2


def near_field_mask(rho: np.ndarray, pitch: float, delta: float, dy: int, dx: int) -> np.ndarray:
    """[n][n] booleans: test unknown u of the element at offset d = (dy, dx)
    from the source element, source unknown v, patch centres closer than delta."""
    P = rho.shape[0]
    shift = np.array([pitch * dx, pitch * dy, 0.0])
    disp = rho[:, None, :] - rho[None, :, :] + shift          # [p_test][q_source][3]
    near = np.sqrt(np.sum(disp * disp, axis=-1)) < delta        # [P][P]
    pu = unknown_patch(P)
    return near[pu[:, None], pu[None, :]]


def reaches_beyond_neighbours(rho: np.ndarray, pitch: float, delta: float) -> bool:
    """True if some pair of patches two or more lattice steps apart is closer
    than delta (the tiled preconditioner couples adjacent elements only)."""
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            if max(abs(dy), abs(dx)) == 2 and near_field_mask(rho, pitch, delta, dy, dx).any():
                return True
    return False


def near_field_blocks(T_of, rho: np.ndarray, pitch: float, delta: float, nx: int = 2, ny: int = 2) -> dict:
    """T_NF(d) for the neighbour offsets a nx x ny lattice has: T(d) where the
    mask holds, else 0."""
    out = {}
    for dy, dx in OFFSETS:
        if (dy, dx) == (0, 0) or abs(dx) >= nx or abs(dy) >= ny:
            continue
        out[(dy, dx)] = np.where(near_field_mask(rho, pitch, delta, dy, dx), T_of(dy, dx), 0.0)
    return out


def tiles(nx: int, ny: int, tile_x: int, tile_y: int):
    """Elements (iy, ix) of every tile, tiles in row-major order of their corner."""
    out = []
    for ty0 in range(0, ny, tile_y):
        for tx0 in range(0, nx, tile_x):
            out.append([(iy, ix) for iy in range(ty0, min(ny, ty0 + tile_y))
                        for ix in range(tx0, min(nx, tx0 + tile_x))])
    return out


def tile_matrix(S: np.ndarray, tm: np.ndarray, Tnf: dict, elems) -> np.ndarray:
    """Dense block of P = I - S T_NF over the elements of one tile (in the
    given order): block (a, b) = delta_ab I - S_type(a) T_NF(pos(a) - pos(b))."""
    n = S.shape[-1]
    k = len(elems)
    Pm = np.eye(k * n, dtype=np.complex128)
    for a, (iya, ixa) in enumerate(elems):
        Sa = S[tm[iya, ixa]]
        for b, (iyb, ixb) in enumerate(elems):
            d = (iya - iyb, ixa - ixb)
            if d == (0, 0) or d not in Tnf:
                continue
            Pm[a * n:(a + 1) * n, b * n:(b + 1) * n] -= Sa @ Tnf[d]
    return Pm


def dense_P(S: np.ndarray, tm: np.ndarray, Tnf: dict, nx: int, ny: int) -> np.ndarray:
    """The whole P over the lattice, elements m = iy nx + ix (small lattices)."""
    return tile_matrix(S, tm, Tnf, [(iy, ix) for iy in range(ny) for ix in range(nx)])


def apply_Pinv(S: np.ndarray, tm: np.ndarray, Tnf: dict, tile_x: int, tile_y: int, y: np.ndarray) -> np.ndarray:
    """x = P^-1 y for the tiled P, one dense LU solve per tile.
    y, x: [nrhs][ny][nx][n]."""
    nrhs, ny, nx, n = y.shape
    x = np.zeros_like(y, dtype=np.complex128)
    for elems in tiles(nx, ny, tile_x, tile_y):
        Pm = tile_matrix(S, tm, Tnf, elems)
        rows = np.stack([y[:, iy, ix, :] for iy, ix in elems], axis=1).reshape(nrhs, -1)   # [r][k n]
        sol = np.linalg.solve(Pm, rows.T).T.reshape(nrhs, len(elems), n)
        for a, (iy, ix) in enumerate(elems):
            x[:, iy, ix, :] = sol[:, a]
    return x


def apply_A_fn(T_apply, S, tm):
    """x -> x - S T x on [nrhs][ny][nx][n] arrays (the unpreconditioned operator)."""
    return lambda x: MM.apply_A(T_apply, S, tm, x)
