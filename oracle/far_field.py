"""Oracle (test infrastructure only): far field radiated by the equivalent
currents of every box.

Paper passages followed (Patel, Triverio, Hum): Sec. II-A (Love's equivalence:
J and M on each fictitious surface radiate the correct fields outside it) and
Sec. III (the solved unknowns are those currents on every box); the radiated
pattern is what the paper's results compare (Sec. V).

Far field of J and M in free space (eta = 1, e^{jwt}), common factor
-jk e^{-jkr} / (4 pi r) dropped:
    E_theta = N . theta^ + L . phi^,      E_phi = N . phi^ - L . theta^,
    N = sum over sources of A_q J_q e^{jk rhat . r'},  L likewise with M,
with the point-sampled currents used here: on patch q of element m,
J = sum_a xJ[m, q, a] t_qa at r' = rho_q + pitch (ix, iy, 0) (M likewise).
Directions are given by direction cosines (u, v) with w = cos(theta) =
sqrt(1 - u^2 - v^2) >= 0 (upper half space; lower=True takes w <= 0); theta^
and phi^ are the spherical unit vectors, phi = 0 at the zenith.

Directivity (Sec. V plots it in the phi = 0, 45 and 90 degree cuts):
D = 4 pi U / P_rad with U = |E_theta|^2 + |E_phi|^2 (the dropped common
factor cancels).  The paper does not say how it integrates the radiated
power; here P_rad is the midpoint rule in direction cosines over the bins of
the lattice DFT in both half spaces, dOmega = du dv / |w|, the grid on which
the far field is sampled anyway.

Pins (tests/test_oracle_far_field.py): an x-directed electric element and a
y-directed magnetic element in closed form, the array factor of a uniform
lattice (Dirichlet kernels), the translation phase, and linearity.
"""
from __future__ import annotations

import numpy as np


def unit_vectors(u, v, lower: bool = False):
    """rhat, theta^, phi^ for direction cosines (u, v) (arrays), upper half
    space (lower half space with lower=True)."""
    u = np.asarray(u, dtype=float)
    v = np.asarray(v, dtype=float)
    w = np.sqrt(np.maximum(0.0, 1.0 - u * u - v * v))
    if lower:
        w = -w
    st = np.sqrt(u * u + v * v)
    cp = np.where(st > 0, u / np.where(st > 0, st, 1.0), 1.0)
    sp = np.where(st > 0, v / np.where(st > 0, st, 1.0), 0.0)
    rhat = np.stack([u, v, w], axis=-1)
    th = np.stack([w * cp, w * sp, -st], axis=-1)
    ph = np.stack([-sp, cp, np.zeros_like(u)], axis=-1)
    return rhat, th, ph


def far_field(rho, area, tan, pitch: float, k: float, x: np.ndarray, u, v, lower: bool = False) -> np.ndarray:
    """E_theta, E_phi for every right-hand side of x ([nrhs][ny][nx][n_eq],
    n_eq = 4 P, J unknowns first) at directions (u, v) (1-D arrays of equal
    length): complex128 [nrhs][ndir][2]."""
    nrhs, ny, nx, n = x.shape
    P = rho.shape[0]
    rhat, th, ph = unit_vectors(u, v, lower)                            # [d][3]
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    R = np.stack([pitch * ix, pitch * iy, np.zeros_like(ix, dtype=float)], axis=-1).reshape(-1, 3)  # [m][3]
    pos = R[:, None, :] + rho[None, :, :]                               # [m][q][3]
    phase = np.exp(1j * k * np.einsum("di,mqi->dmq", rhat, pos)) * area[None, None, :]   # [d][m][q]
    xm = x.reshape(nrhs, ny * nx, n)
    xJ = xm[:, :, : 2 * P].reshape(nrhs, ny * nx, P, 2)
    xM = xm[:, :, 2 * P:].reshape(nrhs, ny * nx, P, 2)
    # current vectors per source: sum_a x[.., q, a] t_qa
    Jv = np.einsum("rmqa,qai->rmqi", xJ, tan)
    Mv = np.einsum("rmqa,qai->rmqi", xM, tan)
    N = np.einsum("dmq,rmqi->rdi", phase, Jv)
    L = np.einsum("dmq,rmqi->rdi", phase, Mv)
    out = np.zeros((nrhs, len(np.atleast_1d(u)), 2), dtype=np.complex128)
    out[:, :, 0] = np.einsum("rdi,di->rd", N, th) + np.einsum("rdi,di->rd", L, ph)
    out[:, :, 1] = np.einsum("rdi,di->rd", N, ph) - np.einsum("rdi,di->rd", L, th)
    return out


def fft_bin_directions(Lu: int, Lv: int, pitch: float, k: float):
    """Direction cosines of the bins of an Lu x Lv lattice DFT with kernel
    e^{+j 2 pi (p ix / Lu + q iy / Lv)}: k pitch u = 2 pi p' / Lu with p' the
    signed bin index; returns (u, v) arrays [Lv][Lu] (bin q, p)."""
    p = np.arange(Lu)
    q = np.arange(Lv)
    ps = np.where(p < (Lu + 1) // 2, p, p - Lu)
    qs = np.where(q < (Lv + 1) // 2, q, q - Lv)
    u = 2.0 * np.pi * ps / (Lu * k * pitch)
    v = 2.0 * np.pi * qs / (Lv * k * pitch)
    return np.broadcast_to(u[None, :], (Lv, Lu)).copy(), np.broadcast_to(v[:, None], (Lv, Lu)).copy()


def directivity(rho, area, tan, pitch: float, k: float, x: np.ndarray, Lu: int, Lv: int):
    """Directivity at the bins of an Lu x Lv lattice DFT in both half spaces.

    Returns (D, P_rad): D float64 [nrhs][2][Lv][Lu] (half space 0: w >= 0,
    1: w < 0; zero at bins outside the visible region u^2 + v^2 < 1) and
    P_rad [nrhs] = sum over both half spaces and visible bins of
    U du dv / |w|, U = |E_theta|^2 + |E_phi|^2, du = 2 pi / (Lu k pitch),
    dv = 2 pi / (Lv k pitch); D = 4 pi U / P_rad."""
    nrhs = x.shape[0]
    u, v = fft_bin_directions(Lu, Lv, pitch, k)
    vis = u * u + v * v < 1.0
    du = 2.0 * np.pi / (Lu * k * pitch)
    dv = 2.0 * np.pi / (Lv * k * pitch)
    w = np.sqrt(np.where(vis, 1.0 - u * u - v * v, 1.0))
    U = np.zeros((nrhs, 2, Lv, Lu))
    for h in range(2):
        E = far_field(rho, area, tan, pitch, k, x, u[vis], v[vis], lower=h == 1)
        U[:, h][:, vis] = np.sum(np.abs(E) ** 2, axis=-1)
    P_rad = np.sum(U * np.where(vis, du * dv / w, 0.0)[None, None], axis=(1, 2, 3))
    return 4.0 * np.pi * U / P_rad[:, None, None, None], P_rad
