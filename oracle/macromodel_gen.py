"""Oracle (test infrastructure only): macromodel generation for unique cells.

Paper passages followed (Patel, Triverio, Hum):
* Sec. II-D, eq. (Zmacromodel): the discretised and reduced system of one cell
  is [[Z_eq,eq, Z_eq,int], [Z_int,eq, Z_int,int]] [X_eq; X_int] = 0; the
  interior unknowns are eliminated with the Schur complement,
      Z~ = Z_eq,eq - Z_eq,int Z_int,int^-1 Z_int,eq,
  which needs an LU factorisation of Z_int,int; only unique cells need one
  (Sec. II-D), and cells are independent (parallel).
* Sec. III-A/III-C with the block-Jacobi reading taken here: the element
  operator of (I - S T) x = b is S = -(Z~ + Z_o^self)^-1, Z_o^self being the
  self block of the outer operator (identical for every box).

The interior blocks here are synthetic (the paper's come from its meshes).
Library primitives: numpy.linalg.solve (LAPACK zgesv) and numpy.linalg.inv.
Pins (tests/test_oracle_macromodel_gen.py): an uncoupled interior, 1 x 1
closed forms, the determinant identity det Z = det Z_int,int det Z~, the full
system solved with zero interior excitation, and (Z~ + Z_self) S = -I.
"""
from __future__ import annotations

import numpy as np


def schur_macromodel(Z: np.ndarray, n_eq: int) -> np.ndarray:
    """Z~ of one cell, Z = [[Z_eq,eq, Z_eq,int], [Z_int,eq, Z_int,int]] with
    the n_eq equivalent-surface unknowns first."""
    n = n_eq
    Zee, Zei = Z[:n, :n], Z[:n, n:]
    Zie, Zii = Z[n:, :n], Z[n:, n:]
    if Zii.shape[0] == 0:
        return Zee.copy()
    return Zee - Zei @ np.linalg.solve(Zii, Zie)


def macromodel_S(Zt: np.ndarray, Zself: np.ndarray) -> np.ndarray:
    """S = -(Z~ + Z_self)^-1."""
    return -np.linalg.inv(Zt + Zself)


def macromodels(Z: np.ndarray, n_eq: int, Zself: np.ndarray):
    """Batch over cell types: Z [T][N][N] -> (Z~ [T][n][n], S [T][n][n])."""
    Zt = np.stack([schur_macromodel(z, n_eq) for z in Z])
    S = np.stack([macromodel_S(z, Zself) for z in Zt])
    return Zt, S
