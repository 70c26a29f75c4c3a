"""Oracle: the block-diagonal macromodel operator S and A = I - S T.

Paper passages followed:
* Sec. III-A, eq. (Zmacromodel_Array): the array's macromodel matrix is
  block-diagonal with one dense block per element acting on that element's
  equivalent currents only; the unknown vector stacks the elements in order.
* Sec. II-D (end): macromodels are needed for unique cells only, so elements
  of one cell type share one block.
* Sec. III-C, eq. (out3), summed with the outer equations, and the split of
  the coupling matrix into its self blocks and its mutual blocks: with
  D = Z_eq + Z_o^self (block-diagonal, one block per cell type) and
  T = Z_o^mut, left-multiplying by D^-1 turns (Z_eq + Z_o) Y = V into
  (I - S T) Y = D^-1 V with S = -D^-1.  The library and this oracle take S
  and T as given.

Parity: S pinned against a library block-diagonal assembly and identity /
scaled-identity special cases; A pinned through the closed-form solves
(single element, single scatterer, two elements) and dense LU.
"""
from __future__ import annotations

import numpy as np


def apply_S(S_types: np.ndarray, type_map: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y[r, m] = S_{type(m)} x[r, m]; x, y [nrhs][ny][nx][n_eq], S_types [T][n][n]."""
    S_elem = S_types[type_map]                        # [ny][nx][n][n]
    return np.einsum("yxuv,ryxv->ryxu", S_elem, x)


def apply_A(apply_T, S_types: np.ndarray, type_map: np.ndarray, x: np.ndarray) -> np.ndarray:
    """A x = x - S (T x)."""
    return x - apply_S(S_types, type_map, apply_T(x))


def dense_S(S_types: np.ndarray, type_map: np.ndarray) -> np.ndarray:
    ny, nx = type_map.shape
    n = S_types.shape[-1]
    M = nx * ny
    S = np.zeros((M * n, M * n), dtype=np.complex128)
    for m, t in enumerate(type_map.ravel()):
        S[m * n:(m + 1) * n, m * n:(m + 1) * n] = S_types[t]
    return S
