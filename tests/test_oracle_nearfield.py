"""Pins of the near-field preconditioner oracle (Sec. IV-A, eq. (final_precond))
against closed-form geometry counts, special cases that reduce P to I or to A,
the block structure of the tiled factorisation, and dense LU."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM
from oracle import nearfield as NF

LAM10 = 0.1 * W.WAVELENGTH


def _surface(nx, ny, npch=24, n_types=3, seed=0):
    g = W.box_geometry(npch)
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    S = W.random_types(n_types, g.n_eq, seed=seed)
    tm = W.random_type_map(nx, ny, n_types, seed=seed)
    T_of = lambda dy, dx: B[dy + ny - 1, dx + nx - 1]
    return g, B, S, tm, T_of


def test_near_pairs_at_lambda_over_10_closed_form():
    # 24 patches, side faces of 2 x 2 patches (0.225 along the edge, 0.05 high),
    # gap 0.05 between facing side faces: each side patch is within lambda/10 of
    # the facing patch (0.05) and of the one above or below it (sqrt(2) 0.05),
    # not of the one along the edge (0.23); a near patch pair gives 4 x 4
    # unknown pairs (2 currents x 2 tangents on either side)
    g = W.box_geometry(24)
    for d in [(0, 1), (0, -1), (1, 0), (-1, 0)]:
        m = NF.near_field_mask(g.rho, W.PITCH, LAM10, *d)
        assert m.sum() == 4 * 2 * 16
    for d in [(1, 1), (-1, 1), (1, -1), (-1, -1)]:
        assert not NF.near_field_mask(g.rho, W.PITCH, LAM10, *d).any()
    # 48 patches: side faces of 4 x 1 patches (0.1125 x 0.1): only the facing patch
    g = W.box_geometry(48)
    assert NF.near_field_mask(g.rho, W.PITCH, LAM10, 0, 1).sum() == 4 * 1 * 16
    # lambda/6 reaches the diagonal neighbours' corner patches but never two steps away
    assert NF.near_field_mask(g.rho, W.PITCH, W.WAVELENGTH / 6, 1, 1).sum() > 0
    assert not NF.reaches_beyond_neighbours(g.rho, W.PITCH, W.WAVELENGTH / 6)
    assert NF.reaches_beyond_neighbours(g.rho, W.PITCH, 0.8)


def test_mask_transposes_under_offset_negation():
    g = W.box_geometry(72)
    for d in NF.OFFSETS:
        a = NF.near_field_mask(g.rho, W.PITCH, 0.15, *d)
        b = NF.near_field_mask(g.rho, W.PITCH, 0.15, -d[0], -d[1])
        assert np.array_equal(a, b.T)


def test_zero_distance_gives_identity_and_the_plain_iterates():
    nx, ny = 3, 2
    g, B, S, tm, T_of = _surface(nx, ny, seed=1)
    Tnf = NF.near_field_blocks(T_of, g.rho, W.PITCH, 0.0)
    assert all(not np.any(v) for v in Tnf.values())
    y = W.random_vectors(2, nx, ny, g.n_eq, seed=3)
    assert np.allclose(NF.apply_Pinv(S, tm, Tnf, 2, 2, y), y, rtol=0, atol=1e-15)
    Tf = lambda v: C.apply_T_dense(B, v)
    Af = lambda v: MM.apply_A(Tf, S, tm, v.reshape(y[:1].shape)).ravel()
    b = y[0].ravel()
    x0, i0 = K.gmres(Af, b, 1e-12)
    x1, i1 = K.gmres(Af, b, 1e-12, M_inv=lambda v: v)
    assert i0.iters == i1.iters and np.array_equal(x0, x1)


@pytest.mark.parametrize("nx,ny", [(2, 1), (1, 2), (2, 2)])
def test_far_reaching_distance_gives_P_equal_A(nx, ny):
    # every pair of patches of adjacent (and, on 2 x 2, diagonal) elements is
    # within Delta, so T_NF = T and one tile covering the lattice makes P = A:
    # the preconditioned operator is I and GMRES stops after one step at the LU solution
    g, B, S, tm, T_of = _surface(nx, ny, seed=4)
    Tnf = NF.near_field_blocks(T_of, g.rho, W.PITCH, 10.0, nx, ny)
    A = np.eye(nx * ny * g.n_eq) - MM.dense_S(S, tm) @ C.dense_T(B, nx, ny)
    Pd = NF.dense_P(S, tm, Tnf, nx, ny)
    assert np.allclose(Pd, A, rtol=0, atol=1e-14)
    b = W.plane_wave_rhs(W.small_config(nx, ny, 24, 3, 1, seed=2), g)
    shape = b.shape
    Af = lambda v: MM.apply_A(lambda z: C.apply_T_dense(B, z), S, tm, v.reshape(shape)).ravel()
    Minv = lambda v: NF.apply_Pinv(S, tm, Tnf, nx, ny, v.reshape(shape)).ravel()
    x, info = K.gmres(Af, b.ravel(), 1e-12, M_inv=Minv)
    x_lu = K.solve_dense(A, b.ravel())
    assert info.iters == 1 and np.linalg.norm(x - x_lu) <= 1e-13 * np.linalg.norm(x_lu)


def test_tiled_inverse_is_block_diagonal_over_tiles_and_exact_on_one_tile():
    nx, ny, tx, ty = 5, 3, 2, 2
    g, B, S, tm, T_of = _surface(nx, ny, seed=5)
    Tnf = NF.near_field_blocks(T_of, g.rho, W.PITCH, 0.15)
    n = g.n_eq
    # a vector supported on one tile maps into that tile only
    y = np.zeros((1, ny, nx, n), complex)
    y[0, 0:2, 2:4, :] = W.random_vectors(1, 2, 2, n, seed=6)[0]
    x = NF.apply_Pinv(S, tm, Tnf, tx, ty, y)
    outside = np.ones((ny, nx), bool)
    outside[0:2, 2:4] = False
    assert not np.any(x[0][outside])
    # tile = lattice: the dense LU of the whole P
    y = W.random_vectors(2, nx, ny, n, seed=7)
    Pd = NF.dense_P(S, tm, Tnf, nx, ny)
    x = NF.apply_Pinv(S, tm, Tnf, nx, ny, y)
    assert np.linalg.norm((Pd @ x.reshape(2, -1).T).T - y.reshape(2, -1)) <= 1e-13 * np.linalg.norm(y)
    # the near field between tiles is what the tiled form drops: P_tiled differs from P
    xt = NF.apply_Pinv(S, tm, Tnf, tx, ty, y)
    assert np.linalg.norm(xt - x) > 1e-6 * np.linalg.norm(x)


@pytest.mark.parametrize("tile", [(2, 2), (4, 3)])
def test_preconditioned_solution_matches_lu(tile):
    nx, ny = 4, 3
    g, B, S, tm, T_of = _surface(nx, ny, npch=24, seed=8)
    Tnf = NF.near_field_blocks(T_of, g.rho, W.PITCH, W.WAVELENGTH / 6)
    A = np.eye(nx * ny * g.n_eq) - MM.dense_S(S, tm) @ C.dense_T(B, nx, ny)
    b = W.plane_wave_rhs(W.small_config(nx, ny, 24, 3, 1, seed=9), g)
    shape = b.shape
    Af = lambda v: MM.apply_A(lambda z: C.apply_T_dense(B, z), S, tm, v.reshape(shape)).ravel()
    Minv = lambda v: NF.apply_Pinv(S, tm, Tnf, tile[0], tile[1], v.reshape(shape)).ravel()
    x, info = K.gmres(Af, b.ravel(), 1e-12, M_inv=Minv)
    x0, info0 = K.gmres(Af, b.ravel(), 1e-12)
    x_lu = K.solve_dense(A, b.ravel())
    assert info.converged and np.linalg.norm(x - x_lu) <= 1e-10 * np.linalg.norm(x_lu)
    assert info.iters <= info0.iters
