"""Pins of the oracle's macromodel apply, operator A = I - S T and GMRES against
library routines (block_diag, zgesv, scipy GMRES) and closed-form solves."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM


def _lattice(nx, ny, npch=24, n_types=4, seed=0, physical=True, n=None):
    if physical:
        g = W.box_geometry(npch)
        B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
        n = g.n_eq
    else:
        B = W.random_blocks(nx, ny, n, seed=seed)
    S = W.random_types(n_types, n, seed=seed)
    tm = W.random_type_map(nx, ny, n_types, seed=seed)
    return B, S, tm, n


def _ops(B, S, tm):
    ny, nx = tm.shape
    Tfun = lambda x: C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    Afun = lambda x: MM.apply_A(Tfun, S, tm, x)
    return Tfun, Afun


# ----------------------------------------------------------------------------- S
def test_apply_S_matches_library_block_diag():
    nx, ny, n = 3, 2, 5
    S = W.random_types(3, n, seed=1)
    tm = W.random_type_map(nx, ny, 3, seed=1)
    x = W.random_vectors(2, nx, ny, n, seed=2)
    D = scipy.linalg.block_diag(*[S[t] for t in tm.ravel()])
    y = MM.apply_S(S, tm, x)
    assert np.allclose(y.reshape(2, -1), x.reshape(2, -1) @ D.T, atol=1e-15)
    assert np.array_equal(MM.dense_S(S, tm), D)


def test_apply_S_identity_and_scaled_types():
    nx, ny, n = 4, 3, 6
    x = W.random_vectors(1, nx, ny, n, seed=4)
    tm = W.random_type_map(nx, ny, 2, seed=4)
    I2 = np.stack([np.eye(n), 2.5j * np.eye(n)]).astype(np.complex128)
    y = MM.apply_S(I2, tm, x)
    expect = np.where((tm == 0)[None, :, :, None], x, 2.5j * x)
    assert np.array_equal(y, expect)


# ----------------------------------------------------------------------------- solves
def test_single_element_solve_is_b():
    # 1 x 1 lattice: T has only its zero self block, so A = I and x = b; GMRES stops
    # after one Arnoldi step on a lucky breakdown.
    B, S, tm, n = _lattice(1, 1)
    _, Afun = _ops(B, S, tm)
    b = W.random_vectors(1, 1, 1, n, seed=1)
    x, info = K.gmres(lambda v: Afun(v.reshape(b.shape)).ravel(), b.ravel(), 1e-12)
    assert info.converged and info.iters == 1
    assert np.allclose(x, b.ravel(), atol=1e-15)


def test_single_scatterer_closed_form():
    # S nonzero at one element m0 only: S T S = S_m0 T(0) S_m0 = 0, so (S T)^2 = 0
    # and A^-1 = I + S T exactly: x = b + S T b; GMRES needs at most 2 steps.
    nx, ny = 4, 4
    B, S, tm, n = _lattice(nx, ny)
    S2 = np.stack([np.zeros((n, n), complex), S[0]])
    tm2 = np.zeros((ny, nx), np.int32)
    tm2[1, 2] = 1
    Tfun, Afun = _ops(B, S2, tm2)
    b = W.plane_wave_rhs(W.small_config(nx, ny))
    closed = b + MM.apply_S(S2, tm2, Tfun(b))
    x, info = K.gmres(lambda v: Afun(v.reshape(b.shape)).ravel(), b.ravel(), 1e-14)
    assert info.converged and info.iters <= 2
    assert np.linalg.norm(x - closed.ravel()) <= 1e-13 * np.linalg.norm(closed)


def test_two_element_closed_form():
    # 1 x 2 lattice: eliminate x2 = b2 + S2 T21 x1, then
    # (I - S1 T12 S2 T21) x1 = b1 + S1 T12 b2, solved by LAPACK on n x n.
    nx, ny = 2, 1
    B, S, tm, n = _lattice(nx, ny, seed=3)
    tm = np.array([[0, 1]], np.int32)
    S1, S2 = S[0], S[1]
    T12 = B[0, -1 + nx - 1]          # test element 1 = (0,0), source 2 = (0,1): d = (0, -1)
    T21 = B[0, 1 + nx - 1]
    b = W.random_vectors(1, nx, ny, n, seed=9)
    b1, b2 = b[0, 0, 0], b[0, 0, 1]
    x1 = np.linalg.solve(np.eye(n) - S1 @ T12 @ S2 @ T21, b1 + S1 @ T12 @ b2)
    x2 = b2 + S2 @ T21 @ x1
    _, Afun = _ops(B, S, tm)
    x, info = K.gmres(lambda v: Afun(v.reshape(b.shape)).ravel(), b.ravel(), 1e-14)
    ref = np.concatenate([x1, x2])
    assert info.converged
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("nx,ny,npch", [(4, 4, 24), (8, 8, 24)])
def test_gmres_matches_dense_lu(nx, ny, npch):
    B, S, tm, n = _lattice(nx, ny, npch)
    _, Afun = _ops(B, S, tm)
    A = np.eye(nx * ny * n) - MM.dense_S(S, tm) @ C.dense_T(B, nx, ny)
    b = W.plane_wave_rhs(W.small_config(nx, ny, npch))
    x_lu = K.solve_dense(A, b.ravel())
    x, info = K.gmres(lambda v: Afun(v.reshape(b.shape)).ravel(), b.ravel(), 1e-14)
    assert info.converged
    assert np.linalg.norm(x - x_lu) <= 1e-12 * np.linalg.norm(x_lu)
    assert info.rel_res_true <= 1e-14


def test_config1_solve_against_lu_and_scipy():
    c = W.config(1)
    g = W.box_geometry(c.n_patch)
    B = C.coupling_blocks(g.rho, g.area, g.tan, c.nx, c.ny, W.PITCH, W.K0)
    S, tm = W.s_types(c), W.type_map(c)
    _, Afun = _ops(B, S, tm)
    A = np.eye(c.n_unknowns) - MM.dense_S(S, tm) @ C.dense_T(B, c.nx, c.ny)
    b = W.plane_wave_rhs(c, g).ravel()
    x, info = K.gmres(lambda v: Afun(v.reshape(1, c.ny, c.nx, c.n_eq)).ravel(), b, c.tol)
    x_lu = np.linalg.solve(A, b)
    assert info.converged and np.linalg.norm(A @ x - b) <= c.tol * np.linalg.norm(b)
    assert np.linalg.norm(x - x_lu) <= 1e-9 * np.linalg.norm(x_lu)
    # scipy's GMRES (same restart, no preconditioner, relative tolerance only):
    # iteration counts within one of each other
    count = [0]
    xs, flag = scipy.sparse.linalg.gmres(A, b, rtol=c.tol, atol=0.0, restart=30, maxiter=20,
                                         callback=lambda r: count.__setitem__(0, count[0] + 1),
                                         callback_type="pr_norm")
    assert flag == 0
    assert abs(count[0] - info.iters) <= 1
    # Neumann series: rho(S T) is small, so sum_k (S T)^k b converges to the same x
    ST = MM.dense_S(S, tm) @ C.dense_T(B, c.nx, c.ny)
    xn, term = b.copy(), b.copy()
    for _ in range(40):
        term = ST @ term
        xn += term
    assert np.linalg.norm(xn - x_lu) <= 1e-12 * np.linalg.norm(x_lu)


def test_gmres_finite_termination_and_monotone():
    rng = np.random.default_rng(5)
    n = 8
    A = np.eye(n) + 0.8 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = K.gmres(lambda v: A @ v, b, 1e-13, restart=30)
    assert info.converged and info.iters <= n
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)
    h = info.history
    assert all(h[i + 1] <= h[i] * (1 + 1e-12) for i in range(len(h) - 1))


def test_gmres_restart_still_solves():
    rng = np.random.default_rng(6)
    n = 40
    A = np.eye(n) + 0.5 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = K.gmres(lambda v: A @ v, b, 1e-12, restart=3, max_iter=400)
    assert info.converged and info.restarts > 1
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_gmres_not_converged_and_zero_rhs():
    rng = np.random.default_rng(7)
    n = 20
    A = np.eye(n) + 0.5 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n).astype(complex)
    x, info = K.gmres(lambda v: A @ v, b, 1e-30, max_iter=1)
    assert not info.converged and info.iters == 1 and np.linalg.norm(x) > 0
    x, info = K.gmres(lambda v: A @ v, np.zeros(n, complex), 1e-10)
    assert info.converged and info.iters == 0 and not np.any(x)


def test_givens_zeroes_second_component():
    for a, b in [(1 + 2j, 3 - 1j), (0, 2j), (1.5, 0), (-2j, 1e-300)]:
        c, s = K.givens(a, b)
        top = c * a + s * b
        bot = -np.conj(s) * a + c * b
        assert abs(bot) <= 1e-15 * max(1.0, abs(top))
        assert abs(abs(top) - np.hypot(abs(a), abs(b))) <= 1e-15 * abs(top)
        assert abs(c * c + abs(s) ** 2 - 1) <= 1e-15


def test_gmres_multi_columns_against_lu():
    # independent instances per right-hand side: each column of the [nrhs][...]
    # input is solved to the dense LU solution, with the iteration count the
    # one-column solve reports, and the output keeps the input's shape
    B, S, tm, n = _lattice(2, 2, seed=11)
    _, Afun = _ops(B, S, tm)
    A = np.eye(4 * n) - MM.dense_S(S, tm) @ C.dense_T(B, 2, 2)
    b = W.random_vectors(3, 2, 2, n, seed=12)
    b[1] *= 1e-3                                    # scale must not matter per column
    xs, infos = K.gmres_multi(Afun, b, 1e-12)
    assert xs.shape == b.shape and len(infos) == 3
    for r in range(3):
        x_lu = K.solve_dense(A, b[r].ravel())
        assert np.linalg.norm(xs[r].ravel() - x_lu) <= 1e-11 * np.linalg.norm(x_lu)
        x1, i1 = K.gmres(lambda v: Afun(v.reshape((1,) + b.shape[1:])).ravel(), b[r].ravel(), 1e-12)
        assert infos[r].iters == i1.iters and np.array_equal(x1, xs[r].ravel())
