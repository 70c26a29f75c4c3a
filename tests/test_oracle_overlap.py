"""Pins of the touching-box incidence U_o (Sec. III-D, eqs. (connections_IUI),
(final)) and of the coincident-patch Green's term, against closed-form counts,
structural identities and a numerical integral."""
import numpy as np
import pytest
import scipy.integrate

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM
from oracle import overlap as OV

BOX = W.BOX_A                      # touching boxes: pitch = box edge


@pytest.mark.parametrize("npch,nx,ny", [(24, 3, 2), (48, 2, 3), (72, 2, 2)])
def test_shared_face_and_ground_plane_counts(npch, nx, ny):
    g = W.box_geometry(npch)
    n_t, s_a, s_h = W.PATCH_GRIDS[npch]
    N = nx * ny * g.n_eq
    shared = (nx - 1) * ny + nx * (ny - 1)
    U = OV.incidence(g.rho, g.tan, nx, ny, BOX)
    # every shared face drops the 4 unknowns of each of its s_a s_h patches once
    assert U.shape == (N, N - shared * s_a * s_h * 4)
    Ug = OV.incidence(g.rho, g.tan, nx, ny, BOX, ground_plane=True)
    # the ground plane removes the 2 M unknowns of each bottom patch of every box
    assert Ug.shape[1] == U.shape[1] - nx * ny * n_t * n_t * 2
    # boxes that do not touch keep every unknown
    assert np.array_equal(OV.incidence(g.rho, g.tan, nx, ny, W.PITCH), np.eye(N))


def test_incidence_structure_and_cancelling_face_currents():
    g = W.box_geometry(48)
    nx, ny = 3, 2
    U = OV.incidence(g.rho, g.tan, nx, ny, BOX)
    G = U.T @ U
    mult = np.diag(G)
    assert np.array_equal(G, np.diag(mult)) and set(np.unique(mult)) == {1.0, 2.0}
    # the expanded currents on each shared face cancel pairwise (opposite normals)
    rng = np.random.default_rng(1)
    xt = rng.standard_normal(U.shape[1]) + 1j * rng.standard_normal(U.shape[1])
    x = (U @ xt).reshape(ny, nx, g.n_eq)
    P = g.n_patch
    for iy in range(ny):
        for ix in range(nx - 1):
            for p in range(P):
                for q in range(P):
                    if np.linalg.norm(g.rho[p] - (g.rho[q] + np.array([BOX, 0, 0]))) < 1e-12:
                        for tau in (0, 1):
                            jp = x[iy, ix, tau * 2 * P + 2 * p:tau * 2 * P + 2 * p + 2] @ g.tan[p]
                            jq = x[iy, ix + 1, tau * 2 * P + 2 * q:tau * 2 * P + 2 * q + 2] @ g.tan[q]
                            assert np.allclose(jp + jq, 0.0, atol=1e-14)


def test_coincident_patch_term_against_the_square_integral():
    # static part: integral of 1/(4 pi R) over a square of side a about its centre
    for A in (0.01, 0.0025, 0.011):
        a = np.sqrt(A)
        val, err = scipy.integrate.dblquad(lambda y, x: 1.0 / np.hypot(x, y), 0, a / 2, 0, a / 2, epsabs=1e-13)
        term = C.coincident_patch_term(A, W.K0)
        assert abs(term.real - 4 * val / (4 * np.pi)) <= 1e-9 * term.real
        assert abs(term.imag + W.K0 * A / (4 * np.pi)) <= 1e-15
    # the fill takes it exactly where boxes touch and nowhere else
    g = W.box_geometry(24)
    B = C.coupling_blocks(g.rho, g.area, g.tan, 2, 1, BOX, W.K0)
    assert np.all(np.isfinite(B))
    Bp = C.coupling_blocks(g.rho, g.area, g.tan, 2, 1, W.PITCH, W.K0)
    assert np.all(np.isfinite(Bp)) and not np.any(np.isclose(np.abs(Bp[0, 2]), np.abs(C.coincident_patch_term(g.area[0], W.K0))))


def test_reduced_solution_solves_the_projected_full_system():
    # x = U x~ with A~ x~ = U^T (D + T) b-form right-hand side: U^T (D + T) U x~ = U^T V,
    # i.e. the full residual (D + T) U x~ - V is orthogonal to range(U_o)
    g = W.box_geometry(24)
    nx, ny = 2, 2
    S = W.random_types(2, g.n_eq, seed=3)
    tm = W.random_type_map(nx, ny, 2, seed=3)
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, BOX, W.K0)
    T = C.dense_T(B, nx, ny)
    D = OV.dense_D(S, tm)
    assert np.allclose(D @ MM.dense_S(S, tm), -np.eye(D.shape[0]), atol=1e-10)
    U = OV.incidence(g.rho, g.tan, nx, ny, BOX, ground_plane=True)
    At = OV.reduced_operator(U, D, T)
    V = W.random_vectors(1, nx, ny, g.n_eq, seed=4).ravel()
    xt = K.solve_dense(At, U.T @ V)
    r = (D + T) @ (U @ xt) - V
    assert np.linalg.norm(U.T @ r) <= 1e-10 * np.linalg.norm(U.T @ V)
    # without touching or ground plane the reduced system is the full one
    Bp = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    Up = OV.incidence(g.rho, g.tan, nx, ny, W.PITCH)
    Tp = C.dense_T(Bp, nx, ny)
    assert np.array_equal(OV.reduced_operator(Up, D, Tp), D + Tp)
