"""Pins of the macromodel-generation oracle (Schur complement of the interior
unknowns, S = -(Z~ + Z_self)^-1) against closed forms and identities that do
not retype its formulas."""
import numpy as np
import pytest

import workload as W
from oracle import macromodel_gen as MG


def test_uncoupled_interior_leaves_surface_block():
    Z, _ = W.cell_interiors(1, 6, 9, seed=1)
    Z[0, :6, 6:] = 0.0
    Z[0, 6:, :6] = 0.0
    assert np.array_equal(MG.schur_macromodel(Z[0], 6), Z[0, :6, :6])


def test_scalar_closed_form():
    a, b, c, d = 2 + 1j, 0.5 - 0.25j, -0.75j, 1.5 + 0.5j
    Z = np.array([[a, b], [c, d]])
    assert abs(MG.schur_macromodel(Z, 1)[0, 0] - (a - b * c / d)) <= 1e-15
    zs = 0.25 + 0.5j
    S = MG.macromodel_S(MG.schur_macromodel(Z, 1), np.array([[zs]]))
    assert abs(S[0, 0] + 1.0 / (a - b * c / d + zs)) <= 1e-15


def test_no_interior_unknowns():
    Z, _ = W.cell_interiors(1, 5, 0, seed=2)
    assert np.array_equal(MG.schur_macromodel(Z[0], 5), Z[0])


@pytest.mark.parametrize("n,m", [(4, 7), (12, 5), (24, 48)])
def test_determinant_identity(n, m):
    Z, _ = W.cell_interiors(1, n, m, seed=n + m)
    Zt = MG.schur_macromodel(Z[0], n)
    s_full, l_full = np.linalg.slogdet(Z[0])
    s_ii, l_ii = np.linalg.slogdet(Z[0, n:, n:])
    s_t, l_t = np.linalg.slogdet(Zt)
    assert abs(l_full - (l_ii + l_t)) <= 1e-10 * max(1.0, abs(l_full))
    assert abs(s_full - s_ii * s_t) <= 1e-10


@pytest.mark.parametrize("n,m", [(6, 10), (20, 33)])
def test_macromodel_reproduces_full_solve(n, m):
    # with no interior excitation, the surface part of the full solution
    # solves the macromodel equation
    Z, _ = W.cell_interiors(1, n, m, seed=7)
    rng = np.random.default_rng(3)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    full = np.linalg.solve(Z[0], np.concatenate([f, np.zeros(m)]))
    Zt = MG.schur_macromodel(Z[0], n)
    assert np.abs(Zt @ full[:n] - f).max() <= 1e-12 * np.abs(f).max()


def test_S_inverts_shifted_macromodel_and_has_modest_norm():
    Z, Zself = W.cell_interiors(3, 16, 24, seed=4)
    Zt, S = MG.macromodels(Z, 16, Zself)
    for t in range(3):
        assert np.abs((Zt[t] + Zself) @ S[t] + np.eye(16)).max() <= 1e-13
        assert 0.2 < np.linalg.norm(S[t], 2) < 1.0
