"""Pins of the structured (L, K) outer operator of the oracle against
finite-difference derivatives of the scalar Green's function, the far-field
limit, reciprocity and structural zeros -- none of them a retyping of the
oracle's closed-form derivatives."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import coupling_lk as LK


def _geom(npch=48):
    g = W.box_geometry(npch)
    return g, (g.rho, g.area, g.tan)


def _fd_grad_hess(r, k, h):
    """Central-difference gradient and Hessian of g(|r|) in the displacement r."""
    f = lambda v: C.green(np.array(np.linalg.norm(v)), k)
    e = np.eye(3)
    grad = np.array([(f(r + h * e[i]) - f(r - h * e[i])) / (2 * h) for i in range(3)])
    H = np.zeros((3, 3), dtype=complex)
    for i in range(3):
        for j in range(3):
            H[i, j] = (f(r + h * e[i] + h * e[j]) - f(r + h * e[i] - h * e[j])
                       - f(r - h * e[i] + h * e[j]) + f(r - h * e[i] - h * e[j])) / (4 * h * h)
    return grad, H


@pytest.mark.parametrize("d", [(0, 1), (1, 0), (-1, 1), (2, -3), (0, 5)])
def test_entries_match_finite_difference_derivatives(d):
    g, G = _geom()
    L, K = LK.lk_blocks_at(*G, [d], W.PITCH, W.K0)
    rng = np.random.default_rng(7)
    P = g.n_patch
    for _ in range(12):
        p, q = rng.integers(0, P, size=2)
        a, b = rng.integers(0, 2, size=2)
        r = g.rho[p] - g.rho[q] + W.PITCH * np.array([d[1], d[0], 0.0])
        grad, H = _fd_grad_hess(r, W.K0, 1e-4 * np.linalg.norm(r))
        tp, tq = g.tan[p, a], g.tan[q, b]
        dyad = C.green(np.array(np.linalg.norm(r)), W.K0) * np.eye(3) + H / W.K0 ** 2
        l_fd = g.area[q] * tp @ dyad @ tq
        k_fd = g.area[q] * tp @ np.cross(grad, tq)
        scale = np.abs(L[0]).max()
        assert abs(L[0][2 * p + a, 2 * q + b] - l_fd) <= 1e-6 * scale
        assert abs(K[0][2 * p + a, 2 * q + b] - k_fd) <= 1e-6 * np.abs(K[0]).max()


def test_far_field_is_transverse():
    # at R ~ 20 wavelengths the dyadic tends to (I - Rhat Rhat) g and grad g to -jk g Rhat
    g, G = _geom(24)
    d = (0, 40)
    L, K = LK.lk_blocks_at(*G, [d], W.PITCH, W.K0)
    P = g.n_patch
    disp = g.rho[:, None, :] - g.rho[None, :, :] + np.array([W.PITCH * d[1], 0.0, 0.0])
    R = np.linalg.norm(disp, axis=-1)
    Rh = disp / R[..., None]
    gR = C.green(R, W.K0)
    Lff = np.zeros_like(L[0])
    Kff = np.zeros_like(K[0])
    for p in range(P):
        for q in range(P):
            T = np.eye(3) - np.outer(Rh[p, q], Rh[p, q])
            for a in range(2):
                for b in range(2):
                    Lff[2 * p + a, 2 * q + b] = g.area[q] * gR[p, q] * (g.tan[p, a] @ T @ g.tan[q, b])
                    Kff[2 * p + a, 2 * q + b] = (g.area[q] * (-1j * W.K0) * gR[p, q]
                                                 * (g.tan[p, a] @ np.cross(Rh[p, q], g.tan[q, b])))
    kr = W.K0 * R.min()
    assert np.abs(L[0] - Lff).max() <= 2.0 / kr * np.abs(L[0]).max()
    assert np.abs(K[0] - Kff).max() <= 2.0 / kr * np.abs(K[0]).max()


@pytest.mark.parametrize("d", [(0, 1), (1, 2), (-2, 1), (3, 0)])
def test_reciprocity_identities(d):
    # L and K are both reciprocal up to the source-area weight: X(-d)^T = D X(d) D^-1
    g, G = _geom()
    L, K = LK.lk_blocks_at(*G, [d, (-d[0], -d[1])], W.PITCH, W.K0)
    D = np.repeat(g.area, 2)
    for X in (L, K):
        lhs = X[1].T
        rhs = D[:, None] * X[0] / D[None, :]
        assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(X[0]).max()


def test_k_vanishes_for_coplanar_tangents():
    # two +z-face patches at an in-plane offset: Rhat and both tangents lie in
    # the plane z = h/2, so every triple product t_p . (Rhat x t_q) vanishes
    g, G = _geom()
    top = [p for p in range(g.n_patch) if g.normal[p][2] == 1.0]
    L, K = LK.lk_blocks_at(*G, [(1, 2)], W.PITCH, W.K0)
    idx = [2 * p + a for p in top for a in range(2)]
    assert np.abs(K[0][np.ix_(idx, idx)]).max() <= 1e-15 * np.abs(K[0]).max()
    assert np.abs(L[0][np.ix_(idx, idx)]).max() > 0


def test_self_offset_is_zero_and_assembly_layout():
    g, G = _geom(24)
    L, K = LK.lk_blocks_at(*G, [(0, 0), (0, 1)], W.PITCH, W.K0)
    assert not np.any(L[0]) and not np.any(K[0])
    coef = LK.paper_coefficients(W.K0)
    T = LK.lk_assemble(L, K, coef)
    nh = L.shape[-1]
    assert T.shape == (2, 2 * nh, 2 * nh)
    assert not np.any(T[0])
    a, b, c, e = coef
    assert np.array_equal(T[1][:nh, :nh], a * L[1]) and np.array_equal(T[1][:nh, nh:], b * K[1])
    assert np.array_equal(T[1][nh:, :nh], c * K[1]) and np.array_equal(T[1][nh:, nh:], e * L[1])


def test_lk_blocks_index_convention():
    # block [dy+ny-1][dx+nx-1] holds offset (dy, dx) = test - source
    g, G = _geom(24)
    Lb, Kb = LK.lk_blocks(*G, 3, 2, W.PITCH, W.K0)
    L1, K1 = LK.lk_blocks_at(*G, [(1, -2)], W.PITCH, W.K0)
    assert np.array_equal(Lb[1 + 1, -2 + 2], L1[0]) and np.array_equal(Kb[1 + 1, -2 + 2], K1[0])


def test_workload_constants_are_the_paper_reading():
    assert np.allclose(W.OUTER_COEF, LK.paper_coefficients(W.K0), rtol=0, atol=0)


def test_sampled_rows_match_dense_assembly():
    # the on-the-fly row evaluator equals the dense Toeplitz matrix of the
    # assembled blocks (a different summation path through coupling.dense_T)
    g, G = _geom(24)
    nx, ny = 3, 4
    Lb, Kb = LK.lk_blocks(*G, nx, ny, W.PITCH, W.K0)
    T = C.dense_T(LK.lk_assemble(Lb, Kb, W.OUTER_COEF), nx, ny)
    x = W.random_vectors(2, nx, ny, g.n_eq, seed=3)
    y = (x.reshape(2, -1) @ T.T).reshape(x.shape)
    elems = [(0, 0), (2, 1), (3, 2)]
    rows = LK.apply_T_elements_lk(*G, W.PITCH, W.K0, W.OUTER_COEF, x, elems, chunk_rows=2)
    for i, (iy, ix) in enumerate(elems):
        assert np.abs(rows[i] - y[:, iy, ix]).max() <= 1e-13 * np.abs(y).max()


def test_structured_operator_reciprocity_needs_the_signed_weights():
    # With the paper's constants (b = -c) the assembled outer operator satisfies
    # T(-d) = W^-1 T(d)^T W with W = diag(A, -A) (J half, M half); with b = c it
    # would take W = diag(A, A).  A reciprocal store of the structured form
    # therefore needs the sign.
    g, G = _geom()
    d = (1, 2)
    L, K = LK.lk_blocks_at(*G, [d, (-d[0], -d[1])], W.PITCH, W.K0)
    a = np.repeat(g.area, 2)
    for coef, w in [(W.OUTER_COEF, np.concatenate([a, -a])),
                    ((W.OUTER_COEF[0], 1.0, 1.0, W.OUTER_COEF[3]), np.concatenate([a, a]))]:
        T = LK.lk_assemble(L[None, None, 0], K[None, None, 0], coef)[0, 0]
        Tm = LK.lk_assemble(L[None, None, 1], K[None, None, 1], coef)[0, 0]
        assert np.abs(Tm - (T.T * w[None, :]) / w[:, None]).max() <= 1e-13 * np.abs(T).max()
    T = LK.lk_assemble(L[None, None, 0], K[None, None, 0], W.OUTER_COEF)[0, 0]
    Tm = LK.lk_assemble(L[None, None, 1], K[None, None, 1], W.OUTER_COEF)[0, 0]
    wrong = np.concatenate([a, a])
    assert np.abs(Tm - (T.T * wrong[None, :]) / wrong[:, None]).max() > 1e-3 * np.abs(T).max()
