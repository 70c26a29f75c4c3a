"""Pins of the far-field oracle against closed forms (elementary electric and
magnetic sources, the array factor of a uniform lattice), the translation
phase and linearity -- none of them a retyping of its sums."""
import numpy as np
import pytest

import workload as W
from oracle import far_field as FF


def _single_patch_geometry():
    rho = np.zeros((1, 3))
    area = np.array([0.5])
    tan = np.array([[[1.0, 0, 0], [0, 1.0, 0]]])          # t_0 = x, t_1 = y
    return rho, area, tan


def _dirs(n=7, seed=0):
    rng = np.random.default_rng(seed)
    r = np.sqrt(rng.uniform(0, 0.95, n))
    a = rng.uniform(0, 2 * np.pi, n)
    return r * np.cos(a), r * np.sin(a)


def test_x_electric_element_closed_form():
    # J = x at the origin: E_theta = A cos(theta) cos(phi), E_phi = -A sin(phi)
    rho, area, tan = _single_patch_geometry()
    x = np.zeros((1, 1, 1, 4), complex)
    x[0, 0, 0, 0] = 1.0
    u, v = _dirs()
    E = FF.far_field(rho, area, tan, 0.5, W.K0, x, u, v)
    th = np.arcsin(np.sqrt(u * u + v * v))
    phi = np.arctan2(v, u)
    assert np.allclose(E[0, :, 0], 0.5 * np.cos(th) * np.cos(phi), atol=1e-14)
    assert np.allclose(E[0, :, 1], -0.5 * np.sin(phi), atol=1e-14)


def test_y_magnetic_element_closed_form():
    # M = y at the origin: L = A y, E_theta = L . phi^ = A cos(phi), E_phi = -L . theta^ = -A cos(theta) sin(phi)
    rho, area, tan = _single_patch_geometry()
    x = np.zeros((1, 1, 1, 4), complex)
    x[0, 0, 0, 3] = 1.0
    u, v = _dirs(seed=1)
    E = FF.far_field(rho, area, tan, 0.5, W.K0, x, u, v)
    th = np.arcsin(np.sqrt(u * u + v * v))
    phi = np.arctan2(v, u)
    assert np.allclose(E[0, :, 0], 0.5 * np.cos(phi), atol=1e-14)
    assert np.allclose(E[0, :, 1], -0.5 * np.cos(th) * np.sin(phi), atol=1e-14)


@pytest.mark.parametrize("nx,ny", [(5, 3), (8, 8)])
def test_uniform_lattice_array_factor(nx, ny):
    # identical currents on every element multiply the element pattern by the
    # product of two Dirichlet kernels
    g = W.box_geometry(24)
    rng = np.random.default_rng(2)
    xe = rng.standard_normal(g.n_eq) + 1j * rng.standard_normal(g.n_eq)
    x = np.broadcast_to(xe, (1, ny, nx, g.n_eq)).copy()
    u, v = _dirs(seed=3)
    E = FF.far_field(g.rho, g.area, g.tan, W.PITCH, W.K0, x, u, v)
    E1 = FF.far_field(g.rho, g.area, g.tan, W.PITCH, W.K0, x[:, :1, :1], u, v)

    def dirichlet(N, psi):
        return np.exp(1j * (N - 1) * psi / 2) * np.sin(N * psi / 2) / np.sin(psi / 2)

    af = dirichlet(nx, W.K0 * W.PITCH * u) * dirichlet(ny, W.K0 * W.PITCH * v)
    assert np.allclose(E[0], E1[0] * af[:, None], rtol=1e-12, atol=1e-12 * np.abs(E).max())


def test_translation_phase_and_linearity():
    g = W.box_geometry(24)
    x = W.random_vectors(2, 3, 4, g.n_eq, seed=5)
    u, v = _dirs(seed=4)
    E = FF.far_field(g.rho, g.area, g.tan, W.PITCH, W.K0, x, u, v)
    # moving every current one element along x adds k pitch u to the phase
    ny, nx = x.shape[1], x.shape[2]
    xs = np.zeros((2, ny, nx + 1, g.n_eq), complex)
    xs[:, :, 1:, :] = x
    Es = FF.far_field(g.rho, g.area, g.tan, W.PITCH, W.K0, xs, u, v)
    assert np.allclose(Es, E * np.exp(1j * W.K0 * W.PITCH * u)[None, :, None], rtol=1e-12, atol=1e-12)
    # linear in the currents
    y = W.random_vectors(2, 3, 4, g.n_eq, seed=6)
    Ey = FF.far_field(g.rho, g.area, g.tan, W.PITCH, W.K0, y, u, v)
    Ez = FF.far_field(g.rho, g.area, g.tan, W.PITCH, W.K0, 2 * x - 1j * y, u, v)
    assert np.allclose(Ez, 2 * E - 1j * Ey, rtol=1e-12, atol=1e-12)


def test_fft_bins_map_to_lattice_phases():
    # bin (q, p) of the lattice DFT with kernel e^{+j2pi(p ix/Lu + q iy/Lv)} is the
    # direction whose lattice phase k pitch (u ix + v iy) equals that kernel mod 2 pi
    Lu, Lv = 12, 8
    u, v = FF.fft_bin_directions(Lu, Lv, W.PITCH, W.K0)
    ix, iy = 5, 3
    for q in range(Lv):
        for p in range(Lu):
            a = np.exp(1j * W.K0 * W.PITCH * (u[q, p] * ix + v[q, p] * iy))
            b = np.exp(2j * np.pi * (p * ix / Lu + q * iy / Lv))
            assert abs(a - b) <= 1e-12


def test_z_electric_element_closed_form():
    # J = z (a side-face tangent): E_theta = -A sin(theta), E_phi = 0
    rho = np.zeros((1, 3))
    area = np.array([0.25])
    tan = np.array([[[0, 0, 1.0], [1.0, 0, 0]]])
    x = np.zeros((1, 1, 1, 4), complex)
    x[0, 0, 0, 0] = 1.0
    u, v = _dirs(seed=8)
    E = FF.far_field(rho, area, tan, 0.5, W.K0, x, u, v)
    th = np.arcsin(np.sqrt(u * u + v * v))
    assert np.allclose(E[0, :, 0], -0.25 * np.sin(th), atol=1e-14)
    assert np.allclose(E[0, :, 1], 0.0, atol=1e-14)


def _bin_at(Lu, Lv, u0, v0):
    u, v = FF.fft_bin_directions(Lu, Lv, W.PITCH, W.K0)
    q, p = np.unravel_index(np.argmin((u - u0) ** 2 + (v - v0) ** 2), u.shape)
    return q, p


def test_directivity_of_an_electric_element_and_a_huygens_source():
    # Directivity 3/2 of an elementary electric current at broadside, and 3 of
    # a Huygens source (J = x with M = y, pattern (1 + cos theta)^2) at
    # broadside with a null behind it; the bin quadrature of P_rad converges
    # to the closed-form sphere integrals (8 pi / 3 and 16 pi / 3) as the grid refines
    rho, area, tan = _single_patch_geometry()
    for Lu, tol in ((256, 2e-2), (1024, 6e-3)):
        x = np.zeros((2, 1, 1, 4), complex)
        x[0, 0, 0, 0] = 1.0                      # J = x
        x[1, 0, 0, 0] = 1.0                      # J = x ...
        x[1, 0, 0, 3] = 1.0                      # ... with M = y
        D, P = FF.directivity(rho, area, tan, W.PITCH, W.K0, x, Lu, Lu)
        q, p = _bin_at(Lu, Lu, 0.0, 0.0)
        assert abs(D[0, 0, q, p] - 1.5) <= tol * 1.5, (Lu, D[0, 0, q, p])
        assert abs(D[1, 0, q, p] - 3.0) <= tol * 3.0, (Lu, D[1, 0, q, p])
        assert D[1, 1, q, p] <= 1e-20
        assert abs(P[0] / (area[0] ** 2) - 8 * np.pi / 3) <= tol * 8 * np.pi / 3
        assert abs(P[1] / (area[0] ** 2) - 16 * np.pi / 3) <= tol * 16 * np.pi / 3


def test_directivity_lower_half_space_mirrors_the_upper():
    # sources in the z = 0 plane radiate symmetric patterns up and down for a
    # current pair whose fields mirror: an electric current alone
    rho, area, tan = _single_patch_geometry()
    x = np.zeros((1, 1, 1, 4), complex)
    x[0, 0, 0, 1] = 2.0 - 1.0j
    D, _ = FF.directivity(rho, area, tan, W.PITCH, W.K0, x, 64, 48)
    assert np.allclose(D[0, 0], D[0, 1], rtol=1e-13, atol=0)
