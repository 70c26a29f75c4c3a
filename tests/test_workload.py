"""Pins of the seeded input generator (geometry, macromodels, excitation)."""
import math

import numpy as np
import pytest

import workload as W


@pytest.mark.parametrize("npch", [24, 48, 72])
def test_box_geometry(npch):
    g = W.box_geometry(npch)
    assert g.n_patch == npch and g.n_eq == 4 * npch
    # patches tile the whole box surface: 2 a^2 + 4 a h
    assert math.isclose(g.area.sum(), 2 * W.BOX_A ** 2 + 4 * W.BOX_A * W.BOX_H, rel_tol=1e-14)
    # every centre lies on the face its normal names
    for c, n in zip(g.rho, g.normal):
        ax = int(np.argmax(np.abs(n)))
        half = W.BOX_H / 2 if ax == 2 else W.BOX_A / 2
        assert math.isclose(c[ax], np.sign(n[ax]) * half, abs_tol=1e-15)
        others = [i for i in range(3) if i != ax]
        for i in others:
            lim = W.BOX_H / 2 if i == 2 else W.BOX_A / 2
            assert abs(c[i]) < lim
    # tangents: orthonormal pair, both perpendicular to the normal
    for t, n in zip(g.tan, g.normal):
        assert np.allclose(t @ t.T, np.eye(2), atol=1e-15)
        assert np.allclose(t @ n, 0.0, atol=1e-15)


def test_closest_centres_across_gap():
    # facing side patches of neighbouring boxes are pitch - a = 0.05 apart
    g = W.box_geometry(24)
    pts0 = g.rho
    pts1 = g.rho + np.array([W.PITCH, 0, 0])
    d = np.linalg.norm(pts0[:, None] - pts1[None], axis=-1)
    assert math.isclose(d.min(), W.PITCH - W.BOX_A, rel_tol=1e-12)


@pytest.mark.parametrize("cfg", [1, 2])
def test_s_types_norm(cfg):
    c = W.config(cfg)
    S = W.s_types(c)
    assert S.shape == (c.n_types, c.n_eq, c.n_eq)
    for t in range(c.n_types):
        assert abs(np.linalg.norm(S[t], 2) - 0.5) < 1e-14


def test_seeded_reproducible():
    a = W.s_types(W.config(1))
    b = W.s_types(W.config(1))
    assert np.array_equal(a, b)
    assert np.array_equal(W.type_map(W.config(2)), W.type_map(W.config(2)))
    assert W.config(3).nrhs == 16 and W.config(4).nrhs == 4


def test_config_sizes():
    # unknown counts quoted with the lattice workloads
    assert W.config(1).n_unknowns == 1536
    assert W.config(2).n_unknowns == 196608
    assert W.config(4).n_unknowns == 3145728
    assert W.config(3).n_eq == 288


def test_plane_wave_normal_incidence_closed_form():
    # theta = 0, TE: E = y e^{jkz}, H = k x E = x e^{jkz}.  On the +z face (n = z):
    # J = n x H = y e^{jk h/2}, M = -n x E = x e^{jk h/2}; on the -z face both flip
    # sign and take the phase e^{-jk h/2}.
    c = W.config(1)
    g = W.box_geometry(c.n_patch)
    b = W.plane_wave_rhs(c, g)
    P = g.n_patch
    ph = np.exp(1j * W.K0 * W.BOX_H / 2)
    for p in range(P):
        if g.normal[p][2] == 1.0:
            assert np.allclose(b[0, 0, 0, 2 * p: 2 * p + 2], [0, ph], atol=1e-15)
            assert np.allclose(b[0, 0, 0, 2 * P + 2 * p: 2 * P + 2 * p + 2], [ph, 0], atol=1e-15)
        if g.normal[p][2] == -1.0:
            assert np.allclose(b[0, 0, 0, 2 * p: 2 * p + 2], [0, -np.conj(ph)], atol=1e-15)
            assert np.allclose(b[0, 0, 0, 2 * P + 2 * p: 2 * P + 2 * p + 2], [-np.conj(ph), 0], atol=1e-15)
    # normal incidence: every element sees the same excitation
    assert np.allclose(b[0], b[0, :1, :1], atol=1e-15)


def test_plane_wave_oblique_phase_progression():
    # theta = 30 deg: neighbouring elements along x differ by exp(-j k pitch sin(theta))
    c = W.config(2)
    b = W.plane_wave_rhs(W.Config(2, 3, 2, 48, 1, c.angles, 1e-8))
    shifted = b[0, :, :-1, :] * np.exp(-1j * W.K0 * W.PITCH * 0.5)
    assert np.allclose(b[0, :, 1:, :], shifted, atol=1e-14)
    assert np.abs(b).max() > 0.5
    # no phase progression along y at phi = 0
    assert np.allclose(b[0, 1], b[0, 0], atol=1e-15)


def test_serving_stream_ranges():
    cat = W.serving_catalogue(12)
    assert all(8 <= s.n <= 96 and s.n_patch in (24, 48, 72) for s in cat)
    reqs = W.serving_stream(50, rate_hz=10.0, n_surfaces=len(cat))
    assert all(0 <= r.surface < 12 and 1 <= r.nrhs <= 32 and len(r.angles) == r.nrhs for r in reqs)
    assert all(reqs[i].arrival_s < reqs[i + 1].arrival_s for i in range(len(reqs) - 1))
    fast = W.serving_stream(50, rate_hz=20.0, n_surfaces=len(cat))
    assert np.allclose([2 * f.arrival_s for f in fast], [r.arrival_s for r in reqs])
