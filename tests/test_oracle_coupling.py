"""Pins of the oracle's coupling operator against closed forms, invariants, the
paper's 1-D worked example and a library FFT convolution -- none of them a
retyping of the oracle's own fill or apply code."""
import math
import os

import numpy as np
import pytest

import workload as W
from oracle import coupling as C

HERE = os.path.dirname(os.path.abspath(__file__))


def _geom(npch=24):
    g = W.box_geometry(npch)
    return g, (g.rho, g.area, g.tan)


# ----------------------------------------------------------------------------- fill
def test_self_block_is_zero():
    g, G = _geom()
    assert np.count_nonzero(C.coupling_block(*G, 0, 0, W.PITCH, W.K0)) == 0


@pytest.mark.parametrize("d", [(0, 1), (1, 0), (0, -1), (-1, 0)])
def test_same_patch_one_pitch_closed_form(d):
    # identical patch on the neighbouring box: R = pitch = 1/2 wavelength, so
    # g = e^{-j pi} / (2 pi) = -1/(2 pi); the tangent product is 1, weight A_q.
    g, G = _geom()
    T = C.coupling_block(*G, d[0], d[1], W.PITCH, W.K0)
    P = g.n_patch
    for p in range(P):
        for a in range(2):
            for tau in range(2):
                u = tau * 2 * P + 2 * p + a
                assert abs(T[u, u] - (-g.area[p] / (2 * math.pi))) < 1e-15


def test_diagonal_neighbour_closed_form():
    g, G = _geom(48)
    T = C.coupling_block(*G, 1, 1, W.PITCH, W.K0)
    R = W.PITCH * math.sqrt(2.0)
    val = np.exp(-1j * 2 * math.pi * R) / (4 * math.pi * R)
    P = g.n_patch
    for p in range(P):
        assert abs(T[2 * p, 2 * p] - g.area[p] * val) < 1e-15


@pytest.mark.parametrize("dx,src_face,tst_face", [(-1, -1.0, +1.0), (+1, +1.0, -1.0)])
def test_gap_pair_is_the_strongest_entry(dx, src_face, tst_face):
    # d = test - source.  For dx = -1 the test box sits left of the source box, so
    # the test box's +x face looks at the source's -x face across the 0.05 gap.
    # Dividing out the source-area weight leaves the bare Green's function, whose
    # largest value is at the smallest distance: the facing pair across the gap.
    g, G = _geom()
    T = C.coupling_block(*G, 0, dx, W.PITCH, W.K0)
    P = g.n_patch
    a = np.tile(np.repeat(g.area, 2), 2)
    u, v = np.unravel_index(np.argmax(np.abs(T / a[None, :])), T.shape)
    p, q = (u % (2 * P)) // 2, (v % (2 * P)) // 2
    assert g.normal[p][0] == tst_face and g.normal[q][0] == src_face
    assert np.allclose(g.rho[p][1:], g.rho[q][1:])
    gap = W.PITCH - W.BOX_A
    expect = g.area[q] * np.exp(-1j * W.K0 * gap) / (4 * math.pi * gap)
    assert abs(abs(T[u, v]) - abs(expect)) < 1e-12 * abs(expect)
    assert abs(T[u, v] - expect) < 1e-12 * abs(expect)


def test_structural_zeros():
    g, G = _geom()
    T = C.coupling_block(*G, 1, -2, W.PITCH, W.K0)
    P = g.n_patch
    assert np.count_nonzero(T[: 2 * P, 2 * P:]) == 0       # J <- M
    assert np.count_nonzero(T[2 * P:, : 2 * P]) == 0       # M <- J
    assert np.array_equal(T[: 2 * P, : 2 * P], T[2 * P:, 2 * P:])
    # orthogonal tangents do not couple: top-face x-tangent vs side-face z-tangent
    for p in range(P):
        for q in range(P):
            for a in range(2):
                for b in range(2):
                    if abs(g.tan[p, a] @ g.tan[q, b]) < 1e-15:
                        assert T[2 * p + a, 2 * q + b] == 0


@pytest.mark.parametrize("d", [(0, 1), (2, -1), (-3, 2)])
def test_reciprocity(d):
    # Green's function reciprocity with source-area weights: T(-d)^T = D_A T(d) D_A^-1
    g, G = _geom(48)
    T = C.coupling_block(*G, d[0], d[1], W.PITCH, W.K0)
    Tm = C.coupling_block(*G, -d[0], -d[1], W.PITCH, W.K0)
    a = np.tile(np.repeat(g.area, 2), 2)
    assert np.allclose(Tm.T, (a[:, None] * T) / a[None, :], rtol=0, atol=1e-15)


def test_blocks_layout():
    g, G = _geom()
    B = C.coupling_blocks(*G, 3, 2, W.PITCH, W.K0)
    assert B.shape == (3, 5, 96, 96)
    for dy in (-1, 0, 1):
        for dx in (-2, 0, 2):
            assert np.array_equal(B[dy + 1, dx + 2], C.coupling_block(*G, dy, dx, W.PITCH, W.K0))


# ----------------------------------------------------------------------------- dense T
def test_dense_T_is_block_toeplitz():
    nx, ny, n = 3, 3, 4
    B = W.random_blocks(nx, ny, n, seed=1)
    T = C.dense_T(B, nx, ny)
    # shift by one element along x and along y: block (i, j) == block (i+s, j+s)
    def blk(m, mp):
        return T[m * n:(m + 1) * n, mp * n:(mp + 1) * n]
    for (m, mp), s in [((0, 4), 1), ((1, 3), 3), ((3, 0), 1), ((1, 7), 1), ((0, 5), 3)]:
        assert np.array_equal(blk(m, mp), blk(m + s, mp + s))
    assert np.count_nonzero(blk(4, 4)) == 0


def test_point_source_response_is_strongest_at_left_neighbour():
    # A unit J on the -x face of element (1, 2) radiates most strongly into the
    # element whose +x face looks at it across the gap: its left neighbour (1, 1).
    g, G = _geom()
    nx, ny = 4, 3
    B = C.coupling_blocks(*G, nx, ny, W.PITCH, W.K0)
    x = np.zeros((1, ny, nx, g.n_eq), dtype=np.complex128)
    q = int(np.where(g.normal[:, 0] == -1.0)[0][0])
    x[0, 1, 2, 2 * q] = 1.0
    y = C.apply_T_dense(B, x)
    mag = np.linalg.norm(y[0], axis=-1)
    assert np.unravel_index(np.argmax(mag), mag.shape) == (1, 1)


@pytest.mark.parametrize("nx,ny,nrhs", [(1, 1, 1), (3, 1, 2), (1, 4, 1), (3, 2, 3), (5, 3, 1)])
def test_dense_and_direct_agree(nx, ny, nrhs):
    n = 6
    B = W.random_blocks(nx, ny, n, seed=nx * 10 + ny)
    x = W.random_vectors(nrhs, nx, ny, n, seed=3)
    yd = C.apply_T_dense(B, x)
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    assert np.allclose(yd, yr, rtol=0, atol=1e-13 * np.abs(yd).max() + 1e-300)
    if nx * ny == 1:
        assert np.count_nonzero(yd) == 0


def test_library_fft_convolution_matches_direct():
    # 2-D generalisation (end of Sec. IV-B): circulant embedding on a padded grid,
    # kernel = T(d) at index d mod L (first column), products summed over the
    # local source index in the Fourier domain.  numpy.fft is the library route.
    nx, ny, n, nrhs = 5, 3, 6, 2
    B = W.random_blocks(nx, ny, n, seed=11)
    x = W.random_vectors(nrhs, nx, ny, n, seed=12)
    Ly, Lx = 2 * ny, 2 * nx
    K = np.zeros((Ly, Lx, n, n), dtype=np.complex128)
    for dy in range(-(ny - 1), ny):
        for dx in range(-(nx - 1), nx):
            K[dy % Ly, dx % Lx] = B[dy + ny - 1, dx + nx - 1]
    Kh = np.fft.fft2(K, axes=(0, 1))
    xp = np.zeros((nrhs, Ly, Lx, n), dtype=np.complex128)
    xp[:, :ny, :nx] = x
    xh = np.fft.fft2(xp, axes=(1, 2))
    yh = np.einsum("yxuv,ryxv->ryxu", Kh, xh)
    y = np.fft.ifft2(yh, axes=(1, 2))[:, :ny, :nx]
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    assert np.linalg.norm(y - yr) <= 1e-13 * np.linalg.norm(yr)


def test_sampled_elements_match_full_apply():
    g, G = _geom()
    nx, ny, nrhs = 4, 3, 2
    B = C.coupling_blocks(*G, nx, ny, W.PITCH, W.K0)
    x = W.random_vectors(nrhs, nx, ny, g.n_eq, seed=5)
    y = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    elems = [(0, 0), (2, 3), (1, 2)]
    ys = C.apply_T_elements(*G, W.PITCH, W.K0, x, elems, chunk_rows=2)
    ysb = C.apply_T_elements_from_blocks(B, x, elems)
    for e, (iy, ix) in enumerate(elems):
        assert np.allclose(ys[e], y[:, iy, ix], atol=1e-14)
        assert np.allclose(ysb[e], y[:, iy, ix], atol=1e-14)


# ----------------------------------------------------------------------------- paper 1-D example
def _load_golden():
    tabs, cur = {}, None
    with open(os.path.join(HERE, "golden", "paper_1d_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.isalpha() or line.startswith("LJV"):
                cur = line
                tabs[cur] = []
                continue
            tabs[cur].append(line.split())
    return tabs


def _paper_1d_L():
    """Oracle dense T of a 1 x 3 lattice with two local basis functions per box;
    L[m][n] with the paper's 1-based global ids (1,a)(2,b)(3,a)(4,b)(5,a)(6,b)."""
    B = W.random_blocks(3, 1, 2, seed=21, zero_self=False)
    T = C.dense_T(B, 3, 1)
    return B, (lambda lab: T[int(lab[0]) - 1, int(lab[1]) - 1]), T


def test_paper_1d_example_regrouping():
    tabs = _load_golden()
    B, L, T = _paper_1d_L()
    J = W.random_vectors(1, 3, 1, 2, seed=22).ravel()      # J_1..J_6 in global order
    order = [0, 2, 4, 1, 3, 5]                              # J1 J3 J5 | J2 J4 J6
    M1 = np.array([[L(e) for e in row] for row in tabs["LJV1"]])
    # regrouping is a symmetric permutation of the product (eq. LJV1 vs the one above it)
    assert np.allclose(M1 @ J[order], (T @ J)[order], atol=1e-15)


def test_paper_1d_example_circulant_and_fft():
    tabs = _load_golden()
    B, L, T = _paper_1d_L()
    C5 = np.array([[L(e) for e in row] for row in tabs["LJV3"]])
    # the printed embedding is a true circulant: C5[i][j] depends on (i - j) mod 5 only,
    # which holds only if the oracle's T is Toeplitz in the paper's (test, source) order
    col = C5[:, 0]
    for i in range(5):
        for j in range(5):
            assert C5[i, j] == col[(i - j) % 5]
    # its first column is [L11 L31 L51 L15 L13]
    assert [r[0] for r in tabs["LJV3"]] == ["11", "31", "51", "15", "13"]
    J = W.random_vectors(1, 3, 1, 2, seed=23).ravel()
    Ja = np.array([J[0], J[2], J[4], 0, 0])
    direct = C5 @ Ja
    via_fft = np.fft.ifft(np.fft.fft(col) * np.fft.fft(Ja))          # eq. (LJV5), first column
    assert np.allclose(via_fft, direct, atol=1e-15)
    # the top three entries are L^aa J^a taken from the oracle's dense T
    Laa = T[np.ix_([0, 2, 4], [0, 2, 4])]
    assert np.allclose(direct[:3], Laa @ J[[0, 2, 4]], atol=1e-15)
    # "four 1-D FFTs": aa + ab products summed in the Fourier domain give the
    # a-rows of the full oracle product
    def circ_col(i_loc, j_loc):
        # first column of the circulant of block L^{ij}: [c(0) c(1) c(2) c(-2) c(-1)]
        return np.array([B[0, d + 2, i_loc, j_loc] for d in (0, 1, 2, -2, -1)])
    Jb = np.array([J[1], J[3], J[5], 0, 0])
    acc = np.fft.fft(circ_col(0, 0)) * np.fft.fft(Ja) + np.fft.fft(circ_col(0, 1)) * np.fft.fft(Jb)
    ya = np.fft.ifft(acc)[:3]
    assert np.allclose(ya, (T @ J)[[0, 2, 4]], atol=1e-14)


def test_paper_1d_example_first_row_reading_fails():
    # Taken literally, eq. (LJV5) transforms the circulant's first ROW; for
    # non-symmetric blocks that is the transposed convolution and gives O(1) error.
    tabs = _load_golden()
    B, L, T = _paper_1d_L()
    C5 = np.array([[L(e) for e in row] for row in tabs["LJV3"]])
    J = W.random_vectors(1, 3, 1, 2, seed=24).ravel()
    Ja = np.array([J[0], J[2], J[4], 0, 0])
    good = C5 @ Ja
    wrong = np.fft.ifft(np.fft.fft(C5[0, :]) * np.fft.fft(Ja))
    assert np.linalg.norm(wrong[:3] - good[:3]) > 1e-2 * np.linalg.norm(good[:3])


@pytest.mark.parametrize("nx,ny,Lx,Ly", [(3, 2, 6, 4), (2, 2, 3, 3), (5, 3, 12, 6), (4, 1, 8, 1)])
def test_spectral_reciprocity_of_the_circulant_embedding(nx, ny, Lx, Ly):
    # With T(-d) = W^-1 T(d)^T W the kernel spectrum obeys That[-k] = W^-1 That[k]^T W
    # (library FFT of the zero-padded circulant embedding, padded lengths even and
    # odd); this is what lets a plan keep one block per pair {k, -k}.
    g, G = _geom(24)
    B = C.coupling_blocks(*G, nx, ny, W.PITCH, W.K0)
    w = np.tile(np.repeat(g.area, 2), 2)
    n = B.shape[-1]
    K = np.zeros((Ly, Lx, n, n), dtype=np.complex128)
    for dy in range(-(ny - 1), ny):
        for dx in range(-(nx - 1), nx):
            K[dy % Ly, dx % Lx] = B[dy + ny - 1, dx + nx - 1]
    Kh = np.fft.fft2(K, axes=(0, 1))
    scale = np.abs(Kh).max()
    for ky in range(Ly):
        for kx in range(Lx):
            mine = Kh[(-ky) % Ly, (-kx) % Lx]
            mirrored = (Kh[ky, kx].T * w[None, :]) / w[:, None]
            assert np.abs(mine - mirrored).max() <= 1e-13 * scale
    # a non-reciprocal operator does not have the property
    Bn = W.random_blocks(nx, ny, n, seed=3)
    Kn = np.zeros_like(K)
    for dy in range(-(ny - 1), ny):
        for dx in range(-(nx - 1), nx):
            Kn[dy % Ly, dx % Lx] = Bn[dy + ny - 1, dx + nx - 1]
    Knh = np.fft.fft2(Kn, axes=(0, 1))
    if nx * ny > 1:
        assert np.abs(Knh[(-1) % Ly, (-1) % Lx] - Knh[1 % Ly, 1 % Lx].T).max() > 1e-3


def test_reciprocal_workload_blocks_satisfy_the_identity():
    # the seeded reciprocal generator used by the GPU tests honours its contract
    w = W.random_weights(9, seed=2)
    B = W.random_reciprocal_blocks(4, 3, 9, w, seed=5, zero_self=False)
    for dy in range(-2, 3):
        for dx in range(-3, 4):
            T, Tm = B[dy + 2, dx + 3], B[-dy + 2, -dx + 3]
            assert np.abs(Tm - np.diag(1 / w) @ T.T @ np.diag(w)).max() <= 1e-15
    assert np.abs(B[2, 3]).max() > 0
