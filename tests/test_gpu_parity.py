"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerance: FP64 results must match the oracle to 1e-12 relative (normwise per
right-hand side); FP32 results are reported and bounded loosely (their error
is set by FP32 rounding of the Fourier-domain blocks and FFTs)."""
import math

import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_per_rhs(y, yr):
    """Normwise relative error per right-hand side; a zero reference must be
    matched exactly (reported as 0 or inf)."""
    y = np.asarray(y).reshape(yr.shape[0], -1)
    yr = yr.reshape(yr.shape[0], -1)
    num = np.linalg.norm(y - yr, axis=1)
    den = np.linalg.norm(yr, axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num == 0, 0.0, np.inf))


def say(msg):
    print(msg, flush=True)


def random_plan(nx, ny, n, nrhs, seed, n_types=3, zero_self=True, store=3):
    e = E()
    B = W.random_blocks(nx, ny, n, seed=seed, zero_self=zero_self)
    S = W.random_types(n_types, n, seed=seed)
    tm = W.random_type_map(nx, ny, n_types, seed=seed)
    plan = e.emsurf_plan_create(nx, ny, n, n_types, nrhs, B, S, tm, store=store)
    return plan, B, S, tm


# ----------------------------------------------------------------------------- apply_T
@pytest.mark.parametrize("nx,ny,n,nrhs", [
    (1, 1, 4, 1), (2, 1, 3, 1), (1, 3, 5, 2), (3, 2, 7, 1), (5, 3, 6, 3), (4, 4, 16, 2),
    (9, 7, 10, 1), (17, 5, 12, 2), (33, 2, 8, 1), (2, 65, 4, 1), (129, 1, 3, 1), (6, 6, 130, 1),
    (3, 4, 257, 1), (8, 8, 40, 9), (5, 5, 33, 17),
    # padded lengths with a factor 3: 24, 48, 96, 192, 384, 768
    (10, 3, 5, 1), (20, 12, 6, 2), (33, 1, 4, 1), (65, 2, 3, 1), (130, 2, 2, 1), (300, 1, 2, 1), (24, 24, 4, 3),
    # padded lengths 512 and 1024 along either axis
    (200, 1, 3, 1), (3, 200, 2, 2), (400, 1, 2, 1), (2, 450, 2, 1), (257, 3, 2, 1),
])
def test_apply_T_fp64_random_blocks(nx, ny, n, nrhs):
    say(f"apply_T fp64 random {nx}x{ny} n={n} nrhs={nrhs}")
    e = E()
    plan, B, S, tm = random_plan(nx, ny, n, max(nrhs, 1), seed=nx * 100 + ny)
    x = W.random_vectors(nrhs, nx, ny, n, seed=7)
    y = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP64, nrhs, dev(x), y)
    torch.cuda.synchronize()
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    err = rel_per_rhs(y.cpu().numpy(), yr)
    say(f"  rel err per rhs {err}")
    assert np.all(err <= FP64_TOL)
    # nonzero self block is honoured too
    plan.destroy()


def test_apply_T_nonzero_self_block():
    e = E()
    nx, ny, n = 3, 2, 5
    plan, B, S, tm = random_plan(nx, ny, n, 1, seed=5, zero_self=False)
    x = W.random_vectors(1, nx, ny, n, seed=8)
    y = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP64, 1, dev(x), y)
    torch.cuda.synchronize()
    yr = C.apply_T_dense(B, x)
    assert rel_per_rhs(y.cpu().numpy(), yr).max() <= FP64_TOL


@pytest.mark.parametrize("nx,ny,n,nrhs", [
    (9, 6, 24, 3), (65, 17, 8, 2),
    # FP32 passes of 64, 128 and 256 points over >= 64 columns run 512-thread
    # workgroups: y passes at L = 64 (72 columns) and L = 256 (80, ragged),
    # x passes at L = 128 (70, ragged) and L = 256 (64)
    (32, 28, 24, 3), (50, 3, 70, 1), (100, 1, 64, 1), (2, 100, 40, 2),
    # padded lengths 512 and 1024
    (200, 2, 4, 1), (1, 400, 3, 2),
])
def test_apply_T_fp32_error_reported(nx, ny, n, nrhs):
    e = E()
    plan, B, S, tm = random_plan(nx, ny, n, nrhs, seed=3)
    x = W.random_vectors(nrhs, nx, ny, n, seed=9)
    y = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP32, nrhs, dev(x.astype(np.complex64)), y)
    torch.cuda.synchronize()
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    err = rel_per_rhs(y.cpu().numpy().astype(np.complex128), yr)
    say(f"apply_T fp32 rel err per rhs {err}")
    assert np.all(err <= 1e-5)


def test_apply_T_delta_columns():
    # T e_{m0,v} returns the columns T(m - m0)[:, v] for every element m
    e = E()
    nx, ny, n = 5, 4, 6
    plan, B, S, tm = random_plan(nx, ny, n, 1, seed=13)
    iy0, ix0, v = 2, 1, 4
    x = np.zeros((1, ny, nx, n), dtype=np.complex128)
    x[0, iy0, ix0, v] = 1.0
    y = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP64, 1, dev(x), y)
    torch.cuda.synchronize()
    yy = y.cpu().numpy()[0]
    for iy in range(ny):
        for ix in range(nx):
            col = B[iy - iy0 + ny - 1, ix - ix0 + nx - 1][:, v]
            assert np.allclose(yy[iy, ix], col, rtol=0, atol=1e-13)


def test_apply_T_shift_invariance():
    # a source pattern shifted inside the lattice gives the shifted response on the
    # region the lattice edges do not affect
    e = E()
    nx, ny, n = 8, 6, 5
    plan, B, S, tm = random_plan(nx, ny, n, 1, seed=17)
    x = np.zeros((1, ny, nx, n), dtype=np.complex128)
    rng = np.random.default_rng(1)
    x[0, 1:3, 1:3] = rng.standard_normal((2, 2, n)) + 1j * rng.standard_normal((2, 2, n))
    xs = np.roll(np.roll(x, 2, axis=1), 3, axis=2)
    y = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    ys = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP64, 1, dev(x), y)
    e.emsurf_apply_T(plan, e.EMSURF_FP64, 1, dev(xs), ys)
    torch.cuda.synchronize()
    a, b = y.cpu().numpy()[0], ys.cpu().numpy()[0]
    # response of x at (iy, ix) equals response of xs at (iy+2, ix+3), for all (iy, ix)
    # whose shifted position is inside the lattice
    assert np.allclose(b[2:, 3:], a[: ny - 2, : nx - 3], rtol=0, atol=1e-13 * np.abs(a).max())


# ----------------------------------------------------------------------------- Green fill
@pytest.mark.parametrize("npch,nx,ny", [(24, 3, 2), (48, 2, 3), (72, 2, 2)])
def test_green_fill_matches_oracle(npch, nx, ny):
    e = E()
    g = W.box_geometry(npch)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    n = g.n_eq
    Tb = torch.empty((2 * ny - 1, 2 * nx - 1, n, n), dtype=torch.complex128, device="cuda")
    e.emsurf_fill_T_point_green(geom, nx, ny, Tb)
    torch.cuda.synchronize()
    ref = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    got = Tb.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    assert np.array_equal(got == 0, ref == 0)


def test_plan_green_config1_fp64():
    e = E()
    c = W.config(1)
    g = W.box_geometry(c.n_patch)
    S, tm = W.s_types(c), W.type_map(c)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(c.nx, c.ny, c.n_types, 2, geom, S, tm)
    B = C.coupling_blocks(g.rho, g.area, g.tan, c.nx, c.ny, W.PITCH, W.K0)
    x = np.concatenate([W.plane_wave_rhs(c, g), W.random_vectors(1, c.nx, c.ny, c.n_eq, seed=1)])
    y = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP64, 2, dev(x), y)
    torch.cuda.synchronize()
    yr = C.apply_T_dense(B, x)
    err = rel_per_rhs(y.cpu().numpy(), yr)
    say(f"config 1 green apply_T fp64 rel err {err}")
    assert np.all(err <= FP64_TOL)


# ----------------------------------------------------------------------------- S and A
@pytest.mark.parametrize("nx,ny,n,nrhs,nt", [(3, 2, 5, 2, 3), (8, 8, 96, 1, 4), (7, 5, 70, 3, 5), (40, 1, 8, 1, 2),
                                              # several column blocks and row blocks per type, ragged tiles
                                              (9, 8, 192, 4, 3), (5, 4, 288, 9, 2), (17, 3, 20, 3, 1)])
def test_apply_S_and_A_fp64(nx, ny, n, nrhs, nt):
    e = E()
    plan, B, S, tm = random_plan(nx, ny, n, nrhs, seed=nx + ny, n_types=nt)
    x = W.random_vectors(nrhs, nx, ny, n, seed=11)
    y = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_apply_S(plan, e.EMSURF_FP64, nrhs, dev(x), y)
    torch.cuda.synchronize()
    ys = MM.apply_S(S, tm, x)
    assert rel_per_rhs(y.cpu().numpy(), ys).max() <= FP64_TOL
    e.emsurf_apply_A(plan, e.EMSURF_FP64, nrhs, dev(x), y)
    torch.cuda.synchronize()
    Tf = lambda v: C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], v)
    ya = MM.apply_A(Tf, S, tm, x)
    err = rel_per_rhs(y.cpu().numpy(), ya)
    say(f"apply_A fp64 {nx}x{ny} n={n}: {err}")
    assert err.max() <= FP64_TOL
    # in-place S apply (same buffer)
    xd = dev(x)
    e.emsurf_apply_S(plan, e.EMSURF_FP64, nrhs, xd, xd)
    torch.cuda.synchronize()
    assert rel_per_rhs(xd.cpu().numpy(), ys).max() <= FP64_TOL


@pytest.mark.parametrize("nx,ny,n,nrhs,nt", [(3, 2, 5, 2, 3), (9, 8, 192, 4, 3), (5, 4, 288, 16, 2), (17, 3, 20, 3, 1)])
def test_apply_S_fp32(nx, ny, n, nrhs, nt):
    # the FP32 matrix-core apply against the FP64 oracle (FP32 bar 1e-5)
    e = E()
    plan, B, S, tm = random_plan(nx, ny, n, nrhs, seed=nx * ny + n, n_types=nt)
    x = W.random_vectors(nrhs, nx, ny, n, seed=12)
    y = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    e.emsurf_apply_S(plan, e.EMSURF_FP32, nrhs, dev(x.astype(np.complex64)), y)
    torch.cuda.synchronize()
    err = rel_per_rhs(y.cpu().numpy().astype(np.complex128), MM.apply_S(S, tm, x))
    say(f"apply_S fp32 {nx}x{ny} n={n} nrhs={nrhs}: {err}")
    assert err.max() <= 1e-5


def test_apply_A_fp32_error_reported():
    e = E()
    nx, ny, n, nrhs = 6, 5, 48, 2
    plan, B, S, tm = random_plan(nx, ny, n, nrhs, seed=2)
    x = W.random_vectors(nrhs, nx, ny, n, seed=4)
    y = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    e.emsurf_apply_A(plan, e.EMSURF_FP32, nrhs, dev(x.astype(np.complex64)), y)
    torch.cuda.synchronize()
    Tf = lambda v: C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], v)
    ya = MM.apply_A(Tf, S, tm, x)
    err = rel_per_rhs(y.cpu().numpy().astype(np.complex128), ya)
    say(f"apply_A fp32 rel err {err}")
    assert err.max() <= 1e-5


# ----------------------------------------------------------------------------- errors
def test_argument_errors():
    e = E()
    plan, B, S, tm = random_plan(3, 2, 4, 2, seed=1)
    x = dev(W.random_vectors(2, 3, 2, 4, seed=1))
    y = torch.empty_like(x)
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_apply_T(plan, e.EMSURF_FP64, 3, x, y)       # nrhs > max_rhs
    assert ei.value.status == e.EMSURF_ERR_ARG
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_apply_T(plan, e.EMSURF_FP64, 1, x, x)       # aliasing
    assert ei.value.status == e.EMSURF_ERR_ARG
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_apply_T(plan, 7, 1, x, y)
    assert ei.value.status == e.EMSURF_ERR_ARG
    bad_tm = tm.copy()
    bad_tm[0, 0] = 99
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_plan_create(3, 2, 4, 3, 1, B, S, bad_tm)
    assert ei.value.status == e.EMSURF_ERR_ARG
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_plan_create(0, 2, 4, 3, 1, B, S, tm)
    assert ei.value.status == e.EMSURF_ERR_ARG
    p64 = e.emsurf_plan_create(3, 2, 4, 3, 1, B, S, tm, store=e.EMSURF_STORE_FP64)
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_apply_T(p64, e.EMSURF_FP32, 1, x.to(torch.complex64), y.to(torch.complex64))
    assert ei.value.status == e.EMSURF_ERR_UNSUPPORTED
    assert e.emsurf_plan_bytes(0, 1, 1, 1, 1) == 0
    assert e.emsurf_plan_bytes(4, 4, 96, 4, 1) > 0
