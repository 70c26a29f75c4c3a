"""GPU parity of the near-field right preconditioner (Sec. IV-A, eq.
(final_precond)) through the C ABI against the oracle (oracle/nearfield.py):
P^-1 y tile by tile at 1e-12 (FP64), right-preconditioned solves against
dense LU and the oracle's preconditioned GMRES iteration counts, argument
errors, and sampled tiles of the 128 x 128 workload."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM
from oracle import nearfield as NF

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
LAM10, LAM6 = 0.1 * W.WAVELENGTH, W.WAVELENGTH / 6


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(msg):
    print(msg, flush=True)


def rel_per_rhs(y, yr):
    y = np.asarray(y).reshape(yr.shape[0], -1)
    yr = yr.reshape(yr.shape[0], -1)
    return np.linalg.norm(y - yr, axis=1) / np.linalg.norm(yr, axis=1)


def green_case(e, nx, ny, npch, n_types, nrhs, seed):
    g = W.box_geometry(npch)
    S = W.random_types(n_types, g.n_eq, seed=seed)
    tm = W.random_type_map(nx, ny, n_types, seed=seed)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, n_types, nrhs, geom, S, tm)
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    T_of = lambda dy, dx: B[dy + ny - 1, dx + nx - 1]
    return g, geom, S, tm, plan, B, T_of


@pytest.mark.parametrize("nx,ny,npch,tile,delta,nrhs", [
    (3, 2, 24, (2, 2), LAM10, 1), (5, 4, 24, (2, 2), LAM6, 3), (4, 3, 24, (4, 3), LAM6, 2),
    (6, 5, 48, (3, 2), LAM6, 1), (7, 3, 72, (2, 2), 0.12, 5), (2, 2, 24, (1, 1), LAM6, 1),
])
def test_precond_apply_green_matches_oracle(nx, ny, npch, tile, delta, nrhs):
    e = E()
    g, geom, S, tm, plan, B, T_of = green_case(e, nx, ny, npch, 3, nrhs, seed=nx * 10 + ny)
    pc = e.emsurf_precond_create(plan, geom, delta, tile[0], tile[1])
    st = pc.stats()
    say(f"precond {nx}x{ny} npch {npch} tile {tile} delta {delta:.3f}: {st}")
    y = W.random_vectors(nrhs, nx, ny, g.n_eq, seed=3)
    x = torch.empty(y.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_precond_apply(pc, nrhs, dev(y), x)
    torch.cuda.synchronize()
    Tnf = NF.near_field_blocks(T_of, g.rho, W.PITCH, delta, nx, ny)
    xr = NF.apply_Pinv(S, tm, Tnf, tile[0], tile[1], y)
    err = rel_per_rhs(x.cpu().numpy(), xr)
    say(f"  rel err per rhs {err}")
    assert np.all(err <= FP64_TOL)
    if tile == (1, 1):
        # single-element tiles have no near pair inside a tile: P = I
        assert st["nq_max"] == 0 and np.array_equal(x.cpu().numpy(), y)
    pc.destroy()
    plan.destroy()


@pytest.mark.parametrize("n,tile", [(8, (2, 2)), (12, (3, 2))])
def test_precond_apply_caller_blocks_matches_oracle(n, tile):
    # random dense non-symmetric coupling blocks, the geometric near-field mask
    # of a synthetic box with n_eq / 4 patches (here the 24-patch box's first
    # n / 4 patch centres)
    e = E()
    nx, ny, nrhs = 5, 3, 2
    g = W.box_geometry(24)
    npch = n // 4
    rho, area, tan = g.rho[:npch].copy(), g.area[:npch].copy(), g.tan[:npch].copy()
    geom = e.Geometry(rho, area, tan, W.PITCH, W.K0)
    B = W.random_blocks(nx, ny, n, seed=7)
    S = W.random_types(2, n, seed=7)
    tm = W.random_type_map(nx, ny, 2, seed=7)
    plan = e.emsurf_plan_create(nx, ny, n, 2, nrhs, B, S, tm)
    T_near = np.stack([np.stack([B[dy + ny - 1, dx + nx - 1] for dx in (-1, 0, 1)]) for dy in (-1, 0, 1)])
    # top-face patches of adjacent boxes are 0.275 apart, diagonal ones 0.39
    pc = e.emsurf_precond_create(plan, geom, 0.3, tile[0], tile[1], T_near=T_near)
    T_of = lambda dy, dx: B[dy + ny - 1, dx + nx - 1]
    Tnf = NF.near_field_blocks(T_of, rho, W.PITCH, 0.3, nx, ny)
    assert any(np.any(v) for v in Tnf.values())
    y = W.random_vectors(nrhs, nx, ny, n, seed=8)
    x = torch.empty(y.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_precond_apply(pc, nrhs, dev(y), x)
    torch.cuda.synchronize()
    err = rel_per_rhs(x.cpu().numpy(), NF.apply_Pinv(S, tm, Tnf, tile[0], tile[1], y))
    say(f"caller blocks n {n} tile {tile}: rel err {err}")
    assert np.all(err <= FP64_TOL)
    pc.destroy()
    plan.destroy()


@pytest.mark.parametrize("tile", [(2, 2), (4, 3)])
def test_solve_precond_matches_lu_and_oracle_iterations(tile):
    e = E()
    nx, ny = 4, 3
    g, geom, S, tm, plan, B, T_of = green_case(e, nx, ny, 24, 3, 2, seed=8)
    cfg = W.small_config(nx, ny, 24, 3, 2, seed=9)
    b = W.plane_wave_rhs(cfg, g)
    pc = e.emsurf_precond_create(plan, geom, LAM6, tile[0], tile[1])
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve_precond(plan, pc, e.solve_opts(e.EMSURF_FP64, tol=1e-12), 2, dev(b), x)
    x0 = torch.zeros_like(x)
    st0, info0 = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-12), 2, dev(b), x0)
    torch.cuda.synchronize()
    say(f"tile {tile}: preconditioned iterations {[i['iters'] for i in info]}, plain {[i['iters'] for i in info0]}")
    assert st == e.EMSURF_OK
    A = np.eye(nx * ny * g.n_eq) - MM.dense_S(S, tm) @ C.dense_T(B, nx, ny)
    Tnf = NF.near_field_blocks(T_of, g.rho, W.PITCH, LAM6, nx, ny)
    Af = lambda v: MM.apply_A(lambda z: C.apply_T_dense(B, z), S, tm, v.reshape(b[:1].shape)).ravel()
    Minv = lambda v: NF.apply_Pinv(S, tm, Tnf, tile[0], tile[1], v.reshape(b[:1].shape)).ravel()
    xs = x.cpu().numpy()
    for r in range(2):
        x_lu = K.solve_dense(A, b[r].ravel())
        assert np.linalg.norm(xs[r].ravel() - x_lu) <= 1e-10 * np.linalg.norm(x_lu)
        _, io = K.gmres(Af, b[r].ravel(), 1e-12, M_inv=Minv)
        assert info[r]["iters"] == io.iters, (r, info[r]["iters"], io.iters)
        assert info[r]["iters"] <= info0[r]["iters"]
    # FP32 inner solves with FP64 refinement, preconditioned
    xi = torch.zeros_like(x)
    st2, info2 = e.emsurf_solve_precond(plan, pc, e.solve_opts(e.EMSURF_FP32_IR, tol=1e-7), 2, dev(b), xi)
    torch.cuda.synchronize()
    assert st2 == e.EMSURF_OK
    for r in range(2):
        res = np.linalg.norm(A @ xi.cpu().numpy()[r].ravel() - b[r].ravel()) / np.linalg.norm(b[r])
        assert info2[r]["converged"] and res <= 1e-7
    pc.destroy()
    plan.destroy()


def test_precond_zero_distance_is_identity_and_keeps_the_solve():
    e = E()
    nx, ny = 3, 3
    g, geom, S, tm, plan, B, T_of = green_case(e, nx, ny, 24, 2, 1, seed=2)
    pc = e.emsurf_precond_create(plan, geom, 0.0, 2, 2)
    assert pc.stats()["nq_max"] == 0 and pc.stats()["near_entries"] == 0
    b = W.plane_wave_rhs(W.small_config(nx, ny, 24, 2, 1, seed=3), g)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    x0 = torch.zeros_like(x)
    _, info = e.emsurf_solve_precond(plan, pc, e.solve_opts(e.EMSURF_FP64, tol=1e-12), 1, dev(b), x)
    _, info0 = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-12), 1, dev(b), x0)
    torch.cuda.synchronize()
    assert info[0]["iters"] == info0[0]["iters"]
    assert torch.linalg.norm(x - x0).item() <= 1e-13 * torch.linalg.norm(x0).item()
    pc.destroy()
    plan.destroy()


def test_precond_argument_errors():
    e = E()
    g, geom, S, tm, plan, B, T_of = green_case(e, 3, 2, 24, 2, 1, seed=4)
    _, geom2, _, _, plan2, _, _ = green_case(e, 3, 2, 24, 2, 1, seed=5)
    for args in [(0.8, 2, 2), (-1.0, 2, 2), (LAM10, 0, 2), (LAM10, 9, 8)]:
        with pytest.raises(e.EmsurfError) as ei:
            e.emsurf_precond_create(plan, geom, *args)
        assert ei.value.status == e.EMSURF_ERR_ARG
    pc2 = e.emsurf_precond_create(plan2, geom2, LAM10, 2, 2)
    b = torch.zeros((1, 2, 3, g.n_eq), dtype=torch.complex128, device="cuda")
    b[0, 0, 0, 0] = 1
    x = torch.zeros_like(b)
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_solve_precond(plan, pc2, e.solve_opts(e.EMSURF_FP64, tol=1e-10), 1, b, x)
    assert ei.value.status == e.EMSURF_ERR_ARG
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_precond_apply(pc2, 2, b, x)
    assert ei.value.status == e.EMSURF_ERR_ARG
    pc2.destroy()
    plan.destroy()
    plan2.destroy()


def test_precond_fullsize_128x128_sampled_tiles_and_solves():
    """The 128 x 128, n_eq 192, 4-RHS workload with Delta_NF = lambda/10 and
    2 x 2 tiles: P^-1 y at sampled tiles against the oracle's dense tile
    solve, and both preconditioned solves reach 1e-6."""
    e = E()
    c = W.config(4)
    g = W.box_geometry(c.n_patch)
    S, tm = W.s_types(c), W.type_map(c)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(c.nx, c.ny, c.n_types, c.nrhs, geom, S, tm, recip=1)
    pc = e.emsurf_precond_create(plan, geom, LAM10, 2, 2)
    st = pc.stats()
    say(f"128x128 precond: {st}")
    b = W.plane_wave_rhs(c, g)
    y = dev(b)
    x = torch.empty_like(y)
    e.emsurf_precond_apply(pc, c.nrhs, y, x)
    torch.cuda.synchronize()
    xs = x.cpu().numpy()
    blocks = {d: C.coupling_block(g.rho, g.area, g.tan, d[0], d[1], W.PITCH, W.K0) for d in NF.OFFSETS}
    Tnf = NF.near_field_blocks(lambda dy, dx: blocks[(dy, dx)], g.rho, W.PITCH, LAM10)
    for (ty0, tx0) in [(0, 0), (64, 126), (126, 30)]:
        elems = [(iy, ix) for iy in (ty0, ty0 + 1) for ix in (tx0, tx0 + 1)]
        Pm = NF.tile_matrix(S, tm, Tnf, elems)
        rows = np.stack([b[:, iy, ix, :] for iy, ix in elems], axis=1).reshape(c.nrhs, -1)
        ref = np.linalg.solve(Pm, rows.T).T
        got = np.stack([xs[:, iy, ix, :] for iy, ix in elems], axis=1).reshape(c.nrhs, -1)
        err = rel_per_rhs(got, ref)
        say(f"  tile at ({ty0},{tx0}): rel err {err}")
        assert np.all(err <= FP64_TOL)
    for prec in (e.EMSURF_FP32_IR, e.EMSURF_FP64):
        xx = torch.zeros_like(y)
        stt, info = e.emsurf_solve_precond(plan, pc, e.solve_opts(prec, tol=c.tol), c.nrhs, y, xx)
        torch.cuda.synchronize()
        say(f"  preconditioned solve prec {prec}: {e.emsurf_status_str(stt)} {[i['iters'] for i in info]}")
        assert stt == e.EMSURF_OK and all(i["converged"] and i["rel_res_true"] <= c.tol for i in info)
    pc.destroy()
    plan.destroy()
