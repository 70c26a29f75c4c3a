"""GPU GMRES solves through the C ABI, checked against the oracle (dense LU,
oracle GMRES, closed forms) and the true residual of the FP64 oracle operator."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(msg):
    print(msg, flush=True)


def physical(nx, ny, npch=24, n_types=4, seed=0, max_rhs=2, cfg=None):
    e = E()
    if cfg is not None:
        c = W.config(cfg)
        nx, ny, npch, n_types = c.nx, c.ny, c.n_patch, c.n_types
        S, tm = W.s_types(c), W.type_map(c)
    else:
        S = W.random_types(n_types, 4 * npch, seed=seed)
        tm = W.random_type_map(nx, ny, n_types, seed=seed)
    g = W.box_geometry(npch)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, n_types, max_rhs, geom, S, tm)
    return plan, g, S, tm


def dense_A(g, S, tm, nx, ny):
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    return np.eye(nx * ny * g.n_eq) - MM.dense_S(S, tm) @ C.dense_T(B, nx, ny), B


def test_config1_fp64_matches_lu_and_oracle_gmres():
    e = E()
    c = W.config(1)
    plan, g, S, tm = physical(0, 0, cfg=1)
    b = W.plane_wave_rhs(c, g)
    A, B = dense_A(g, S, tm, c.nx, c.ny)
    x_lu = K.solve_dense(A, b.ravel())
    # to the paper-config tolerance: iteration count equals the oracle GMRES
    xd = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=c.tol), 1, dev(b), xd)
    Af = lambda v: (A @ v.ravel()).reshape(v.shape)
    xo, io = K.gmres(lambda v: A @ v, b.ravel(), c.tol)
    say(f"config1 fp64 tol {c.tol}: gpu iters {info[0]['iters']} oracle iters {io.iters} rel {info[0]['rel_res_true']:.2e}")
    assert st == e.EMSURF_OK and info[0]["converged"]
    assert info[0]["iters"] == io.iters
    x = xd.cpu().numpy().ravel()
    assert np.linalg.norm(A @ x - b.ravel()) <= c.tol * np.linalg.norm(b)
    assert np.linalg.norm(x - xo) <= 1e-9 * np.linalg.norm(xo)
    # to 1e-14: matches LU to 1e-12 (cond(A) is about 1.1)
    xd.zero_()
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-14), 1, dev(b), xd)
    x = xd.cpu().numpy().ravel()
    err = np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu)
    say(f"config1 fp64 tol 1e-14: iters {info[0]['iters']} err vs LU {err:.2e}")
    assert st == e.EMSURF_OK and err <= 1e-12


def test_single_element_and_zero_rhs():
    e = E()
    plan, g, S, tm = physical(1, 1, max_rhs=2)
    b = np.concatenate([W.random_vectors(1, 1, 1, g.n_eq, seed=3), np.zeros((1, 1, 1, g.n_eq), complex)])
    xd = torch.empty(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-12), 2, dev(b), xd)
    x = xd.cpu().numpy()
    assert st == e.EMSURF_OK
    assert info[0]["iters"] == 1 and np.allclose(x[0], b[0], atol=1e-15)     # A = I: lucky breakdown
    assert info[1]["iters"] == 0 and info[1]["converged"] and not np.any(x[1])


def test_single_scatterer_closed_form():
    e = E()
    nx, ny, npch = 4, 3, 24
    g = W.box_geometry(npch)
    n = g.n_eq
    S = np.stack([np.zeros((n, n), complex), W.random_types(1, n, seed=5)[0]])
    tm = np.zeros((ny, nx), np.int32)
    tm[1, 2] = 1
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 2, 1, geom, S, tm)
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    b = W.plane_wave_rhs(W.small_config(nx, ny, npch))
    closed = b + MM.apply_S(S, tm, C.apply_T_dense(B, b))
    xd = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-14), 1, dev(b), xd)
    x = xd.cpu().numpy()
    say(f"single scatterer: iters {info[0]['iters']}")
    assert st == e.EMSURF_OK and info[0]["iters"] <= 2
    assert np.linalg.norm(x - closed) <= 1e-12 * np.linalg.norm(closed)


def test_multi_rhs_independent_and_match_single():
    # each right-hand side of a batched solve equals its own single solve
    e = E()
    nx, ny = 5, 4
    plan, g, S, tm = physical(nx, ny, max_rhs=3, seed=2)
    cfg = W.small_config(nx, ny, 24, nrhs=3)
    b = W.plane_wave_rhs(cfg, g)
    b[2] *= 1e-3                                   # different scale, different convergence path
    xd = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-10), 3, dev(b), xd)
    assert st == e.EMSURF_OK
    xb = xd.cpu().numpy()
    A, B = dense_A(g, S, tm, nx, ny)
    for r in range(3):
        x1 = torch.zeros((1,) + b.shape[1:], dtype=torch.complex128, device="cuda")
        st1, info1 = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-10), 1, dev(b[r:r + 1]), x1)
        assert info1[0]["iters"] == info[r]["iters"]
        assert np.array_equal(x1.cpu().numpy()[0], xb[r])
        assert np.linalg.norm(A @ xb[r].ravel() - b[r].ravel()) <= 1e-10 * np.linalg.norm(b[r])


def test_restart_and_use_x0():
    e = E()
    nx, ny = 6, 5
    plan, g, S, tm = physical(nx, ny, max_rhs=1, seed=4)
    b = W.plane_wave_rhs(W.small_config(nx, ny, 24), g)
    A, B = dense_A(g, S, tm, nx, ny)
    xd = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-12, restart=2), 1, dev(b), xd)
    xo, io = K.gmres(lambda v: A @ v, b.ravel(), 1e-12, restart=2)
    say(f"restart=2: gpu iters {info[0]['iters']} cycles {info[0]['outer_iters']} oracle {io.iters}/{io.restarts}")
    assert st == e.EMSURF_OK and info[0]["outer_iters"] > 1
    assert info[0]["iters"] == io.iters
    assert np.linalg.norm(A @ xd.cpu().numpy().ravel() - b.ravel()) <= 1e-12 * np.linalg.norm(b)
    # warm restart from the converged x: zero further Arnoldi steps
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-12, use_x0=1), 1, dev(b), xd)
    assert st == e.EMSURF_OK and info[0]["iters"] == 0


def test_not_converged_and_bad_rhs():
    e = E()
    nx, ny = 3, 3
    plan, g, S, tm = physical(nx, ny, max_rhs=1, seed=6)
    b = W.plane_wave_rhs(W.small_config(nx, ny, 24), g)
    xd = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-30, max_iter=1), 1, dev(b), xd)
    assert st == e.EMSURF_ERR_NOT_CONVERGED and info[0]["iters"] == 1 and not info[0]["converged"]
    assert torch.linalg.norm(xd).item() > 0
    bad = b.copy()
    bad[0, 0, 0, 0] = np.nan
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-8), 1, dev(bad), xd)
    assert ei.value.status == e.EMSURF_ERR_ARG


def test_fp32_ir_reaches_1e6_and_fp32_solve():
    e = E()
    nx, ny = 8, 8
    plan, g, S, tm = physical(nx, ny, npch=48, max_rhs=2, seed=8)
    cfg = W.small_config(nx, ny, 48, nrhs=2)
    b = W.plane_wave_rhs(cfg, g)
    A, B = dense_A(g, S, tm, nx, ny)
    xd = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP32_IR, tol=1e-6), 2, dev(b), xd)
    x = xd.cpu().numpy()
    for r in range(2):
        res = np.linalg.norm(A @ x[r].ravel() - b[r].ravel()) / np.linalg.norm(b[r])
        say(f"fp32+IR rhs {r}: iters {info[r]['iters']} outer {info[r]['outer_iters']} oracle residual {res:.2e}")
        assert res <= 1e-6
    assert st == e.EMSURF_OK
    # tighter: IR keeps refining to 1e-10 with the FP64 residual
    xd.zero_()
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP32_IR, tol=1e-10, max_outer=20), 2, dev(b), xd)
    x = xd.cpu().numpy()
    for r in range(2):
        assert np.linalg.norm(A @ x[r].ravel() - b[r].ravel()) <= 1e-10 * np.linalg.norm(b[r])
    # plain FP32 solve: residual w.r.t. the FP64 operator limited by FP32 rounding
    xd.zero_()
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP32, tol=1e-5), 2, dev(b), xd)
    x = xd.cpu().numpy()
    res = max(np.linalg.norm(A @ x[r].ravel() - b[r].ravel()) / np.linalg.norm(b[r]) for r in range(2))
    say(f"fp32 solve: residual vs FP64 operator {res:.2e}")
    assert st == e.EMSURF_OK and res <= 1e-4


def test_solve_workspace_reused_across_calls():
    # the GMRES workspace stays in the plan per stream: solves with a growing and
    # then shrinking nrhs and restart on one plan each match LU, and the plan
    # reports the cached bytes after the first solve
    e = E()
    nx, ny = 3, 2
    plan, g, S, tm = physical(nx, ny, max_rhs=4, seed=7)
    A, _ = dense_A(g, S, tm, nx, ny)
    before = plan.stats().bytes_total
    for nrhs, restart, prec in [(1, 5, e.EMSURF_FP64), (4, 12, e.EMSURF_FP32_IR), (2, 3, e.EMSURF_FP64),
                                (4, 30, e.EMSURF_FP64), (1, 8, e.EMSURF_FP32_IR)]:
        b = W.random_vectors(nrhs, nx, ny, 4 * g.n_patch, seed=nrhs * 10 + restart)
        x = torch.zeros_like(dev(b))
        st, info = e.emsurf_solve(plan, e.solve_opts(prec, tol=1e-10, restart=restart), nrhs, dev(b), x)
        assert st == e.EMSURF_OK
        xs = x.cpu().numpy()
        for r in range(nrhs):
            xref = K.solve_dense(A, b[r].ravel())
            err = float(np.linalg.norm(xs[r].ravel() - xref) / np.linalg.norm(xref))
            say(f"reused workspace: nrhs {nrhs} restart {restart} prec {prec} rhs {r}: error vs LU {err:.2e}")
            assert err <= 1e-8
    assert plan.stats().bytes_total > before
