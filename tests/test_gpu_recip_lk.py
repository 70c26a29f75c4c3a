"""GPU parity of reciprocal structured plans (EMSURF_T_LK with recip = 1: one
[L | K] record per frequency pair {k, -k}, a quarter of the dense bytes)
against the FP64 oracle and against full structured plans, through the C ABI.

L and K are reciprocal one by one, X(-d) = D^-1 X(d)^T D; any constants
a, b, c, e are then served.  Bars as for the structured form: FP64 1e-12,
FP32 2e-5 relative per right-hand side.  Cases: random reciprocal L and K with
signed weights and random constants (ragged n_h, passes over the
right-hand sides, a 1 x 1 lattice), the device fill with its area weights,
the refusal of non-reciprocal blocks, solves against dense LU, and the
128 x 128 workload on sampled rows."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import coupling_lk as LK
from oracle import krylov as K
from oracle import macromodel as MM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 2e-5


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    """Largest normwise relative error over right-hand sides; a zero reference
    must be matched exactly."""
    a = np.asarray(a).reshape(b.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    return float(np.max(np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num == 0, 0.0, np.inf))))


def apply_both(e, plan, x, nrhs):
    x64 = dev(x)
    y64 = torch.empty_like(x64)
    e.emsurf_apply_T(plan, e.EMSURF_FP64, nrhs, x64, y64)
    x32 = x64.to(torch.complex64)
    y32 = torch.empty_like(x32)
    e.emsurf_apply_T(plan, e.EMSURF_FP32, nrhs, x32, y32)
    torch.cuda.synchronize()
    return y64.cpu().numpy(), y32.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("nx,ny,nh,nrhs", [(1, 1, 3, 1), (3, 2, 8, 2), (4, 3, 17, 3), (5, 4, 48, 4),
                                           (2, 3, 96, 9), (6, 2, 100, 5), (3, 5, 24, 6), (2, 2, 200, 3)])
def test_recip_lk_random_blocks(nx, ny, nh, nrhs):
    e = E()
    n = 2 * nh
    say(f"reciprocal LK (random L, K): {nx}x{ny}, n_h {nh}, {nrhs} RHS")
    w = W.random_weights(nh, seed=nh)
    T_in = W.random_reciprocal_lk_blocks(nx, ny, nh, w, seed=30 + nh)
    rng = np.random.default_rng(nh + 1)
    coef = tuple(complex(a, b) for a, b in rng.standard_normal((4, 2)))
    S = W.random_types(2, n, seed=3)
    tm = W.random_type_map(nx, ny, 2, seed=3)
    plan = e.emsurf_plan_create_reciprocal(nx, ny, n, 2, nrhs, T_in, w, S, tm, form=e.EMSURF_T_LK, coef=coef)
    full = e.emsurf_plan_create(nx, ny, n, 2, nrhs, T_in, S, tm, form=e.EMSURF_T_LK, coef=coef)
    st = plan.stats()
    ntr = -(-nh // 16)
    assert st.bytes_that64 == st.n_stored * ntr * 2 * ntr * 256 * 16
    x = W.random_vectors(nrhs, nx, ny, n, seed=nrhs + nh)
    blocks = LK.lk_assemble(T_in[:, :, 0], T_in[:, :, 1], coef)
    ref = C.apply_T_direct(lambda dy, dx: blocks[dy + ny - 1, dx + nx - 1], x)
    y64, y32 = apply_both(e, plan, x, nrhs)
    f64, _ = apply_both(e, full, x, nrhs)
    e64, e32, ef = rel(y64, ref), rel(y32, ref), rel(y64, f64)
    say(f"  {st.n_stored} of {st.n_freq} records; FP64 {e64:.2e}, FP32 {e32:.2e}, vs full plan {ef:.2e}")
    assert e64 <= FP64_TOL and e32 <= FP32_TOL and ef <= FP64_TOL
    plan.destroy()
    full.destroy()


@pytest.mark.parametrize("npch,nx,ny,nrhs", [(24, 5, 4, 4), (48, 3, 3, 2), (24, 1, 1, 1)])
def test_recip_lk_green(npch, nx, ny, nrhs):
    e = E()
    g = W.box_geometry(npch)
    n = 4 * npch
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    S = W.random_types(2, n, seed=5)
    tm = W.random_type_map(nx, ny, 2, seed=5)
    plan = e.emsurf_plan_create_green(nx, ny, 2, nrhs, geom, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF,
                                      recip=1)
    full = e.emsurf_plan_create_green(nx, ny, 2, nrhs, geom, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF)
    x = W.random_vectors(nrhs, nx, ny, n, seed=npch + nx)
    Lb, Kb = LK.lk_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    blocks = LK.lk_assemble(Lb, Kb, W.OUTER_COEF)
    ref = C.apply_T_direct(lambda dy, dx: blocks[dy + ny - 1, dx + nx - 1], x)
    y64, y32 = apply_both(e, plan, x, nrhs)
    f64, _ = apply_both(e, full, x, nrhs)
    e64, e32, ef = rel(y64, ref), rel(y32, ref), rel(y64, f64)
    say(f"reciprocal LK Green {nx}x{ny} npch {npch}: FP64 {e64:.2e}, FP32 {e32:.2e}, vs full plan {ef:.2e}")
    assert e64 <= FP64_TOL and e32 <= FP32_TOL and ef <= FP64_TOL
    plan.destroy()
    full.destroy()


def test_recip_lk_refuses_nonreciprocal_blocks():
    e = E()
    nx, ny, nh = 3, 3, 8
    n = 2 * nh
    w = W.random_weights(nh, seed=2)
    S = W.random_types(1, n, seed=2)
    tm = np.zeros((ny, nx), np.int32)
    good = W.random_reciprocal_lk_blocks(nx, ny, nh, w, seed=4)
    for part in (0, 1):
        bad = good.copy()
        bad[0, 1, part, 2, 3] += 0.1          # one entry of L or K at one offset
        with pytest.raises(e.EmsurfError) as ex:
            e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 1, bad, w, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF)
        assert ex.value.status == e.EMSURF_ERR_ARG
    # the right blocks under the wrong weights
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 1, good, w[::-1].copy(), S, tm, form=e.EMSURF_T_LK,
                                        coef=W.OUTER_COEF)
    assert ex.value.status == e.EMSURF_ERR_ARG
    p = e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 1, good, w, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF)
    p.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_recip_lk_solve_matches_lu(prec):
    e = E()
    nx, ny, npch = 4, 3, 24
    g = W.box_geometry(npch)
    n = 4 * npch
    S = W.random_types(3, n, seed=4)
    tm = W.random_type_map(nx, ny, 3, seed=4)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 3, 2, geom, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF, recip=1)
    Lb, Kb = LK.lk_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    A = np.eye(nx * ny * n) - MM.dense_S(S, tm) @ C.dense_T(LK.lk_assemble(Lb, Kb, W.OUTER_COEF), nx, ny)
    b = W.random_vectors(2, nx, ny, n, seed=9)
    xref = K.solve_dense(A, b.reshape(2, -1).T).T.reshape(b.shape)
    tol = 1e-10 if prec == "fp64" else 1e-6
    p = e.EMSURF_FP64 if prec == "fp64" else e.EMSURF_FP32_IR
    x = torch.zeros_like(dev(b))
    st, info = e.emsurf_solve(plan, e.solve_opts(p, tol=tol), 2, dev(b), x)
    say(f"reciprocal LK solve {prec}: {info}")
    assert st == e.EMSURF_OK and all(i["converged"] for i in info)
    assert rel(x.cpu().numpy(), xref) <= 10 * tol * np.linalg.cond(A)
    plan.destroy()


def test_recip_lk_fullsize_128x128_sampled():
    # the 128 x 128 workload (n_eq 192, 4 RHS) with the structured operator on
    # a reciprocal store; sampled rows against the oracle's row evaluation
    e = E()
    c = W.config(4)
    g = W.box_geometry(c.n_patch)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(c.nx, c.ny, c.n_types, c.nrhs, geom, W.s_types(c), W.type_map(c),
                                      form=e.EMSURF_T_LK, coef=W.OUTER_COEF, recip=1)
    st = plan.stats()
    say(f"reciprocal LK 128x128: {st.n_stored} records, FP32 store {st.bytes_that32 / 2**30:.2f} GiB")
    assert st.bytes_that32 == st.n_stored * 96 * 192 * 8
    b = W.plane_wave_rhs(c, g)
    y64, y32 = apply_both(e, plan, b, c.nrhs)
    elems = [(0, 127), (42, 64), (127, 0)]
    ref = LK.apply_T_elements_lk(g.rho, g.area, g.tan, W.PITCH, W.K0, W.OUTER_COEF, b, elems, chunk_rows=8)
    for i, (iy, ix) in enumerate(elems):
        e64 = float(np.linalg.norm(y64[:, iy, ix] - ref[i]) / np.linalg.norm(ref[i]))
        e32 = float(np.linalg.norm(y32[:, iy, ix] - ref[i]) / np.linalg.norm(ref[i]))
        say(f"  element ({iy},{ix}): FP64 {e64:.2e}, FP32 {e32:.2e}")
        assert e64 <= FP64_TOL and e32 <= FP32_TOL
    plan.destroy()
