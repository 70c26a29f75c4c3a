"""GPU parity of reciprocal plans (one Fourier-domain block per frequency pair
{k, -k}, paired block products) against the FP64 oracle, through the C ABI.

The operator is the same as for a full plan; only the storage and the block
product differ.  Bars: FP64 1e-12 relative per right-hand side against the
oracle's direct sum over offsets (and against a full plan on the same blocks);
FP32 1e-5 against the oracle (2e-5 per sampled element at full size).  Cases
cover padded lengths 1, 3 and 3 * 2^a (odd lengths have one self-paired index,
even ones two), n_eq not a multiple of the row-lane count, every column split
(n_eq up to 512), passes over the right-hand sides, signed weights, the Green
fill with area weights, and the argument checks."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(msg):
    print(msg, flush=True)


def rel_per_rhs(y, yr):
    """Normwise relative error per right-hand side; a zero reference (1 x 1
    lattice, T(0) = 0) must be matched exactly."""
    y = np.asarray(y).reshape(yr.shape[0], -1)
    yr = yr.reshape(yr.shape[0], -1)
    num = np.linalg.norm(y - yr, axis=1)
    den = np.linalg.norm(yr, axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num == 0, 0.0, np.inf))


def recip_plan(nx, ny, n, nrhs, seed, signed=True, zero_self=True, n_types=2, store=3):
    e = E()
    w = W.random_weights(n, seed, signed=signed)
    B = W.random_reciprocal_blocks(nx, ny, n, w, seed, zero_self=zero_self)
    S = W.random_types(n_types, n, seed=seed)
    tm = W.random_type_map(nx, ny, n_types, seed=seed)
    plan = e.emsurf_plan_create_reciprocal(nx, ny, n, n_types, nrhs, B, w, S, tm, store=store)
    return plan, B, w, S, tm


def apply(e, plan, prec, x):
    dt = torch.complex128 if prec == e.EMSURF_FP64 else torch.complex64
    xd = dev(x).to(dt)
    y = torch.empty_like(xd)
    e.emsurf_apply_T(plan, prec, x.shape[0], xd, y)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("nx,ny,n,nrhs", [
    (1, 1, 4, 1), (2, 1, 3, 1), (1, 2, 5, 2), (2, 2, 7, 1), (3, 2, 6, 3), (5, 4, 16, 4),
    (9, 7, 10, 1), (17, 5, 12, 2), (2, 33, 8, 1), (6, 6, 97, 2), (4, 3, 130, 1), (3, 3, 193, 4),
    (3, 2, 200, 2), (2, 2, 385, 1), (2, 2, 512, 1), (8, 8, 40, 9), (5, 5, 33, 17), (10, 3, 5, 5),
    (20, 12, 6, 2), (24, 24, 4, 3), (65, 2, 3, 1),
    # padded lengths 512 and 1024 (pairs k, -k across the long axis)
    (200, 1, 3, 1), (1, 400, 2, 2),
])
def test_recip_apply_T_fp64_random_blocks(nx, ny, n, nrhs):
    say(f"reciprocal apply_T fp64 {nx}x{ny} n={n} nrhs={nrhs}")
    e = E()
    plan, B, w, S, tm = recip_plan(nx, ny, n, nrhs, seed=nx * 100 + ny + n)
    st = plan.stats()
    P = st.Lx * st.Ly
    self_paired = (2 if st.Lx % 2 == 0 else 1) * (2 if st.Ly % 2 == 0 else 1)
    assert st.n_stored == (P + self_paired) // 2
    x = W.random_vectors(nrhs, nx, ny, n, seed=7)
    y = apply(e, plan, e.EMSURF_FP64, x)
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    err = rel_per_rhs(y, yr)
    say(f"  Lx {st.Lx} Ly {st.Ly}, {st.n_stored} of {P} blocks stored, rel err per rhs {err}")
    assert np.all(err <= FP64_TOL)
    plan.destroy()


@pytest.mark.parametrize("nx,ny,n,nrhs", [(9, 6, 24, 3), (65, 17, 8, 2), (4, 4, 192, 4), (3, 3, 300, 2),
                                          (7, 5, 96, 8), (2, 2, 512, 1),
                                          # 16 right-hand sides per pass (two B tiles), and 8 beyond 5 u tiles
                                          (5, 4, 288, 16), (4, 3, 192, 12), (3, 4, 40, 9), (6, 5, 288, 21),
                                          (2, 3, 336, 16)])
def test_recip_apply_T_fp32(nx, ny, n, nrhs):
    e = E()
    plan, B, w, S, tm = recip_plan(nx, ny, n, nrhs, seed=3 + n)
    x = W.random_vectors(nrhs, nx, ny, n, seed=9)
    y = apply(e, plan, e.EMSURF_FP32, x)
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    err = rel_per_rhs(y, yr)
    say(f"reciprocal apply_T fp32 {nx}x{ny} n={n} nrhs={nrhs}: rel err per rhs {err}")
    assert np.all(err <= FP32_TOL)


@pytest.mark.parametrize("prec,n,nrhs", [("fp32", 288, 16), ("fp32", 192, 11), ("fp32", 40, 9), ("fp64", 192, 8),
                                         ("fp64", 40, 13)])
def test_recip_columns_bitwise_alone_and_batched(prec, n, nrhs):
    # every right-hand side gets the same bits alone (a pass of 4) and in a
    # batch of passes of 8 or 16 (one or two B tiles)
    e = E()
    nx, ny = 4, 3
    plan, B, w, S, tm = recip_plan(nx, ny, n, nrhs, seed=n + nrhs)
    p = e.EMSURF_FP32 if prec == "fp32" else e.EMSURF_FP64
    x = W.random_vectors(nrhs, nx, ny, n, seed=31)
    yb = apply(e, plan, p, x)
    for r in range(nrhs):
        ya = apply(e, plan, p, x[r:r + 1])
        assert np.array_equal(ya[0], yb[r]), r
    say(f"reciprocal {prec} n={n}: {nrhs} columns alone == batched")
    plan.destroy()


@pytest.mark.parametrize("signed,zero_self", [(False, True), (True, False)])
def test_recip_matches_full_plan(signed, zero_self):
    # the same blocks in a full plan: FP64 results agree to rounding
    e = E()
    nx, ny, n, nrhs = 7, 6, 20, 3
    plan, B, w, S, tm = recip_plan(nx, ny, n, nrhs, seed=21, signed=signed, zero_self=zero_self)
    full = e.emsurf_plan_create(nx, ny, n, 2, nrhs, B, S, tm)
    x = W.random_vectors(nrhs, nx, ny, n, seed=22)
    y_r = apply(e, plan, e.EMSURF_FP64, x)
    y_f = apply(e, full, e.EMSURF_FP64, x)
    err = rel_per_rhs(y_r, y_f)
    say(f"reciprocal vs full plan (signed weights {signed}, self block {not zero_self}): {err}")
    assert np.all(err <= FP64_TOL)
    # one block per pair, n padded to whole 16 x 16 tiles
    nt = -(-n // 16)
    st = plan.stats()
    assert st.bytes_that64 == st.n_stored * nt * nt * 256 * 16
    assert st.bytes_that32 == st.n_stored * nt * nt * 256 * 8


def test_recip_delta_columns():
    # T e_{m0,v} returns column v of T(m - m0) for every element m, including
    # the columns served by the transposed half of the paired products
    e = E()
    nx, ny, n = 5, 4, 11
    plan, B, w, S, tm = recip_plan(nx, ny, n, 1, seed=13)
    for (iy0, ix0, v) in [(2, 1, 4), (0, 4, 0), (3, 0, 10)]:
        x = np.zeros((1, ny, nx, n), dtype=np.complex128)
        x[0, iy0, ix0, v] = 1.0
        yy = apply(e, plan, e.EMSURF_FP64, x)[0]
        for iy in range(ny):
            for ix in range(nx):
                col = B[iy - iy0 + ny - 1, ix - ix0 + nx - 1][:, v]
                assert np.allclose(yy[iy, ix], col, rtol=0, atol=1e-13)


@pytest.mark.parametrize("npch,nx,ny", [(24, 4, 3), (48, 5, 4), (72, 3, 2)])
def test_recip_green_plan_matches_oracle(npch, nx, ny):
    # the point-sampled fill is reciprocal with the source patch areas as weights
    e = E()
    g = W.box_geometry(npch)
    n = 4 * npch
    S = W.random_types(2, n, seed=4)
    tm = W.random_type_map(nx, ny, 2, seed=4)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 2, 4, geom, S, tm, recip=1)
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    x = W.random_vectors(4, nx, ny, n, seed=5)
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    e64 = rel_per_rhs(apply(e, plan, e.EMSURF_FP64, x), yr)
    e32 = rel_per_rhs(apply(e, plan, e.EMSURF_FP32, x), yr)
    say(f"reciprocal Green plan {nx}x{ny} n={n}: FP64 {e64.max():.2e}, FP32 {e32.max():.2e}")
    assert np.all(e64 <= FP64_TOL) and np.all(e32 <= FP32_TOL)
    plan.destroy()


def test_recip_solve_matches_lu():
    e = E()
    nx, ny, n, nt = 4, 3, 12, 2
    plan, B, w, S, tm = recip_plan(nx, ny, n, 2, seed=31, n_types=nt)
    A = np.eye(nx * ny * n) - MM.dense_S(S, tm) @ C.dense_T(B, nx, ny)
    b = W.random_vectors(2, nx, ny, n, seed=32)
    for prec, tol, bar in [(e.EMSURF_FP64, 1e-11, 1e-9), (e.EMSURF_FP32_IR, 1e-9, 1e-7)]:
        x = torch.zeros_like(dev(b))
        st, info = e.emsurf_solve(plan, e.solve_opts(prec, tol=tol), 2, dev(b), x)
        assert st == e.EMSURF_OK
        xs = x.cpu().numpy()
        for r in range(2):
            xref = K.solve_dense(A, b[r].ravel())
            err = float(np.linalg.norm(xs[r].ravel() - xref) / np.linalg.norm(xref))
            say(f"reciprocal solve prec {prec} rhs {r}: {info[r]['iters']} iterations, error vs LU {err:.2e}")
            assert err <= bar


def test_recip_argument_errors():
    e = E()
    nx, ny, n = 3, 2, 6
    w = W.random_weights(n, 1)
    S = W.random_types(1, n, seed=1)
    tm = np.zeros((ny, nx), np.int32)
    # blocks that are not reciprocal under the weights
    B = W.random_blocks(nx, ny, n, seed=2)
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 1, B, w, S, tm)
    assert ex.value.status == e.EMSURF_ERR_ARG and "not reciprocal" in str(ex.value)
    # reciprocal blocks checked against other weights
    Br = W.random_reciprocal_blocks(nx, ny, n, w, seed=3)
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 1, Br, None, S, tm)
    assert ex.value.status == e.EMSURF_ERR_ARG
    # a zero weight
    w0 = w.copy()
    w0[2] = 0.0
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 1, Br, w0, S, tm)
    assert ex.value.status == e.EMSURF_ERR_ARG
    # the entry point needs desc.recip = 1
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 1, Br, w, S, tm, recip=0)
    assert ex.value.status == e.EMSURF_ERR_ARG
    # a reciprocal plan has only the paired kernel: MFMA variants are refused and
    # the autotuner times variant 0 alone
    Bq = W.random_reciprocal_blocks(4, 4, 64, np.ones(64), seed=6)
    pq = e.emsurf_plan_create(4, 4, 64, 1, 16, Bq, W.random_types(1, 64, seed=6), np.zeros((4, 4), np.int32),
                              recip=1)
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_set_variant(pq, 16, 3)
    assert ex.value.status == e.EMSURF_ERR_UNSUPPORTED
    best, ms = e.emsurf_plan_autotune(pq, 16)
    times = list(ms.values())
    assert best == 0 and times[0] > 0 and all(m is None for m in times[1:])
    pq.destroy()
    # unit weights: symmetric blocks are accepted through emsurf_plan_create too
    Bs = W.random_reciprocal_blocks(nx, ny, n, np.ones(n), seed=4)
    plan = e.emsurf_plan_create(nx, ny, n, 1, 1, Bs, S, tm, recip=1)
    x = W.random_vectors(1, nx, ny, n, seed=5)
    yr = C.apply_T_direct(lambda dy, dx: Bs[dy + ny - 1, dx + nx - 1], x)
    assert rel_per_rhs(apply(e, plan, e.EMSURF_FP64, x), yr).max() <= FP64_TOL
    plan.destroy()


def test_recip_fullsize_128x128_sampled():
    # the 128 x 128 workload (n_eq 192, 4 RHS) as a reciprocal plan, the
    # configuration bench.py times; sampled rows against the oracle's
    # on-the-fly row evaluation
    e = E()
    c = W.config(4)
    g = W.box_geometry(c.n_patch)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(c.nx, c.ny, c.n_types, c.nrhs, geom, W.s_types(c), W.type_map(c), recip=1)
    st = plan.stats()
    say(f"reciprocal 128x128: {st.n_stored} of {st.n_freq} blocks, FP32 store {st.bytes_that32 / 2**30:.2f} GiB")
    # n_eq 192 fills whole tiles: the paired stores are half the full ones plus the self-paired blocks
    assert st.bytes_that32 == st.n_stored * 192 * 192 * 8 and st.bytes_that64 == st.n_stored * 192 * 192 * 16
    b = W.plane_wave_rhs(c, g)
    b64 = torch.from_numpy(b).to("cuda")
    y64 = torch.empty_like(b64)
    e.emsurf_apply_T(plan, e.EMSURF_FP64, c.nrhs, b64, y64)
    x32 = b64.to(torch.complex64)
    y32 = torch.empty_like(x32)
    e.emsurf_apply_T(plan, e.EMSURF_FP32, c.nrhs, x32, y32)
    torch.cuda.synchronize()
    elems = [(0, 127), (42, 64), (127, 0)]
    ref = C.apply_T_elements(g.rho, g.area, g.tan, W.PITCH, W.K0, b, elems, chunk_rows=8)
    got64 = y64.cpu().numpy()
    got32 = y32.cpu().numpy().astype(np.complex128)
    for i, (iy, ix) in enumerate(elems):
        e64 = float(np.linalg.norm(got64[:, iy, ix] - ref[i]) / np.linalg.norm(ref[i]))
        e32 = float(np.linalg.norm(got32[:, iy, ix] - ref[i]) / np.linalg.norm(ref[i]))
        say(f"  element ({iy},{ix}): FP64 {e64:.2e}, FP32 {e32:.2e}")
        assert e64 <= FP64_TOL and e32 <= 2e-5
    plan.destroy()
