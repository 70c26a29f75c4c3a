"""GPU parity of the split-bfloat16 applies (EMSURF_BF16X3, EMSURF_BF16)
through the C ABI.

Bars, derived from the split definition (oracle/split_bf16.py):
* 1 x 1 lattice (padded lengths at most 2: every spectral value of x is x
  itself and the inverse transform averages equal values, all exact in FP32,
  so the apply is the block product alone): against the split model combined
  in FP64, 1e-6 relative per right-hand side -- FP32 accumulation only.  The
  model itself sits 3e-6 or more from the exact product (three products) and
  about 2^-9 (one product), so the bar resolves how the split is formed.
* Lattices against the FP64 oracle: three products 1e-4, one product 1e-2
  per right-hand side.  The split leaves each real product within 3 * 2^-16
  |a||b| (one product: 2^-7 |a||b|); with rounding errors of random sign the
  normwise error is about sqrt(2) 2^-17 / sqrt(3) ~ 6e-6 (one product
  ~ 1.6e-3), and the bars allow a factor of about 15 (6) over that.
* The one-product error must exceed the three-product error twenty-fold,
  which shows the lo terms in use."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import macromodel as MM
from oracle import split_bf16 as SB

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL3 = 1e-4
TOL1 = 1e-2


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(msg):
    print(msg, flush=True)


def rel(y, yr):
    y = np.asarray(y).reshape(yr.shape[0], -1)
    yr = yr.reshape(yr.shape[0], -1)
    return np.linalg.norm(y - yr, axis=1) / np.linalg.norm(yr, axis=1)


def apply(e, plan, prec, x, op="T"):
    xd = dev(x.astype(np.complex64))
    y = torch.empty_like(xd)
    fn = {"T": e.emsurf_apply_T, "A": e.emsurf_apply_A, "S": e.emsurf_apply_S}[op]
    fn(plan, prec, x.shape[0], xd, y)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("n,nrhs", [(32, 1), (96, 5), (288, 17), (480, 33)])
def test_single_element_matches_split_model(n, nrhs):
    e = E()
    say(f"bf16 1x1 n={n} nrhs={nrhs}")
    B = W.random_blocks(1, 1, n, seed=n, zero_self=False)
    S = W.random_types(1, n, seed=1)
    tm = np.zeros((1, 1), dtype=np.int32)
    plan = e.emsurf_plan_create(1, 1, n, 1, nrhs, B, S, tm, store=e.EMSURF_STORE_FP32 | e.EMSURF_STORE_BF16)
    st = plan.stats()
    assert st.Lx <= 2 and st.Ly <= 2
    x = W.random_vectors(nrhs, 1, 1, n, seed=n + 1)
    X = x.reshape(nrhs, n).T
    exact = (B[0, 0] @ X).T.reshape(x.shape)
    for prec, terms in ((e.EMSURF_BF16X3, 3), (e.EMSURF_BF16, 1)):
        want = SB.split_product(B[0, 0], X, terms).T.reshape(x.shape)
        got = apply(e, plan, prec, x)
        err = rel(got, want)
        gap = rel(want, exact)
        say(f"  terms {terms}: rel err vs split model {err.max():.2e} (model vs exact product {gap.min():.2e})")
        assert err.max() <= 1e-6
        # the bar resolves the split: the model is further from the exact product
        assert gap.min() > 2e-6
    plan.destroy()


@pytest.mark.parametrize("nx,ny,n,nrhs", [(4, 4, 96, 16), (5, 3, 64, 4), (3, 5, 32, 33), (2, 2, 160, 1),
                                           (6, 2, 224, 20), (3, 4, 288, 16)])
def test_lattice_against_oracle(nx, ny, n, nrhs):
    e = E()
    say(f"bf16 {nx}x{ny} n={n} nrhs={nrhs}")
    B = W.random_blocks(nx, ny, n, seed=n + nrhs)
    S = W.random_types(2, n, seed=2)
    tm = W.random_type_map(nx, ny, 2, seed=2)
    plan = e.emsurf_plan_create(nx, ny, n, 2, nrhs, B, S, tm,
                                store=e.EMSURF_STORE_FP32 | e.EMSURF_STORE_BF16)
    x = W.random_vectors(nrhs, nx, ny, n, seed=7)
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    e3 = rel(apply(e, plan, e.EMSURF_BF16X3, x), yr)
    e1 = rel(apply(e, plan, e.EMSURF_BF16, x), yr)
    e32 = rel(apply(e, plan, e.EMSURF_FP32, x), yr)
    say(f"  rel err vs oracle: bf16x3 {e3.max():.2e}, bf16 {e1.max():.2e}, fp32 {e32.max():.2e}")
    assert e3.max() <= TOL3 and e1.max() <= TOL1
    assert e1.min() > 20 * e3.max()
    plan.destroy()


def test_columns_are_independent():
    # an output column depends only on its own right-hand side: the first of
    # 16 equals the single-RHS result bit for bit
    e = E()
    nx, ny, n, nrhs = 3, 3, 96, 16
    B = W.random_blocks(nx, ny, n, seed=5)
    plan = e.emsurf_plan_create(nx, ny, n, 1, nrhs, B, W.random_types(1, n, seed=5),
                                np.zeros((ny, nx), dtype=np.int32), store=e.EMSURF_STORE_BF16)
    x = W.random_vectors(nrhs, nx, ny, n, seed=8)
    for prec in (e.EMSURF_BF16X3, e.EMSURF_BF16):
        y1 = apply(e, plan, prec, x[:1])
        y16 = apply(e, plan, prec, x)
        assert np.array_equal(y1[0], y16[0])
    plan.destroy()


def test_apply_A_and_S():
    e = E()
    nx, ny, n, nrhs = 4, 3, 64, 3
    B = W.random_blocks(nx, ny, n, seed=11)
    S = W.random_types(3, n, seed=11)
    tm = W.random_type_map(nx, ny, 3, seed=11)
    plan = e.emsurf_plan_create(nx, ny, n, 3, nrhs, B, S, tm, store=e.EMSURF_STORE_FP32 | e.EMSURF_STORE_BF16)
    x = W.random_vectors(nrhs, nx, ny, n, seed=12)
    Tf = lambda v: C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], v)
    ref = MM.apply_A(Tf, S, tm, x)
    ea = rel(apply(e, plan, e.EMSURF_BF16X3, x, "A"), ref)
    say(f"bf16x3 apply_A rel err {ea.max():.2e}")
    assert ea.max() <= TOL3
    # S is applied in FP32 for the split precisions
    assert np.array_equal(apply(e, plan, e.EMSURF_BF16X3, x, "S"), apply(e, plan, e.EMSURF_FP32, x, "S"))
    plan.destroy()


@pytest.mark.parametrize("prec", [3, 4])
def test_graph_replay_matches_eager(prec):
    e = E()
    nx, ny, n, nrhs = 5, 4, 96, 4
    B = W.random_blocks(nx, ny, n, seed=21)
    S = W.random_types(2, n, seed=21)
    tm = W.random_type_map(nx, ny, 2, seed=21)
    plan = e.emsurf_plan_create(nx, ny, n, 2, nrhs, B, S, tm, store=e.EMSURF_STORE_BF16)
    s = torch.cuda.Stream()
    xg = torch.empty((nrhs, ny, nx, n), dtype=torch.complex64, device="cuda")
    yg = torch.empty_like(xg)
    g = e.emsurf_graph_create(plan, e.EMSURF_OP_T, prec, nrhs, xg, yg, s)
    for rep in range(3):
        x = W.random_vectors(nrhs, nx, ny, n, seed=200 + rep)
        with torch.cuda.stream(s):
            xg.copy_(dev(x).to(torch.complex64))
        g.launch(s)
        s.synchronize()
        ye = torch.empty_like(xg)
        e.emsurf_apply_T(plan, prec, nrhs, xg, ye)
        torch.cuda.synchronize()
        assert np.array_equal(yg.cpu().numpy(), ye.cpu().numpy())
    g.destroy()
    plan.destroy()


def test_store_sizes_and_argument_errors():
    e = E()
    nx, ny, n = 3, 2, 64
    B = W.random_blocks(nx, ny, n, seed=31)
    S = W.random_types(1, n, seed=31)
    tm = np.zeros((ny, nx), dtype=np.int32)
    plan = e.emsurf_plan_create(nx, ny, n, 1, 2, B, S, tm, store=e.EMSURF_STORE_BF16)
    st = plan.stats()
    assert st.bytes_that16 == st.n_freq * n * n * 8 and st.bytes_that32 == 0 and st.bytes_that64 == 0
    assert e.emsurf_plan_bytes(nx, ny, n, 1, 2, store=e.EMSURF_STORE_BF16) >= st.bytes_that16
    x = dev(W.random_vectors(2, nx, ny, n, seed=1).astype(np.complex64))
    y = torch.empty_like(x)
    for prec, status in ((e.EMSURF_FP32, e.EMSURF_ERR_UNSUPPORTED), (e.EMSURF_FP32_IR, e.EMSURF_ERR_ARG), (5, e.EMSURF_ERR_ARG)):
        with pytest.raises(e.EmsurfError) as ex:
            e.emsurf_apply_T(plan, prec, 2, x, y)
        assert ex.value.status == status
    e.emsurf_apply_T(plan, e.EMSURF_BF16X3, 2, x, y)
    torch.cuda.synchronize()
    b = torch.zeros((1, ny, nx, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_solve(plan, e.solve_opts(prec=e.EMSURF_BF16X3), 1, b, torch.empty_like(b))
    assert ex.value.status == e.EMSURF_ERR_ARG
    plan.destroy()
    # no split store: the split precisions are unsupported
    p32 = e.emsurf_plan_create(nx, ny, n, 1, 2, B, S, tm, store=e.EMSURF_STORE_FP32)
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_apply_T(p32, e.EMSURF_BF16, 2, x, y)
    assert ex.value.status == e.EMSURF_ERR_UNSUPPORTED
    p32.destroy()
    # the split store needs a dense full plan with n_eq a multiple of 32
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create(nx, ny, 48, 1, 2, W.random_blocks(nx, ny, 48, seed=1), W.random_types(1, 48, seed=1),
                             tm, store=e.EMSURF_STORE_BF16)
    assert ex.value.status == e.EMSURF_ERR_ARG
    w = W.random_weights(n, 3)
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create_reciprocal(nx, ny, n, 1, 2, W.random_reciprocal_blocks(nx, ny, n, w, 3), w, S, tm,
                                        store=e.EMSURF_STORE_BF16)
    assert ex.value.status == e.EMSURF_ERR_ARG
    LKb = np.zeros((2 * ny - 1, 2 * nx - 1, 2, n // 2, n // 2), dtype=np.complex128)
    with pytest.raises(e.EmsurfError) as ex:
        e.emsurf_plan_create(nx, ny, n, 1, 2, LKb, S, tm, store=e.EMSURF_STORE_BF16, form=e.EMSURF_T_LK,
                             coef=(-1j, 1, -1, 1j))
    assert ex.value.status == e.EMSURF_ERR_ARG


def test_fullsize_64x64_sampled():
    # the 64 x 64 many-RHS workload (72 patches per box, n_eq 288, 16 RHS) with
    # the Green fill; sampled elements against the oracle's row evaluation
    e = E()
    c = W.config(3)
    g = W.box_geometry(c.n_patch)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(c.nx, c.ny, c.n_types, c.nrhs, geom, W.s_types(c), W.type_map(c),
                                      store=e.EMSURF_STORE_BF16)
    st = plan.stats()
    say(f"bf16 64x64: split store {st.bytes_that16 / 2**30:.2f} GiB")
    b = W.plane_wave_rhs(c, g)
    elems = [(0, 63), (21, 40), (63, 0)]
    ref = C.apply_T_elements(g.rho, g.area, g.tan, W.PITCH, W.K0, b, elems, chunk_rows=8)
    for prec, tol in ((e.EMSURF_BF16X3, TOL3), (e.EMSURF_BF16, TOL1)):
        got = apply(e, plan, prec, b)
        for i, (iy, ix) in enumerate(elems):
            err = float(np.linalg.norm(got[:, iy, ix] - ref[i]) / np.linalg.norm(ref[i]))
            say(f"  prec {prec} element ({iy},{ix}): rel err {err:.2e}")
            assert err <= tol
    plan.destroy()
