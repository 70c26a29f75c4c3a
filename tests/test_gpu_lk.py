"""GPU parity of the structured outer operator (EMSURF_T_LK: the plan stores
the Fourier transforms of L and K only, Sec. IV-C) against the FP64 oracle,
through the C ABI: the device fill, applies on the physical fill and on random
dense L and K blocks with random constants (every pass width and the ragged
and radix-3 padded lengths), solves against dense LU, argument errors, and a
full-size 128 x 128 apply on sampled rows.  Bars: FP64 1e-12, FP32 2e-5."""
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
    must be matched exactly (0, else inf)."""
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


@pytest.mark.parametrize("npch,nx,ny", [(24, 1, 1), (24, 3, 2), (48, 2, 3)])
def test_lk_fill_matches_oracle(npch, nx, ny):
    e = E()
    g = W.box_geometry(npch)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    nh = 2 * npch
    out = torch.zeros((2 * ny - 1, 2 * nx - 1, 2, nh, nh), dtype=torch.complex128, device="cuda")
    e.emsurf_fill_LK_point_green(geom, nx, ny, out)
    torch.cuda.synchronize()
    Lb, Kb = LK.lk_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    got = out.cpu().numpy()
    for part, ref in ((0, Lb), (1, Kb)):
        scale = np.abs(ref).max() if np.any(ref) else 1.0
        assert np.abs(got[:, :, part] - ref).max() <= 1e-13 * scale


@pytest.mark.parametrize("nx,ny,npch,nrhs", [(1, 1, 24, 1), (4, 4, 24, 1), (3, 5, 24, 3), (5, 2, 48, 4),
                                             (10, 3, 24, 2), (2, 13, 24, 5), (6, 6, 48, 9)])
def test_apply_T_lk_physical(nx, ny, npch, nrhs):
    e = E()
    g = W.box_geometry(npch)
    n = 4 * npch
    say(f"LK apply (fill): {nx}x{ny}, n_eq {n}, {nrhs} RHS")
    S = W.random_types(2, n, seed=1)
    tm = W.random_type_map(nx, ny, 2, seed=1)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 2, nrhs, geom, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF)
    st = plan.stats()
    nh = n // 2
    assert st.bytes_that64 == st.Lx * st.Ly * 2 * nh * nh * 16
    x = W.random_vectors(nrhs, nx, ny, n, seed=nx * 7 + ny)
    Lb, Kb = LK.lk_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    blocks = LK.lk_assemble(Lb, Kb, W.OUTER_COEF)
    ref = C.apply_T_direct(lambda dy, dx: blocks[dy + ny - 1, dx + nx - 1], x)
    y64, y32 = apply_both(e, plan, x, nrhs)
    e64, e32 = rel(y64, ref), rel(y32, ref)
    say(f"  FP64 {e64:.2e}  FP32 {e32:.2e}")
    assert e64 <= FP64_TOL and e32 <= FP32_TOL
    plan.destroy()


@pytest.mark.parametrize("nx,ny,nh,nrhs", [(1, 1, 3, 1), (2, 3, 5, 2), (4, 3, 17, 3), (7, 2, 8, 8),
                                           (12, 1, 6, 1), (3, 3, 64, 4), (2, 2, 100, 6), (5, 4, 33, 13)])
def test_apply_T_lk_random_blocks(nx, ny, nh, nrhs):
    e = E()
    n = 2 * nh
    say(f"LK apply (random L, K): {nx}x{ny}, n_h {nh}, {nrhs} RHS")
    Lb = W.random_blocks(nx, ny, nh, seed=11 + nh)
    Kb = W.random_blocks(nx, ny, nh, seed=12 + nh)
    rng = np.random.default_rng(nh)
    coef = tuple(complex(a, b) for a, b in rng.standard_normal((4, 2)))
    S = W.random_types(3, n, seed=2)
    tm = W.random_type_map(nx, ny, 3, seed=2)
    T_in = np.stack([Lb, Kb], axis=2)                       # [2ny-1][2nx-1][2][nh][nh]
    plan = e.emsurf_plan_create(nx, ny, n, 3, nrhs, T_in, S, tm, form=e.EMSURF_T_LK, coef=coef)
    x = W.random_vectors(nrhs, nx, ny, n, seed=5)
    blocks = LK.lk_assemble(Lb, Kb, coef)
    ref = C.apply_T_direct(lambda dy, dx: blocks[dy + ny - 1, dx + nx - 1], x)
    y64, y32 = apply_both(e, plan, x, nrhs)
    e64, e32 = rel(y64, ref), rel(y32, ref)
    say(f"  FP64 {e64:.2e}  FP32 {e32:.2e}")
    assert e64 <= FP64_TOL and e32 <= FP32_TOL
    # the same plan built from device blocks
    plan2 = e.emsurf_plan_create(nx, ny, n, 3, nrhs, dev(T_in), S, tm, form=e.EMSURF_T_LK, coef=coef)
    y64b, _ = apply_both(e, plan2, x, nrhs)
    assert np.array_equal(y64b, y64)
    plan.destroy()
    plan2.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir"])
def test_solve_lk_matches_lu(prec):
    e = E()
    nx, ny, npch = 4, 3, 24
    g = W.box_geometry(npch)
    n = 4 * npch
    S = W.random_types(3, n, seed=4)
    tm = W.random_type_map(nx, ny, 3, seed=4)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 3, 2, geom, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF)
    Lb, Kb = LK.lk_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    A = np.eye(nx * ny * n) - MM.dense_S(S, tm) @ C.dense_T(LK.lk_assemble(Lb, Kb, W.OUTER_COEF), nx, ny)
    b = W.random_vectors(2, nx, ny, n, seed=9)
    xref = K.solve_dense(A, b.reshape(2, -1).T).T.reshape(b.shape)
    tol = 1e-10 if prec == "fp64" else 1e-6
    p = e.EMSURF_FP64 if prec == "fp64" else e.EMSURF_FP32_IR
    x = torch.zeros_like(dev(b))
    st, info = e.emsurf_solve(plan, e.solve_opts(p, tol=tol), 2, dev(b), x)
    say(f"LK solve {prec}: {info}")
    assert st == e.EMSURF_OK and all(i["converged"] for i in info)
    err = rel(x.cpu().numpy(), xref)
    assert err <= 10 * tol * np.linalg.cond(A)
    plan.destroy()


def test_lk_argument_errors_and_tuning():
    e = E()
    g = W.box_geometry(24)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    S = W.random_types(1, 96, seed=0)
    tm = np.zeros((2, 2), np.int32)
    with pytest.raises(e.EmsurfError):                        # odd n_eq
        e.emsurf_plan_create(2, 2, 7, 1, 1, np.zeros((3, 3, 2, 3, 3), complex), W.random_types(1, 7, seed=0),
                             tm, form=e.EMSURF_T_LK, coef=(1, 0, 0, 1))
    with pytest.raises(e.EmsurfError):                        # non-finite constant
        e.emsurf_plan_create_green(2, 2, 1, 1, geom, S, tm, form=e.EMSURF_T_LK, coef=(np.nan, 1, -1, 1))
    with pytest.raises(e.EmsurfError):                        # unknown form
        e.emsurf_plan_create_green(2, 2, 1, 1, geom, S, tm, form=7)
    # n_eq = 10 is no multiple of 32: only the streaming kernel applies
    Lb = W.random_blocks(2, 2, 5, seed=1)
    plan10 = e.emsurf_plan_create(2, 2, 10, 1, 16, np.stack([Lb, Lb], axis=2), W.random_types(1, 10, seed=1), tm,
                                  form=e.EMSURF_T_LK, coef=(1, 0.5, -0.5, 1))
    with pytest.raises(e.EmsurfError):
        e.emsurf_plan_set_variant(plan10, 16, e.EMSURF_BP_MFMA_T3)
    best, ms = e.emsurf_plan_autotune(plan10, 16)
    assert best == 0 and ms[e.BP_NAMES[0]] is not None
    assert all(v is None for k, v in ms.items() if k != e.BP_NAMES[0])
    plan10.destroy()
    # n_eq = 96: the matrix-core variants are timed too
    plan = e.emsurf_plan_create_green(2, 2, 1, 16, geom, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF)
    e.emsurf_plan_set_variant(plan, 16, e.EMSURF_BP_MFMA_T3)
    best, ms = e.emsurf_plan_autotune(plan, 16)
    assert ms[e.BP_NAMES[e.EMSURF_BP_MFMA_T3]] is not None and ms[e.BP_NAMES[best]] is not None
    dense = e.emsurf_plan_bytes(64, 64, 192, 16, 4)
    lk = e.emsurf_plan_bytes(64, 64, 192, 16, 4, form=e.EMSURF_T_LK)
    assert lk < dense
    plan.destroy()


def test_lk_fullsize_128x128_sampled():
    e = E()
    c = W.config(4)
    g = W.box_geometry(c.n_patch)
    S, tm = W.s_types(c), W.type_map(c)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(c.nx, c.ny, c.n_types, c.nrhs, geom, S, tm, form=e.EMSURF_T_LK,
                                      coef=W.OUTER_COEF)
    say(f"LK full size: {c.nx}x{c.ny}, n_eq {c.n_eq}, {c.nrhs} RHS, store {plan.stats().bytes_that32 / 1e9:.2f} GB FP32")
    b = W.plane_wave_rhs(c, g)
    y64, y32 = apply_both(e, plan, b, c.nrhs)
    elems = [(0, 0), (77, 31)]
    ref = LK.apply_T_elements_lk(g.rho, g.area, g.tan, W.PITCH, W.K0, W.OUTER_COEF, b, elems, chunk_rows=8)
    for i, (iy, ix) in enumerate(elems):
        e64 = float(np.linalg.norm(y64[:, iy, ix] - ref[i]) / np.linalg.norm(ref[i]))
        e32 = float(np.linalg.norm(y32[:, iy, ix] - ref[i]) / np.linalg.norm(ref[i]))
        say(f"  element ({iy},{ix}): FP64 {e64:.2e}, FP32 {e32:.2e}")
        assert e64 <= FP64_TOL and e32 <= FP32_TOL
    plan.destroy()


def test_lk_graph_replay_and_session_alone_equals_mix():
    # the structured plan under the HIP-graph capture of apply_A (replays with
    # eager work between them) and under continuous batching (a right-hand side
    # bitwise the same alone and joining a busy session)
    e = E()
    nx, ny, npch, nt = 4, 3, 24, 2
    g = W.box_geometry(npch)
    n = 4 * npch
    S = W.random_types(nt, n, seed=8)
    tm = W.random_type_map(nx, ny, nt, seed=8)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, nt, 4, geom, S, tm, form=e.EMSURF_T_LK, coef=W.OUTER_COEF)
    Lb, Kb = LK.lk_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    blocks = LK.lk_assemble(Lb, Kb, W.OUTER_COEF)
    Tf = lambda v: C.apply_T_direct(lambda dy, dx: blocks[dy + ny - 1, dx + nx - 1], v)
    s = torch.cuda.Stream()
    xg = torch.empty((1, ny, nx, n), dtype=torch.complex128, device="cuda")
    yg = torch.empty_like(xg)
    gr = e.emsurf_graph_create(plan, e.EMSURF_OP_A, e.EMSURF_FP64, 1, xg, yg, s)
    for rep in range(3):
        x = W.random_vectors(1, nx, ny, n, seed=40 + rep)
        with torch.cuda.stream(s):
            xg.copy_(dev(x))
        gr.launch(s)
        s.synchronize()
        ye = torch.empty_like(xg)
        e.emsurf_apply_A(plan, e.EMSURF_FP64, 1, xg, ye)
        torch.cuda.synchronize()
        assert rel(yg.cpu().numpy(), MM.apply_A(Tf, S, tm, x)) <= FP64_TOL
        assert np.array_equal(yg.cpu().numpy(), ye.cpu().numpy())
    gr.destroy()
    opts = e.solve_opts(e.EMSURF_FP32_IR, tol=1e-6, restart=5)
    bs = W.random_vectors(3, nx, ny, n, seed=12)
    shape = (ny, nx, n)

    def run(schedule):
        sess = e.emsurf_session_create(plan, 4, opts)
        out, slot_tag = {}, {}
        for step in range(400):
            for tag in schedule.get(step, []):
                slot_tag[e.emsurf_session_submit(sess, dev(bs[tag]), tag)] = tag
            if not slot_tag and step > max(schedule):
                break
            e.emsurf_session_step(sess)
            for slot, tag in e.emsurf_session_finished(sess):
                x = torch.empty(shape, dtype=torch.complex128, device="cuda")
                info = e.emsurf_session_collect(sess, slot, x)
                out[tag] = (x.cpu().numpy(), info)
                del slot_tag[slot]
        sess.destroy()
        return out

    alone = run({0: [0]})
    mix = run({0: [1, 2], 2: [0]})
    assert np.array_equal(alone[0][0], mix[0][0]) and alone[0][1]["converged"]
    A = np.eye(nx * ny * n) - MM.dense_S(S, tm) @ C.dense_T(blocks, nx, ny)
    for t in range(3):
        x, info = mix[t]
        res = np.linalg.norm(A @ x.ravel() - bs[t].ravel()) / np.linalg.norm(bs[t])
        assert info["converged"] and res <= 1e-6
    plan.destroy()


@pytest.mark.parametrize("nx,ny,nh,nrhs", [(3, 3, 48, 16), (2, 3, 96, 8), (4, 2, 144, 16), (3, 2, 16, 20),
                                           (2, 2, 48, 33)])
def test_lk_mfma_variants_match_oracle(nx, ny, nh, nrhs):
    e = E()
    n = 2 * nh
    Lb = W.random_blocks(nx, ny, nh, seed=21 + nh)
    Kb = W.random_blocks(nx, ny, nh, seed=22 + nh)
    rng = np.random.default_rng(nrhs)
    coef = tuple(complex(a, b) for a, b in rng.standard_normal((4, 2)))
    S = W.random_types(2, n, seed=3)
    tm = W.random_type_map(nx, ny, 2, seed=3)
    plan = e.emsurf_plan_create(nx, ny, n, 2, nrhs, np.stack([Lb, Kb], axis=2), S, tm, form=e.EMSURF_T_LK,
                                coef=coef)
    x = W.random_vectors(nrhs, nx, ny, n, seed=6)
    blocks = LK.lk_assemble(Lb, Kb, coef)
    ref = C.apply_T_direct(lambda dy, dx: blocks[dy + ny - 1, dx + nx - 1], x)
    x32 = dev(x).to(torch.complex64)
    ran = []
    for v in range(e.EMSURF_BP_NVARIANTS):
        try:
            e.emsurf_plan_set_variant(plan, nrhs, v)
        except e.EmsurfError:
            continue
        y = torch.empty_like(x32)
        e.emsurf_apply_T(plan, e.EMSURF_FP32, nrhs, x32, y)
        torch.cuda.synchronize()
        err = rel(y.cpu().numpy().astype(np.complex128), ref)
        say(f"  {nx}x{ny} n_h {nh} {nrhs} RHS variant {e.BP_NAMES[v]}: {err:.2e}")
        assert err <= FP32_TOL
        ran.append(v)
    assert 0 in ran and any(v > 0 for v in ran)
    plan.destroy()
