"""Touching fictitious surfaces (Sec. III-D) on the GPU through the C ABI,
against the oracle (oracle/overlap.py, oracle/coupling.py): the coupling fill
and apply at pitch = box edge (coincident patches), U_o and U_o^T, and the
reduced operator U_o^T (D + T) U_o, FP64 1e-12."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import overlap as OV

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOX = W.BOX_A
FP64_TOL = 1e-12


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("npch,nx,ny", [(24, 3, 2), (48, 2, 2), (72, 2, 3)])
def test_touching_fill_and_apply_match_oracle(npch, nx, ny):
    e = E()
    g = W.box_geometry(npch)
    geom = e.Geometry(g.rho, g.area, g.tan, BOX, W.K0)
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, BOX, W.K0)
    assert np.all(np.isfinite(B))
    Tb = torch.empty(B.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_fill_T_point_green(geom, nx, ny, Tb)
    torch.cuda.synchronize()
    assert rel(Tb.cpu().numpy(), B) <= 1e-14
    S = W.random_types(2, g.n_eq, seed=npch)
    tm = W.random_type_map(nx, ny, 2, seed=npch)
    x = W.random_vectors(2, nx, ny, g.n_eq, seed=5)
    for recip in (0, 1):
        plan = e.emsurf_plan_create_green(nx, ny, 2, 2, geom, S, tm, recip=recip)
        y = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
        e.emsurf_apply_T(plan, e.EMSURF_FP64, 2, dev(x), y)
        torch.cuda.synchronize()
        err = rel(y.cpu().numpy(), C.apply_T_dense(B, x))
        say(f"touching {nx}x{ny} npch {npch} recip {recip}: apply_T rel err {err:.2e}")
        assert err <= FP64_TOL
        plan.destroy()


def test_structured_fill_refuses_touching_boxes():
    e = E()
    g = W.box_geometry(24)
    geom = e.Geometry(g.rho, g.area, g.tan, BOX, W.K0)
    S = W.random_types(1, g.n_eq, seed=1)
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_plan_create_green(2, 2, 1, 1, geom, S, np.zeros((2, 2), np.int32), form=e.EMSURF_T_LK,
                                   coef=W.OUTER_COEF)
    assert ei.value.status == e.EMSURF_ERR_ARG


@pytest.mark.parametrize("npch,nx,ny,ground", [(24, 3, 2, 0), (24, 3, 2, 1), (48, 2, 3, 1), (72, 4, 2, 0)])
def test_incidence_and_reduced_operator_match_oracle(npch, nx, ny, ground):
    e = E()
    g = W.box_geometry(npch)
    geom = e.Geometry(g.rho, g.area, g.tan, BOX, W.K0)
    S = W.random_types(3, g.n_eq, seed=nx + ny)
    tm = W.random_type_map(nx, ny, 3, seed=nx * ny)
    nrhs = 2
    plan = e.emsurf_plan_create_green(nx, ny, 3, nrhs, geom, S, tm, recip=1)
    ov = e.emsurf_overlap_create(plan, geom, ground)
    sz = ov.sizes()
    U = OV.incidence(g.rho, g.tan, nx, ny, BOX, ground_plane=bool(ground))
    say(f"overlap {nx}x{ny} npch {npch} ground {ground}: {sz}, oracle U {U.shape}")
    assert (sz["n_full"], sz["n_unique"]) == U.shape
    rng = np.random.default_rng(7)
    xt = rng.standard_normal((nrhs, U.shape[1])) + 1j * rng.standard_normal((nrhs, U.shape[1]))
    x = torch.empty((nrhs, U.shape[0]), dtype=torch.complex128, device="cuda")
    e.emsurf_overlap_expand(ov, nrhs, dev(xt), x)
    y = rng.standard_normal((nrhs, U.shape[0])) + 1j * rng.standard_normal((nrhs, U.shape[0]))
    yt = torch.empty((nrhs, U.shape[1]), dtype=torch.complex128, device="cuda")
    e.emsurf_overlap_reduce(ov, nrhs, dev(y), yt)
    torch.cuda.synchronize()
    assert rel(x.cpu().numpy(), xt @ U.T) <= 1e-15
    assert rel(yt.cpu().numpy(), y @ U) <= 1e-15
    # reduced operator against the dense oracle
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, BOX, W.K0)
    At = OV.reduced_operator(U, OV.dense_D(S, tm), C.dense_T(B, nx, ny))
    zt = torch.empty_like(yt)
    e.emsurf_apply_reduced(ov, nrhs, dev(xt), zt)
    torch.cuda.synchronize()
    ref = xt @ At.T
    err = np.linalg.norm(zt.cpu().numpy() - ref, axis=1) / np.linalg.norm(ref, axis=1)
    say(f"  reduced operator rel err per rhs {err}")
    assert np.all(err <= FP64_TOL)
    ov.destroy()
    plan.destroy()


def test_overlap_on_separated_boxes_is_the_identity():
    e = E()
    g = W.box_geometry(24)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    S = W.random_types(2, g.n_eq, seed=2)
    tm = W.random_type_map(3, 3, 2, seed=2)
    plan = e.emsurf_plan_create_green(3, 3, 2, 1, geom, S, tm)
    ov = e.emsurf_overlap_create(plan, geom, 0)
    sz = ov.sizes()
    assert sz["n_full"] == sz["n_unique"] == 9 * g.n_eq
    x = W.random_vectors(1, 3, 3, g.n_eq, seed=3)
    out = torch.empty(x.shape, dtype=torch.complex128, device="cuda")
    e.emsurf_overlap_expand(ov, 1, dev(x), out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), x)
    ov.destroy()
    plan.destroy()
