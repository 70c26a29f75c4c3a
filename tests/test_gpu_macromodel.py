"""GPU parity of macromodel generation (Schur complement of the interior
unknowns and S = -(Z~ + Z_self)^-1, emsurf_macromodels) against the FP64
oracle, through the C ABI: ragged sizes around the 32-column panels, no
interior unknowns, a missing self block, a singular interior block, the
64 x 64 workload's 32 cell types, and a solve on a plan built from the
generated macromodels.  Bar: FP64 1e-12 relative per cell type."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
from oracle import krylov as K
from oracle import macromodel as MM
from oracle import macromodel_gen as MG

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def E():
    import paper_1911_04576_amd as mod
    mod.lib()
    return mod


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(msg):
    print(msg, flush=True)


def run(e, Z, n, Zself):
    T, N, _ = Z.shape
    S = torch.empty((T, n, n), dtype=torch.complex128, device="cuda")
    Zt = torch.empty_like(S)
    e.emsurf_macromodels(T, n, N - n, dev(Z), None if Zself is None else dev(Zself), S, Zt)
    torch.cuda.synchronize()
    return S.cpu().numpy(), Zt.cpu().numpy()


def rel_types(a, b):
    return max(float(np.linalg.norm(a[t] - b[t]) / np.linalg.norm(b[t])) for t in range(b.shape[0]))


# (the last two: more than 1024 rows below the first panels, which then take
# the global-memory panel in one-panel blocks before the register panels and
# two-panel blocks take over)
@pytest.mark.parametrize("T,n,m", [(1, 1, 0), (1, 1, 1), (1, 3, 5), (2, 7, 33), (3, 33, 70), (2, 40, 0),
                                   (4, 96, 192), (5, 50, 129), (2, 64, 31), (1, 64, 1000), (2, 100, 1100)])
def test_macromodels_match_oracle(T, n, m):
    e = E()
    say(f"macromodels: {T} types, n_eq {n}, n_int {m}")
    Z, Zself = W.cell_interiors(T, n, m, seed=T * 100 + n + m)
    S, Zt = run(e, Z, n, Zself)
    Zt_ref, S_ref = MG.macromodels(Z, n, Zself)
    ez, es = rel_types(Zt, Zt_ref), rel_types(S, S_ref)
    say(f"  Z~ {ez:.2e}  S {es:.2e}")
    assert ez <= FP64_TOL and es <= FP64_TOL


def test_missing_self_block_is_zero():
    e = E()
    Z, _ = W.cell_interiors(2, 20, 30, seed=5)
    S, Zt = run(e, Z, 20, None)
    Zt_ref, S_ref = MG.macromodels(Z, 20, np.zeros((20, 20), complex))
    assert rel_types(S, S_ref) <= FP64_TOL and rel_types(Zt, Zt_ref) <= FP64_TOL


def test_singular_interior_is_reported():
    e = E()
    Z, Zself = W.cell_interiors(3, 8, 12, seed=6)
    Z[1, 8:, 8 + 5] = 0.0                      # type 1: a zero column in Z_int,int
    with pytest.raises(e.EmsurfError) as ex:
        run(e, Z, 8, Zself)
    assert ex.value.status == e.EMSURF_ERR_ARG and "cell type 1" in str(ex.value)


def test_workload_64x64_types_and_solve():
    # the 64 x 64 workload's shape: 32 types, n_eq 288, twice as many interior unknowns
    e = E()
    T, n, m = 32, 288, 576
    Z, Zself = W.cell_interiors(T, n, m, seed=11)
    S, Zt = run(e, Z, n, Zself)
    Zt_ref, S_ref = MG.macromodels(Z, n, Zself)
    es = rel_types(S, S_ref)
    say(f"32 x (288 + 576): S {es:.2e}, Z~ {rel_types(Zt, Zt_ref):.2e}")
    assert es <= FP64_TOL
    # a plan on a small lattice built from generated macromodels solves the coupled system
    g = W.box_geometry(72)
    nx, ny = 3, 2
    tm = W.random_type_map(nx, ny, T, seed=3)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, T, 1, geom, S, tm)
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    A = np.eye(nx * ny * n) - MM.dense_S(S_ref, tm) @ C.dense_T(B, nx, ny)
    b = W.random_vectors(1, nx, ny, n, seed=4)
    x = torch.zeros_like(dev(b))
    st, info = e.emsurf_solve(plan, e.solve_opts(e.EMSURF_FP64, tol=1e-11), 1, dev(b), x)
    assert st == e.EMSURF_OK
    xref = K.solve_dense(A, b.ravel())
    err = float(np.linalg.norm(x.cpu().numpy().ravel() - xref) / np.linalg.norm(xref))
    say(f"  solve with generated S: {info[0]['iters']} iterations, error vs LU {err:.2e}")
    assert err <= 1e-9
    plan.destroy()
