"""Multi-RHS Fourier-domain products (MFMA variants), autotuning and HIP-graph
replay, checked against the FP64 oracle through the C ABI."""
import numpy as np
import pytest

import workload as W
from oracle import coupling as C
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


def rel(y, yr):
    y = np.asarray(y).reshape(yr.shape[0], -1)
    yr = yr.reshape(yr.shape[0], -1)
    return np.linalg.norm(y - yr, axis=1) / np.linalg.norm(yr, axis=1)


def random_plan(nx, ny, n, max_rhs, seed, n_types=3):
    e = E()
    B = W.random_blocks(nx, ny, n, seed=seed)
    S = W.random_types(n_types, n, seed=seed)
    tm = W.random_type_map(nx, ny, n_types, seed=seed)
    return e.emsurf_plan_create(nx, ny, n, n_types, max_rhs, B, S, tm), B, S, tm


@pytest.mark.parametrize("nx,ny,n,nrhs", [(5, 4, 96, 16), (3, 3, 192, 8), (4, 3, 288, 16), (6, 2, 64, 20),
                                           (3, 5, 32, 33), (2, 2, 96, 3), (7, 3, 160, 1)])
def test_fp32_variants_match_oracle(nx, ny, n, nrhs):
    e = E()
    say(f"variants {nx}x{ny} n={n} nrhs={nrhs}")
    plan, B, S, tm = random_plan(nx, ny, n, nrhs, seed=n + nrhs)
    x = W.random_vectors(nrhs, nx, ny, n, seed=3)
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    xd = dev(x.astype(np.complex64))
    outs = {}
    for v in range(e.EMSURF_BP_NVARIANTS):
        tpw = v if v <= 4 else v - 4
        waves = -(-(n // 32) // tpw) if v > 0 else 1
        if v > 0 and waves > 4:
            with pytest.raises(e.EmsurfError):
                e.emsurf_plan_set_variant(plan, nrhs, v)
            continue
        e.emsurf_plan_set_variant(plan, nrhs, v)
        y = torch.empty_like(xd)
        e.emsurf_apply_T(plan, e.EMSURF_FP32, nrhs, xd, y)
        torch.cuda.synchronize()
        outs[v] = y.cpu().numpy().astype(np.complex128)
        err = rel(outs[v], yr)
        say(f"  variant {e.BP_NAMES[v]}: max rel err {err.max():.2e}")
        assert err.max() <= 5e-6
    # an MFMA column depends only on its own right-hand side
    if n % 32 == 0:
        e.emsurf_plan_set_variant(plan, nrhs, e.EMSURF_BP_MFMA_T4)
        e.emsurf_plan_set_variant(plan, 1, e.EMSURF_BP_MFMA_T4)
    else:
        e.emsurf_plan_set_variant(plan, nrhs, e.EMSURF_BP_GEMV)
        e.emsurf_plan_set_variant(plan, 1, e.EMSURF_BP_GEMV)
    y1 = torch.empty((1,) + x.shape[1:], dtype=torch.complex64, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP32, 1, dev(x[:1].astype(np.complex64)), y1)
    torch.cuda.synchronize()
    y2 = torch.empty_like(xd)
    e.emsurf_apply_T(plan, e.EMSURF_FP32, nrhs, xd, y2)
    torch.cuda.synchronize()
    assert np.array_equal(y1.cpu().numpy()[0], y2.cpu().numpy()[0])


def test_mfma_rejected_for_ragged_n():
    e = E()
    plan, B, S, tm = random_plan(3, 2, 40, 16, seed=1)
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_plan_set_variant(plan, 16, e.EMSURF_BP_MFMA_T1)
    assert ei.value.status == e.EMSURF_ERR_UNSUPPORTED


def test_autotune_picks_a_valid_variant():
    e = E()
    nx, ny, n, nrhs = 8, 8, 192, 16
    plan, B, S, tm = random_plan(nx, ny, n, nrhs, seed=4)
    best, ms = e.emsurf_plan_autotune(plan, nrhs)
    say(f"autotune {nx}x{ny} n={n} nrhs={nrhs}: best {e.BP_NAMES[best]} {ms}")
    assert 0 <= best < e.EMSURF_BP_NVARIANTS
    assert ms["gemv"] > 0 and ms["mfma_t2"] > 0 and ms["mfma_t1"] is None   # 6 tiles: T1 needs 6 waves
    assert ms["mfma_t1_deep"] is None and ms["mfma_t3_deep"] > 0
    assert ms[e.BP_NAMES[best]] == min(v for v in ms.values() if v is not None)
    x = W.random_vectors(nrhs, nx, ny, n, seed=5)
    y = torch.empty(x.shape, dtype=torch.complex64, device="cuda")
    e.emsurf_apply_T(plan, e.EMSURF_FP32, nrhs, dev(x.astype(np.complex64)), y)
    torch.cuda.synchronize()
    yr = C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], x)
    assert rel(y.cpu().numpy().astype(np.complex128), yr).max() <= 5e-6


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_matches_eager(prec):
    # a captured apply_A replayed several times, with eager work and host
    # synchronisation between replays, must reproduce the eager result each time
    e = E()
    nx, ny, n, nrhs = 6, 5, 48, 2
    plan, B, S, tm = random_plan(nx, ny, n, nrhs, seed=9)
    dt = torch.complex128 if prec == 0 else torch.complex64
    s = torch.cuda.Stream()
    xg = torch.empty((nrhs, ny, nx, n), dtype=dt, device="cuda")
    yg = torch.empty_like(xg)
    g = e.emsurf_graph_create(plan, e.EMSURF_OP_A, prec, nrhs, xg, yg, s)
    Tf = lambda v: C.apply_T_direct(lambda dy, dx: B[dy + ny - 1, dx + nx - 1], v)
    for rep in range(4):
        x = W.random_vectors(nrhs, nx, ny, n, seed=100 + rep)
        with torch.cuda.stream(s):
            xg.copy_(dev(x).to(dt))
        g.launch(s)
        # eager apply on the null stream in between
        ye = torch.empty_like(xg)
        s.synchronize()
        e.emsurf_apply_A(plan, prec, nrhs, xg, ye)
        torch.cuda.synchronize()
        ref = MM.apply_A(Tf, S, tm, x)
        tol = 1e-12 if prec == 0 else 5e-6
        assert rel(yg.cpu().numpy().astype(np.complex128), ref).max() <= tol
        assert np.array_equal(yg.cpu().numpy(), ye.cpu().numpy())
    g.destroy()
