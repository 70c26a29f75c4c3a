"""Continuous batching: sessions (iteration-level joining) and the multi-surface
server (plan residency, admission by memory, LRU eviction), through the C ABI.
The key property: a right-hand side's result is bitwise the same alone and in
a mix, and every result meets the tolerance with the oracle's FP64 operator."""
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


def surface(nx, ny, npch, n_types, seed):
    g = W.box_geometry(npch)
    S = W.random_types(n_types, g.n_eq, seed=seed)
    tm = W.random_type_map(nx, ny, n_types, seed=seed)
    return g, S, tm


def dense_A(g, S, tm, nx, ny):
    B = C.coupling_blocks(g.rho, g.area, g.tan, nx, ny, W.PITCH, W.K0)
    return np.eye(nx * ny * g.n_eq) - MM.dense_S(S, tm) @ C.dense_T(B, nx, ny)


def rhs_set(nx, ny, npch, count, seed):
    rng = np.random.default_rng(seed)
    ang = tuple((float(rng.uniform(0, 1.0)), "TE" if i % 2 == 0 else "TM") for i in range(count))
    cfg = W.Config(2000 + seed, nx, ny, npch, 1, ang, 1e-8)
    return W.plane_wave_rhs(cfg)


def run_session(e, sess, plan_shape, schedule, max_steps=500):
    """schedule: {step: [(tag, b), ...]}; returns {tag: (x, info)}."""
    out = {}
    slot_tag = {}
    for step in range(max_steps):
        for tag, b in schedule.get(step, []):
            slot = e.emsurf_session_submit(sess, dev(b), tag)
            slot_tag[slot] = tag
        if not slot_tag and step > max(schedule):
            break
        e.emsurf_session_step(sess)
        for slot, tag in e.emsurf_session_finished(sess):
            x = torch.empty(plan_shape, dtype=torch.complex128, device="cuda")
            info = e.emsurf_session_collect(sess, slot, x)
            out[tag] = (x.cpu().numpy(), info)
            del slot_tag[slot]
    assert not slot_tag, "session did not finish"
    return out


@pytest.mark.parametrize("recip", [0, 1])
@pytest.mark.parametrize("prec", [0, 2])
def test_session_alone_equals_mix(prec, recip):
    # recip = 1: the paired block product on the reciprocal store, the store
    # the serving benchmark uses (its column sums have a fixed rounding order)
    e = E()
    nx, ny, npch = 5, 4, 24
    g, S, tm = surface(nx, ny, npch, 3, seed=1)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 3, 6, geom, S, tm, recip=recip)
    bs = rhs_set(nx, ny, npch, 5, seed=2)
    bs[3] *= 1e3
    opts = e.solve_opts(prec, tol=1e-8 if prec == 0 else 1e-6, restart=4)
    shape = (ny, nx, g.n_eq)
    sess = e.emsurf_session_create(plan, 6, opts)
    alone = run_session(e, sess, shape, {0: [(0, bs[0])]})
    # the same right-hand side joining a busy session two iterations in
    mix = run_session(e, sess, shape, {0: [(1, bs[1]), (2, bs[2])], 2: [(0, bs[0]), (3, bs[3])], 3: [(4, bs[4])]})
    xa, ia = alone[0]
    xm, im = mix[0]
    say(f"prec {prec} recip {recip}: alone iters {ia['iters']} cycles {ia['outer_iters']}; mix iters {im['iters']}")
    assert ia["iters"] == im["iters"] and ia["converged"]
    assert np.array_equal(xa, xm)
    A = dense_A(g, S, tm, nx, ny)
    tol = opts.tol
    for tag in range(5):
        x, info = mix[tag]
        res = np.linalg.norm(A @ x.ravel() - bs[tag].ravel()) / np.linalg.norm(bs[tag])
        say(f"  tag {tag}: iters {info['iters']} cycles {info['outer_iters']} oracle residual {res:.2e}")
        assert info["converged"] and res <= tol
    sess.destroy()


def test_session_fp64_matches_solve():
    e = E()
    nx, ny, npch = 6, 3, 48
    g, S, tm = surface(nx, ny, npch, 2, seed=3)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 2, 2, geom, S, tm)
    b = rhs_set(nx, ny, npch, 1, seed=4)
    opts = e.solve_opts(0, tol=1e-10, restart=3)
    xs = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    st, info = e.emsurf_solve(plan, opts, 1, dev(b), xs)
    sess = e.emsurf_session_create(plan, 2, opts)
    out = run_session(e, sess, b.shape[1:], {0: [(7, b[0])]})
    x, si = out[7]
    assert si["iters"] == info[0]["iters"]
    assert np.linalg.norm(x - xs.cpu().numpy()[0]) <= 1e-13 * np.linalg.norm(x)


def test_session_busy_zero_and_nonfinite():
    e = E()
    nx, ny, npch = 3, 3, 24
    g, S, tm = surface(nx, ny, npch, 2, seed=5)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 2, 2, geom, S, tm)
    sess = e.emsurf_session_create(plan, 2, e.solve_opts(0, tol=1e-8))
    z = np.zeros((ny, nx, g.n_eq), complex)
    bad = rhs_set(nx, ny, npch, 1, seed=6)[0]
    bad[0, 0, 0] = np.inf
    s0 = e.emsurf_session_submit(sess, dev(z), 10)
    s1 = e.emsurf_session_submit(sess, dev(bad), 11)
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_session_submit(sess, dev(z), 12)
    assert ei.value.status == e.EMSURF_ERR_BUSY
    e.emsurf_session_step(sess)
    fin = dict((t, s) for s, t in e.emsurf_session_finished(sess))
    assert set(fin) == {10, 11}
    x = torch.empty(z.shape, dtype=torch.complex128, device="cuda")
    info = e.emsurf_session_collect(sess, fin[10], x)
    assert info["converged"] and info["iters"] == 0 and not torch.any(x != 0)
    with pytest.raises(e.EmsurfError) as ei:
        e.emsurf_session_collect(sess, fin[11], x)
    assert ei.value.status == e.EMSURF_ERR_ARG
    assert e.emsurf_session_active(sess) == 0


def test_server_many_surfaces_with_eviction():
    e = E()
    opts = e.solve_opts(2, tol=1e-6, restart=8)
    shapes = [(4, 4, 24, 2), (6, 3, 48, 3), (3, 5, 24, 2)]
    surf = []
    for i, (nx, ny, npch, nt) in enumerate(shapes):
        g, S, tm = surface(nx, ny, npch, nt, seed=20 + i)
        surf.append((nx, ny, npch, nt, g, S, tm, e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)))
    # the largest surface with all 4 slots busy cannot share the budget with
    # any other resident surface: forces evictions
    probe = e.emsurf_server_create(1 << 40, 4, opts)
    fixed = [e.emsurf_server_entry_bytes(probe, nx, ny, 4 * npch, nt) for nx, ny, npch, nt, *_ in surf]
    slot = [e.emsurf_server_slot_bytes(probe, nx, ny, 4 * npch, nt) for nx, ny, npch, nt, *_ in surf]
    probe.destroy()
    assert min(fixed) > 0 and min(slot) > 0
    # slots hold (restart + 4) unknown vectors each
    assert slot[0] == (8 + 4) * 4 * 4 * 96 * 16
    needs = [f + 4 * s for f, s in zip(fixed, slot)]
    srv = e.emsurf_server_create(max(needs) + min(fixed) - 1, 4, opts)
    reqs = {}
    rng = np.random.default_rng(0)
    for r in range(9):
        k = r % 3
        nx, ny, npch, nt, g, S, tm, geom = surf[k]
        nrhs = int(rng.integers(1, 5))
        b = rhs_set(nx, ny, npch, nrhs, seed=100 + r)
        rid = e.emsurf_server_submit(srv, k, nx, ny, nt, geom, S, tm, b)
        reqs[rid] = (k, b)
    got = {}
    for _ in range(2000):
        e.emsurf_server_step(srv)
        while True:
            c = e.emsurf_server_next_completed(srv)
            if c is None:
                break
            rid, nrhs, nu = c
            x, infos, times = e.emsurf_server_fetch(srv, rid, nrhs, nu)
            got[rid] = (x, infos, times)
        if len(got) == len(reqs):
            break
    stats = e.emsurf_server_query(srv)
    say(f"server stats {stats}")
    assert len(got) == len(reqs)
    assert stats["plans_built"] >= 3 and stats["evictions"] >= 1
    dense = {}
    for rid, (k, b) in reqs.items():
        nx, ny, npch, nt, g, S, tm, geom = surf[k]
        if k not in dense:
            dense[k] = dense_A(g, S, tm, nx, ny)
        x, infos, times = got[rid]
        for r in range(b.shape[0]):
            res = np.linalg.norm(dense[k] @ x[r] - b[r].ravel()) / np.linalg.norm(b[r])
            assert infos[r]["converged"] and res <= 1e-6, (rid, r, res)
    srv.destroy()


@pytest.mark.parametrize("n_rhs_mix", [3, 9])
def test_session_reciprocal_wide_batches_alone_equals_mix(n_rhs_mix):
    """A right-hand side alone (a 4-wide pass of the paired product) and in a
    batch of 9 (8-wide passes over two launches), on a 192-row block (12 row
    tiles: every wavefront adds column sums), FP32 inner with FP64 refinement."""
    e = E()
    nx, ny, npch = 4, 3, 48
    g, S, tm = surface(nx, ny, npch, 2, seed=8)
    geom = e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)
    plan = e.emsurf_plan_create_green(nx, ny, 2, 10, geom, S, tm, recip=1)
    bs = rhs_set(nx, ny, npch, n_rhs_mix, seed=9)
    opts = e.solve_opts(2, tol=1e-7, restart=5)
    shape = (ny, nx, g.n_eq)
    sess = e.emsurf_session_create(plan, 10, opts)
    alone = run_session(e, sess, shape, {0: [(0, bs[0])]})
    mix = run_session(e, sess, shape, {0: [(t, bs[t]) for t in range(1, n_rhs_mix)], 1: [(0, bs[0])]})
    assert np.array_equal(alone[0][0], mix[0][0]) and alone[0][1]["iters"] == mix[0][1]["iters"]
    A = dense_A(g, S, tm, nx, ny)
    for tag in range(n_rhs_mix):
        x, info = mix[tag]
        res = np.linalg.norm(A @ x.ravel() - bs[tag].ravel()) / np.linalg.norm(bs[tag])
        assert info["converged"] and res <= 1e-7, (tag, res)
    sess.destroy()
    plan.destroy()


def test_server_reciprocal_plans_match_sessions_alone():
    """Server on reciprocal plans (the bench's serving configuration): each
    right-hand side's result is bitwise the one it gets solved alone in a
    session of the same plan shape, slots and options, and meets the tolerance
    with the oracle's FP64 operator."""
    e = E()
    opts = e.solve_opts(2, tol=1e-6, restart=8)
    slots = 4
    shapes = [(4, 4, 24, 2), (6, 3, 48, 3)]
    surf = []
    for i, (nx, ny, npch, nt) in enumerate(shapes):
        g, S, tm = surface(nx, ny, npch, nt, seed=40 + i)
        surf.append((nx, ny, npch, nt, g, S, tm, e.Geometry(g.rho, g.area, g.tan, W.PITCH, W.K0)))
    srv = e.emsurf_server_create(1 << 36, slots, opts)
    reqs = {}
    rng = np.random.default_rng(3)
    for r in range(6):
        k = r % 2
        nx, ny, npch, nt, g, S, tm, geom = surf[k]
        nrhs = int(rng.integers(1, 4))
        b = rhs_set(nx, ny, npch, nrhs, seed=300 + r)
        rid = e.emsurf_server_submit(srv, k, nx, ny, nt, geom, S, tm, b, recip=1)
        reqs[rid] = (k, b)
    got = {}
    for _ in range(2000):
        e.emsurf_server_step(srv)
        while True:
            c = e.emsurf_server_next_completed(srv)
            if c is None:
                break
            rid, nrhs, nu = c
            got[rid] = e.emsurf_server_fetch(srv, rid, nrhs, nu)
        if len(got) == len(reqs):
            break
    srv.destroy()
    assert len(got) == len(reqs)
    for k, (nx, ny, npch, nt, g, S, tm, geom) in enumerate(surf):
        plan = e.emsurf_plan_create_green(nx, ny, nt, slots, geom, S, tm, recip=1)
        sess = e.emsurf_session_create(plan, slots, opts)
        A = dense_A(g, S, tm, nx, ny)
        for rid, (kk, b) in reqs.items():
            if kk != k:
                continue
            x, infos, _ = got[rid]
            for r in range(b.shape[0]):
                xa, ia = run_session(e, sess, b.shape[1:], {0: [(r, b[r])]})[r]
                assert np.array_equal(xa.ravel(), x[r]), (rid, r)
                assert ia["iters"] == infos[r]["iters"]
                res = np.linalg.norm(A @ x[r] - b[r].ravel()) / np.linalg.norm(b[r])
                assert infos[r]["converged"] and res <= 1e-6, (rid, r, res)
        sess.destroy()
        plan.destroy()
