"""Batched solves and the server against solo solves of the same problems and
against the float64 oracle.

A batched launch runs each problem's blocks with that problem's own arguments,
state and reduction scratch, in the same per-problem order as the solo kernels,
so every result must equal the solo reco_solve_cgls result bit for bit.  A
seeded subset of problems (sides 64-256, 2-3 WMG levels, one Tikhonov and one
unpreconditioned problem) is also compared with the oracle's PCGLS at the
iteration count the GPU stopped at, within 3x the oracle's float32 envelope at
each geometry's measured operator error (the float32 bar of the solver tests).
"""
import time

import numpy as np
import pytest

import inputs
from gpu_common import (f32_envelope, oracle_W, oracle_d, operator_eps, phantom_and_data,
                        print_case, rel, to_gpu, to_np)
from oracle import solvers, wmg

torch = pytest.importorskip("torch")
reco = pytest.importorskip("paper_1310_0956_amd")

pytestmark = pytest.mark.gpu


def _geoms(specs):
    cache = {}
    out = []
    for (n, m, nb, lv) in specs:
        key = (n, m, nb, lv)
        if key not in cache:
            cache[key] = reco.Geometry(n, m, nb, lv, reco.F32)
        out.append(cache[key])
    return out


def _data(g, n_ellipses, seed, noise=0.01):
    """Seeded phantom projected on the device, plus seeded Gaussian noise."""
    x = torch.from_numpy(inputs.ellipse_phantom(g.n, n_ellipses, seed).astype(np.float32)).cuda()
    b = g.project(x)
    torch.cuda.synchronize()
    if noise:
        e = inputs.standard_normal(g.m * g.nb, seed + 500000)
        b += torch.from_numpy((noise * float(b.abs().max()) * e).astype(np.float32)).cuda().view_as(b)
    torch.cuda.synchronize()
    return b


def _solo(g, b, **kw):
    x = g.new_image()
    _, info = g.solve_cgls(b, x=x, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


SMALL = [(64, 90, 91, 2), (128, 90, 182, 2), (128, 180, 182, 3), (128, 180, 182, 3),
         (96, 45, 136, 2), (256, 180, 363, 2), (64, 90, 91, 2), (128, 90, 182, 2)]


def test_batch_matches_solo_small_mix():
    print_case("batch small mix")
    gs = _geoms(SMALL)
    bs = [_data(g, 5 + i, 7000 + i) for i, g in enumerate(gs)]
    bs[6] = torch.zeros_like(bs[6])                       # zero data: done at iteration 0
    tol = [1e-3, 1e-2, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-4]
    lam = [0.0, 0.0, 0.5, 0.0, 0.0, 0.0, 0.0, 0.0]
    pre = [reco.PRECOND_WMG] * 8
    pre[3] = reco.PRECOND_NONE
    fixed = [0, 0, 0, 0, 7, 0, 0, 0]
    xs = [g.new_image().fill_(123.0) for g in gs]         # overwritten: solves start from 0
    infos = reco.solve_batch(gs, bs, xs, tol=tol, lam=lam, precond=pre, fixed_iters=fixed)
    torch.cuda.synchronize()
    for i, g in enumerate(gs):
        xr, ir = _solo(g, bs[i], tol=tol[i], lam=lam[i], precond=pre[i], fixed_iters=fixed[i])
        xb = xs[i].cpu().numpy()
        assert infos[i]["iters"] == ir["iters"], (i, infos[i], ir)
        assert infos[i]["status"] == ir["status"], (i, infos[i], ir)
        assert infos[i]["relres"] == ir["relres"], (i, infos[i], ir)
        assert np.array_equal(xb, xr), (i, float(np.abs(xb - xr).max()))
    assert infos[6]["iters"] == 0 and np.all(xs[6].cpu().numpy() == 0.0)
    assert infos[4]["iters"] == 7
    # a second batch reuses the pooled workspaces and graphs: same bits
    xs2 = [g.new_image() for g in gs]
    infos2 = reco.solve_batch(gs, bs, xs2, tol=tol, lam=lam, precond=pre, fixed_iters=fixed)
    for i in range(len(gs)):
        assert infos2[i]["iters"] == infos[i]["iters"]
        assert torch.equal(xs2[i], xs[i])


def test_batch_matches_solo_tiny_and_large():
    """Small images whose forward blocks span the whole shadow (rays missing the
    image on either side, axis-parallel-only angles, one WMG level) batched
    with a 1024^2 problem whose grid takes one thread per ray where the small
    ones take two: every result equals its solo solve bit for bit."""
    specs = [(24, 2, 35, 3), (14, 6, 33, 2), (5, 3, 8, 1), (31, 9, 45, 1), (16, 4, 23, 3),
             (1024, 720, 1449, 3)]
    print_case("batch tiny and large", specs)
    gs = _geoms(specs)
    bs = [_data(g, 3 + i, 7200 + i) for i, g in enumerate(gs)]
    fixed = [5, 6, 4, 7, 5, 0]
    tol = [1e-3] * 5 + [1e-3]
    pre = [reco.PRECOND_WMG if lv > 1 else reco.PRECOND_NONE for (_, _, _, lv) in specs]
    xs = [g.new_image() for g in gs]
    infos = reco.solve_batch(gs, bs, xs, tol=tol, precond=pre, fixed_iters=fixed)
    torch.cuda.synchronize()
    for i, g in enumerate(gs):
        xr, ir = _solo(g, bs[i], tol=tol[i], precond=pre[i], fixed_iters=fixed[i])
        xb = xs[i].cpu().numpy()
        assert infos[i]["iters"] == ir["iters"] and infos[i]["status"] == ir["status"], (i, infos[i], ir)
        assert np.array_equal(xb, xr), (i, float(np.abs(xb - xr).max()))
        assert np.abs(xb).max() > 0.0


def test_batch_check_every_and_max_iter():
    """Iterations per graph replay and the iteration cap do not change results."""
    print_case("batch tick sizes")
    gs = _geoms([(128, 90, 182, 2)] * 3)
    bs = [_data(g, 10, 7100 + i) for i, g in enumerate(gs)]
    ref = []
    for ce in (1, 5):
        xs = [g.new_image() for g in gs]
        infos = reco.solve_batch(gs, bs, xs, tol=1e-6, max_iter=[4, 9, 13], check_every=ce)
        assert [i["iters"] for i in infos] == [4, 9, 13]
        assert all(i["status"] == "not_converged" for i in infos)
        ref.append([x.cpu().numpy() for x in xs])
    for a, b in zip(ref[0], ref[1]):
        assert np.array_equal(a, b)


def test_batch_mix_sample_full_sizes():
    """The first 12 problems of the 256-problem batched workload at their real sizes."""
    mix = inputs.batch_mix(256)[:12]
    print_case("batch mix sample", [(r.side, r.n_angles) for r in mix])
    gs = _geoms([(r.side, r.n_angles, r.n_bins, inputs.default_levels(r.side)) for r in mix])
    bs = [_data(g, r.n_ellipses, r.seed, r.noise) for g, r in zip(gs, mix)]
    xs = [g.new_image() for g in gs]
    infos = reco.solve_batch(gs, bs, xs, tol=1e-3)
    for i, (g, r) in enumerate(zip(gs, mix)):
        assert infos[i]["status"] == "ok", (i, infos[i])
        xr, ir = _solo(g, bs[i], tol=1e-3)
        assert infos[i]["iters"] == ir["iters"]
        assert np.array_equal(xs[i].cpu().numpy(), xr), i


def test_batch_invalid_arguments():
    g64 = reco.Geometry(64, 90, 91, 2, reco.F64)
    b = torch.zeros((90, 91), dtype=torch.float64, device="cuda")
    x = g64.new_image()
    with pytest.raises(reco.RecoError) as e:
        reco.solve_batch([g64], [b], [x])
    assert e.value.status == reco.RECO_EINVAL
    g = reco.Geometry(64, 90, 91, 2, reco.F32)
    b = torch.zeros((90, 91), dtype=torch.float32, device="cuda")
    with pytest.raises(reco.RecoError):
        reco.solve_batch([g], [b], [g.new_image()], tol=-1.0)
    assert reco.solve_batch([], [], []) == []


# ---------------------------------------------------------------------------
# Server
# ---------------------------------------------------------------------------
def _wait(srv, tickets, timeout=90.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.001)
    return out


REQS = [(128, 90, 182, 2, 1e-3), (256, 180, 363, 2, 1e-2), (128, 180, 182, 3, 1e-3),
        (64, 90, 91, 2, 1e-3), (256, 256, 363, 2, 1e-3), (128, 90, 182, 2, 1e-2)]


def _server_run(budget, slots, gap_s):
    srv = reco.Server(budget, max_slots=slots)
    try:
        gs = _geoms([r[:4] for r in REQS])
        bs = [_data(g, 8 + i, 7300 + i) for i, g in enumerate(gs)]
        xs = [g.new_image() for g in gs]
        tickets = []
        for (n, m, nb, lv, tol), b, x in zip(REQS, bs, xs):
            tickets.append(srv.submit(n, m, nb, lv, b, x, tol=tol))
            time.sleep(gap_s)
        res = _wait(srv, tickets)
        return gs, bs, xs, [res[t] for t in tickets]
    finally:
        srv.close()


def test_server_results_equal_solo():
    print_case("server continuous batching")
    gs, bs, xs, res = _server_run(8 << 30, 16, 0.002)
    for i, (g, r) in enumerate(zip(gs, res)):
        assert r["status"] == "ok", r
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        xr, ir = _solo(g, bs[i], tol=REQS[i][4])
        assert r["iters"] == ir["iters"]
        assert np.array_equal(xs[i].cpu().numpy(), xr), i


def test_server_tiers_mixed_sizes():
    """Requests whose iteration costs at least that of a 1024^2 image with
    512 angles run in the server's large tier (one at a time, geometry built
    on its own thread); the others are batched in the small tier.  Results
    equal solo solves in both tiers."""
    print_case("server tiers")
    reqs = [(1024, 512, 1449, 4, 1e-2), (128, 90, 182, 2, 1e-3), (1024, 512, 1449, 4, 1e-3),
            (256, 180, 363, 2, 1e-3), (64, 90, 91, 2, 1e-2)]
    srv = reco.Server(8 << 30, max_slots=16)
    try:
        gs = _geoms([r[:4] for r in reqs])
        bs = [_data(g, 6 + i, 7500 + i) for i, g in enumerate(gs)]
        xs = [g.new_image() for g in gs]
        tickets = [srv.submit(n, m, nb, lv, b, x, tol=tol)
                   for (n, m, nb, lv, tol), b, x in zip(reqs, bs, xs)]
        res = _wait(srv, tickets)
    finally:
        srv.close()
    for i, (g, t) in enumerate(zip(gs, tickets)):
        r = res[t]
        assert r["status"] == "ok", r
        xr, ir = _solo(g, bs[i], tol=reqs[i][4])
        assert r["iters"] == ir["iters"]
        assert np.array_equal(xs[i].cpu().numpy(), xr), i
    large = sorted((res[tickets[i]]["t_admit"], res[tickets[i]]["t_done"]) for i in (0, 2))
    assert large[1][0] >= large[0][1] - 1e-6     # the large tier runs one problem at a time


def test_server_one_slot_serialises():
    print_case("server one slot")
    gs, bs, xs, res = _server_run(8 << 30, 1, 0.0)
    order = sorted(range(len(res)), key=lambda i: res[i]["t_admit"])
    for a, b in zip(order, order[1:]):
        assert res[b]["t_admit"] >= res[a]["t_done"] - 1e-6
    for i, g in enumerate(gs):
        xr, _ = _solo(g, bs[i], tol=REQS[i][4])
        assert np.array_equal(xs[i].cpu().numpy(), xr), i


def test_server_budget_limits_and_rejects():
    print_case("server budget")
    # room for about one 256^2 request at a time
    srv = reco.Server(3 << 20, max_slots=8)
    try:
        g = reco.Geometry(256, 180, 363, 2, reco.F32)
        b = _data(g, 10, 7400)
        xs = [g.new_image() for _ in range(3)]
        ts = [srv.submit(256, 180, 363, 2, b, x) for x in xs]
        big_b = torch.zeros(2048 * 2897, dtype=torch.float32, device="cuda")
        big_x = torch.zeros(2048 * 2048, dtype=torch.float32, device="cuda")
        tb = srv.submit(2048, 2048, 2897, 5, big_b, big_x)
        res = _wait(srv, ts)
        with pytest.raises(reco.RecoError) as e:
            for _ in range(2000):
                if srv.poll(tb) is not None:
                    break
                time.sleep(0.001)
        assert e.value.status == reco.RECO_ENOMEM
        xr, _ = _solo(g, b, tol=1e-3)
        for t, x in zip(ts, xs):
            assert res[t]["status"] == "ok"
            assert np.array_equal(x.cpu().numpy(), xr)
        spans = sorted((res[t]["t_admit"], res[t]["t_done"]) for t in ts)
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert b0 >= a1 - 1e-6          # the budget admitted one at a time
    finally:
        srv.close()


def test_server_invalid_submit():
    srv = reco.Server(1 << 30, max_slots=4)
    try:
        b = torch.zeros(90 * 100, dtype=torch.float32, device="cuda")
        x = torch.zeros(100 * 100, dtype=torch.float32, device="cuda")
        with pytest.raises(reco.RecoError) as e:
            srv.submit(100, 90, 100, 4, b, x)          # 100 is not a multiple of 2^3
        assert e.value.status == reco.RECO_EINVAL
        with pytest.raises(reco.RecoError) as e:
            srv.submit(100, 90, 100, 2, b, x, tol=-1.0)
        assert e.value.status == reco.RECO_EINVAL
        with pytest.raises(ValueError):
            srv.submit(100, 90, 101, 2, b, x)          # b has the wrong size
        with pytest.raises(reco.RecoError) as e:
            srv.poll(987654321)
        assert e.value.status == reco.RECO_ENOTFOUND
    finally:
        srv.close()


# (n, m, nb, levels, precond, lambda, tol): oracle-checked subset
ORACLE_SET = [(64, 90, 91, 2, reco.PRECOND_WMG, 0.0, 1e-3),
              (128, 90, 182, 3, reco.PRECOND_WMG, 0.5, 1e-3),
              (128, 180, 182, 2, reco.PRECOND_NONE, 0.0, 1e-3),
              (256, 180, 363, 3, reco.PRECOND_WMG, 0.0, 1e-2)]


def _oracle_check(label, problems, bs_np, xs, iters):
    for (n, m, nb, lv, pre, lam, tol), b, x, K in zip(problems, bs_np, xs, iters):
        W = oracle_W(n, m, nb)
        M = None
        if pre == reco.PRECOND_WMG:
            d = oracle_d(n, m, nb, lv - 1) + lam
            M = (lambda dd, L: (lambda v: wmg.apply_additive_diag(v, dd, L)))(d, lv - 1)
        refK = solvers.pcgls(W, b, fixed_iters=K, lam=lam, precond=M)
        g = reco.Geometry(n, m, nb, lv, reco.F32)
        e_fwd, e_bwd = operator_eps(g, W, np.random.default_rng(n).random((n, n)), b.reshape(m, nb))
        eps = max(e_fwd, e_bwd)
        env = f32_envelope(lambda h: solvers.pcgls(W, b, fixed_iters=K, lam=lam, precond=M,
                                                   store=h), refK.x, eps)
        dev = rel(to_np(x), refK.x)
        print(f"{label} {n}x{n} {m}x{nb} lv {lv} precond {pre} lam {lam}: K {K} dev {dev:.3e} "
              f"eps {eps:.3e} envelope {env:.3e}", flush=True)
        assert dev <= 3 * env


def test_batch_and_server_results_match_oracle():
    print_case("batch and server vs oracle")
    bs_np, bs = [], []
    for i, (n, m, nb, lv, pre, lam, tol) in enumerate(ORACLE_SET):
        _, b = phantom_and_data(n, m, nb, 6 + i, 7700 + i, noise=0.01)
        bs_np.append(b)
        bs.append(to_gpu(b.reshape(m, nb), torch.float32))
    gs = _geoms([p[:4] for p in ORACLE_SET])
    xs = [g.new_image() for g in gs]
    infos = reco.solve_batch(gs, bs, xs, tol=[p[6] for p in ORACLE_SET],
                             lam=[p[5] for p in ORACLE_SET], precond=[p[4] for p in ORACLE_SET])
    assert all(i["status"] == "ok" for i in infos), infos
    _oracle_check("batched", ORACLE_SET, bs_np, xs, [i["iters"] for i in infos])
    srv = reco.Server(8 << 30, max_slots=16)
    try:
        xs2 = [g.new_image() for g in gs]
        tickets = [srv.submit(n, m, nb, lv, b, x, tol=tol, precond=pre, lam=lam)
                   for (n, m, nb, lv, pre, lam, tol), b, x in zip(ORACLE_SET, bs, xs2)]
        res = _wait(srv, tickets)
    finally:
        srv.close()
    assert all(res[t]["status"] == "ok" for t in tickets)
    _oracle_check("served", ORACLE_SET, bs_np, xs2, [res[t]["iters"] for t in tickets])
