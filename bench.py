"""Benchmark: WMG-CGLS reconstructions per second on one MI355X.

Workload (default): 512 x 512 image on [-1,1]^2, 360 angles over 180 degrees,
725 detector bins of one pixel, seeded 20-ellipse phantoms, additive Gaussian
noise of 1% of the maximum projection, float32 projector/backprojector with
float64 Krylov scalars and reductions, 3-level WMG-preconditioned CGLS to a
relative normal-equation residual of 1e-3.  One step = one full reconstruction
of one sinogram already resident in HBM (geometry and packet diagonal built
once beforehand, reported as setup).

Prints one JSON line with the throughput, the per-kernel roofline of the
dominant kernel (HIP-event timed inside the measured steps) and the CPU
float64 oracle timed on a bounded sample on the host; further objects report
the 512^2 solver comparison (CGLS, WMG-CGLS, WMG-GMRES(30), SIRT), the batched
and served workloads and the 2048^2 reconstruction.
"""
import argparse
import hashlib
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed)
HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(n=512, m=360, nb=725, levels=3, ellipses=20, noise=0.01, seed=1000, tol=1e-3)
# Algorithmic VALU lane-operations per nonzero update of A or A^T: evaluate the
# exact-length weight (one fused multiply-add and one clamp), accumulate it
# (one fused multiply-add) and advance the ray or pixel position (one add).
ALG_OPS_PER_UPDATE = 4.0
COPY_BYTES = 256 << 20


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate CPU time spent on oracle reconstructions")
    ap.add_argument("--batch", type=int, default=256,
                    help="reconstructions in the batched leg (0: skip)")
    ap.add_argument("--serve", type=int, default=400,
                    help="requests in the serving leg (0: skip)")
    ap.add_argument("--serve-fracs", default="0.5,0.7,0.9",
                    help="arrival rates as fractions of the one-at-a-time saturation throughput")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-low-budget-gib", type=float, default=1.0,
                    help="budget of one more run at 0.7 of saturation (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--no-tiny64", action="store_true", help="skip the 64^2 float64 leg")
    ap.add_argument("--no-semiconv", action="store_true",
                    help="skip the 160^2 noisy-data semi-convergence leg")
    ap.add_argument("--no-ct2048", action="store_true", help="skip the 2048^2 leg")
    ap.add_argument("--no-solvers", action="store_true",
                    help="skip the 512^2 solver comparisons (CGLS, GMRES, BiCGStab, SIRT; "
                         "CGLS and BiCGStab with Joseph's kernel)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only run the timed steps (for rocprofv3)")
    ap.add_argument("--profile-workload", choices=("ct512", "ct2048"), default="ct512",
                    help="workload of --profile-only: the 512^2 headline or the 2048^2 "
                         "reconstruction")
    return ap.parse_args()


def make_inputs(reco, torch, g, count):
    import numpy as np
    import inputs
    w = WORKLOAD
    sinos = []
    for i in range(count):
        x = inputs.ellipse_phantom(w["n"], w["ellipses"], w["seed"] + i)
        xt = torch.from_numpy(x.astype(np.float32)).cuda()
        b = g.project(xt)
        torch.cuda.synchronize()
        bmax = float(b.abs().max())
        e = inputs.standard_normal(w["m"] * w["nb"], w["seed"] + i + 500000)
        b += torch.from_numpy((w["noise"] * bmax * e).astype(np.float32)).cuda().view_as(b)
        sinos.append(b.contiguous())
    torch.cuda.synchronize()
    return sinos


def source_hash(files):
    m = hashlib.sha256()
    for name in files:
        m.update(open(os.path.join(ROOT, "paper_1310_0956_amd", "csrc", name), "rb").read())
    return m.hexdigest()[:16]


def traffic_for(family, workload="ct512"):
    """Calibrated HBM bytes per launch of a kernel family from the committed
    rocprofv3 counter summary of a workload, if it was taken on the current
    kernel sources (else None)."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    ent = json.load(open(p)).get(family)
    if not ent or ent.get("source_sha256_16") != source_hash(ent["source_files"]):
        return None
    return ent.get("bytes_per_launch")


def host_info():
    """CPU model, logical CPU count and RAM of the host the oracle runs on."""
    model, mem_gib = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem_gib = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "ram_gib": mem_gib}


def roofline_of(kt, working, nnz, workload):
    """Roofline object of the dominant projector from per-family HIP-event
    totals: algorithmic updates (nnz per launch that did work) over the summed
    launch durations, against the VALU lane-operation peak; beside it the
    calibrated HBM traffic per launch from the committed counter summary and
    the bandwidth fraction it implies."""
    gups = {k: nnz * working[k] / (kt[k][1] * 1e-3) / 1e9 for k in working if kt[k][1] > 0}
    dom = "forward" if kt["forward"][1] >= kt["backward"][1] else "backward"
    peak = PEAK_VALU_LANE_OPS / ALG_OPS_PER_UPDATE / 1e9
    avg_working_ms = kt[dom][1] / working[dom]
    traffic = traffic_for(dom, workload)
    out = {
        "bound": "alu",
        "kernel": dom,
        "achieved": round(gups[dom], 3),
        "peak": round(peak, 3),
        "unit": "Gupdate/s",
        "frac": round(gups[dom] / peak, 4),
        "traffic": traffic,
        "avg_launch_ms": round(kt[dom][1] / kt[dom][0], 5),
        "avg_working_launch_ms": round(avg_working_ms, 5),
        "launches": kt[dom][0],
        "working_launches": working[dom],
        "updates_per_working_launch": nnz,
        "alg_valu_ops_per_update": ALG_OPS_PER_UPDATE,
    }
    if traffic:
        gbs = traffic / (avg_working_ms * 1e-3) / 1e9
        out["hbm_GBs_from_traffic"] = round(gbs, 1)
        out["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    return out, gups


def cpu_baseline(args):
    """Oracle WMG-CGLS on the host: whole reconstructions of the same workload,
    repeated until about ten seconds of CPU time (matrix assembly and packet
    diagonal are setup, as on the GPU).  Returns the matrix too (for the
    matvec timing)."""
    import numpy as np
    import inputs
    from oracle import solvers, wmg
    from oracle.geometry import Geometry as OG
    from oracle.projector import system_matrix
    w = WORKLOAD
    og = OG(w["n"], w["m"], w["nb"])
    W = system_matrix(og)
    L = w["levels"] - 1
    d = wmg.packet_diagonal_by_angles(og, L)
    M = lambda v: wmg.apply_additive_diag(v, d, L)  # noqa: E731
    solved, iters, t_sum = 0, [], 0.0
    while solved < 1 or (t_sum < args.cpu_seconds and solved < 8):
        x = inputs.ellipse_phantom(w["n"], w["ellipses"], w["seed"] + solved)
        b = W @ x.ravel()
        e = inputs.standard_normal(b.size, w["seed"] + solved + 500000)
        b = (b + w["noise"] * np.abs(b).max() * e).astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        res = solvers.pcgls(W, b, tol=w["tol"], max_iter=1000, precond=M)
        t_sum += time.perf_counter() - t0
        iters.append(res.iters)
        solved += 1
    return solved, t_sum, iters, W


def cpu_matvec(W, threads):
    """Oracle A and A^T (scipy CSR, float64; A^T stored as its own CSR matrix)
    at the 512^2 workload: updates per second on one thread and on a pool of
    threads over row blocks (scipy's CSR product releases the GIL)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    WT = W.T.tocsr()
    x = np.ones(W.shape[1])
    y = np.ones(W.shape[0])
    out = {"nnz": int(W.nnz), "threads": threads}

    def rate(fn, reps=3):
        fn()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        return W.nnz * reps / (time.perf_counter() - t0)

    out["A_updates_per_s_1thread"] = round(rate(lambda: W @ x) / 1e6, 2)
    out["AT_updates_per_s_1thread"] = round(rate(lambda: WT @ y) / 1e6, 2)
    ex = ThreadPoolExecutor(threads)
    for name, M, v in (("A", W, x), ("AT", WT, y)):
        cuts = np.linspace(0, M.shape[0], threads + 1).astype(int)
        blocks = [M[cuts[i]:cuts[i + 1]] for i in range(threads)]
        out[f"{name}_updates_per_s_{threads}threads"] = round(
            rate(lambda: list(ex.map(lambda B: B @ v, blocks))) / 1e6, 2)
    ex.shutdown()
    out["unit"] = "M updates/s"
    return out


def cpu_config0():
    """The 64^2 float64 case on the oracle: 50 iterations each of SIRT, CGLS,
    WMG-CGLS with the packet diagonal (the GPU method) and with exact packet
    blocks (the additive-exact variant); relative residual and error against
    the phantom."""
    import numpy as np
    import inputs
    from oracle import solvers, wmg
    from oracle.geometry import Geometry as OG
    from oracle.projector import system_matrix
    n, m, nb, L = 64, 90, 64, 1
    W = system_matrix(OG(n, m, nb))
    x = inputs.ellipse_phantom(n, 10, 0).ravel()
    b = W @ x
    d = wmg.packet_diagonal_by_angles(OG(n, m, nb), L)
    blocks = wmg.galerkin_blocks(W, n, L)
    hybrid = wmg.HybridCycle(W, n, L)
    runs = [("sirt", lambda: solvers.sirt(W, b, fixed_iters=50)),
            ("cgls", lambda: solvers.pcgls(W, b, fixed_iters=50)),
            ("wmg_cgls_diag", lambda: solvers.pcgls(
                W, b, fixed_iters=50, precond=lambda v: wmg.apply_additive_diag(v, d, L))),
            ("wmg_cgls_additive_exact", lambda: solvers.pcgls(
                W, b, fixed_iters=50, precond=lambda v: wmg.apply_additive_exact(v, blocks, n, L))),
            ("wmg_hybrid_bicgstab", lambda: solvers.bicgstab_right(W, b, fixed_iters=50,
                                                                   precond=hybrid))]
    out = {"workload": "tiny64 on the float64 oracle (the tiny64_f64 object's case), "
                       "50 iterations each"}
    for name, fn in runs:
        t0 = time.perf_counter()
        res = fn()
        ms = (time.perf_counter() - t0) * 1e3
        err = float(np.linalg.norm(res.x - x) / np.linalg.norm(x))
        out[name] = {"ms": round(ms, 1), "relres": float("%.4g" % res.relres),
                     "rel_error_vs_phantom": round(err, 5)}
    return out


def percentiles(v):
    import numpy as np
    return (round(float(np.percentile(v, 50)), 4), round(float(np.percentile(v, 99)), 4))


def gpu_sinogram(torch, g, n_ellipses, seed, noise):
    """Seeded phantom projected on the device plus seeded Gaussian noise."""
    import numpy as np
    import inputs
    x = torch.from_numpy(inputs.ellipse_phantom(g.n, n_ellipses, seed).astype(np.float32)).cuda()
    b = g.project(x)
    torch.cuda.synchronize()
    e = inputs.standard_normal(g.m * g.nb, seed + 500000)
    b += torch.from_numpy((noise * float(b.abs().max()) * e).astype(np.float32)).cuda().view_as(b)
    torch.cuda.synchronize()
    return b


def batch_leg(reco, torch, count):
    """256 mixed-size reconstructions: one batched solve against the same
    problems solved one at a time on the same GPU."""
    import inputs
    mix = inputs.batch_mix(count)
    t0 = time.perf_counter()
    geo = {}
    for r in mix:
        k = (r.side, r.n_angles)
        if k not in geo:
            geo[k] = reco.Geometry(r.side, r.n_angles, r.n_bins, inputs.default_levels(r.side),
                                   reco.F32)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    gs = [geo[(r.side, r.n_angles)] for r in mix]
    bs = [gpu_sinogram(torch, g, r.n_ellipses, r.seed, r.noise) for g, r in zip(gs, mix)]
    xs = [g.new_image() for g in gs]
    nnz = {k: g.count_nnz() for k, g in geo.items()}
    # warm-up: the whole batch (its workspaces, up to one per problem, then sit
    # in the geometries' pools, so the timed runs do not allocate) and one solo
    # solve of every geometry
    reco.solve_batch(gs, bs, xs, tol=1e-3)
    seen = set()
    for g, b, x, r in zip(gs, bs, xs, mix):
        if (r.side, r.n_angles) not in seen:
            seen.add((r.side, r.n_angles))
            g.solve_cgls(b, x=x, tol=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = reco.solve_batch(gs, bs, xs, tol=1e-3)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    solo_lat = []
    for g, b, x in zip(gs, bs, xs):
        s0 = time.perf_counter()
        g.solve_cgls(b, x=x, tol=1e-3)
        solo_lat.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    its = [i["iters"] for i in infos]
    updates = sum(2 * nnz[(r.side, r.n_angles)] * (i["iters"] + 0.5) for r, i in zip(mix, infos))
    done_ms = sorted(i["elapsed_ms"] for i in infos)
    return {
        "workload": f"{count} reconstructions, side in {{128,256,512,1024}}, angles in "
                    "{90,180,360,720}, bins ceil(side*sqrt2), 5-30 ellipses, 1% noise, "
                    "WMG-CGLS to rel-res 1e-3",
        "recons_per_s": round(count / t_batch, 3),
        "seconds": round(t_batch, 4),
        "solo_recons_per_s": round(count / t_solo, 3),
        "solo_seconds": round(t_solo, 4),
        "speedup_vs_solo": round(t_solo / t_batch, 3),
        "all_ok": all(i["status"] == "ok" for i in infos),
        "iters_min_max": [min(its), max(its)],
        "gupdates_per_s": round(updates / t_batch / 1e9, 2),
        "completion_ms_p50_p99": percentiles(done_ms),
        "solo_latency_ms_p50_p99": percentiles(solo_lat),
        "geometries": len(geo),
        "setup_s": round(setup_s, 3),
    }


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def serve_setup(reco, torch, count):
    """The served requests (sizes and seeds of the serving mix; they do not
    depend on the arrival rate), their data, and the one-at-a-time baseline:
    each request solved alone in arrival order, the first request of a
    geometry also paying for building it (tables and packet diagonal), as in
    the server.  The saturation throughput is count / total solo time."""
    import inputs
    mix = inputs.serving_mix(count, 1.0)   # arrivals at 1/s; a rate r divides them by r
    geo = {}
    for r in mix:
        k = (r.side, r.n_angles)
        if k not in geo:
            geo[k] = reco.Geometry(r.side, r.n_angles, r.n_bins, inputs.default_levels(r.side),
                                   reco.F32)
    progress(f"serving: {len(geo)} geometries for {count} requests")
    gs = [geo[(r.side, r.n_angles)] for r in mix]
    bs = [gpu_sinogram(torch, g, r.n_ellipses, r.seed, r.noise) for g, r in zip(gs, mix)]
    xs = [g.new_image() for g in gs]
    solo_ms, built = [], set()
    for i, (g, b, x, r) in enumerate(zip(gs, bs, xs, mix)):
        if i % 100 == 0:
            progress(f"serving: solo baseline {i}/{count}")
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        if (r.side, r.n_angles) not in built:
            built.add((r.side, r.n_angles))
            reco.Geometry(r.side, r.n_angles, r.n_bins, inputs.default_levels(r.side), reco.F32)
        g.solve_cgls(b, x=x, tol=r.tol)
        torch.cuda.synchronize()
        solo_ms.append((time.perf_counter() - s0) * 1e3)
    return {"mix": mix, "gs": gs, "bs": bs, "xs": xs, "solo_ms": solo_ms,
            "geometries": len(built), "saturation": count / (sum(solo_ms) * 1e-3)}


def serve_run(reco, torch, S, rate, budget_gib, slots):
    """Poisson arrivals at `rate` into the server; the one-at-a-time FIFO
    server fed the same arrivals is computed from the measured solo times."""
    import threading
    import inputs
    mix, gs, bs = S["mix"], S["gs"], S["bs"]
    count = len(mix)
    arrivals = [r.arrival_s / rate for r in mix]
    fifo_lat, free_at = [], 0.0
    for a, ms in zip(arrivals, S["solo_ms"]):
        start = max(free_at, a)
        free_at = start + ms * 1e-3
        fifo_lat.append((free_at - a) * 1e3)
    progress(f"serving: {count} requests at {rate:.1f}/s, budget {budget_gib} GiB")
    srv = reco.Server(int(budget_gib * (1 << 30)), max_slots=slots)
    tickets = [None] * count
    outs = [g.new_image() for g in gs]
    t_start = reco.clock() + 0.05

    def submitter():
        for i, r in enumerate(mix):
            dt = t_start + arrivals[i] - reco.clock()
            if dt > 0:
                time.sleep(dt)
            tickets[i] = srv.submit(r.side, r.n_angles, r.n_bins, inputs.default_levels(r.side),
                                    bs[i], outs[i], tol=r.tol)

    th = threading.Thread(target=submitter)
    th.start()
    res = [None] * count
    pending, last = list(range(count)), time.time()
    while pending:
        still = []
        for i in pending:
            if tickets[i] is not None:
                res[i] = srv.poll(tickets[i])
            if res[i] is None:
                still.append(i)
        pending = still
        if time.time() - last > 30:
            progress(f"serving: {count - len(pending)}/{count} done")
            last = time.time()
        time.sleep(0.0005)
    th.join()
    srv.close()
    lat = [(v["t_done"] - v["t_submit"]) * 1e3 for v in res]
    span = max(v["t_done"] for v in res) - min(v["t_submit"] for v in res)
    by_side = {}
    for side in sorted({r.side for r in mix}):
        idx = [i for i, r in enumerate(mix) if r.side == side]
        by_side[str(side)] = {"count": len(idx),
                              "latency_ms_p50_p99": percentiles([lat[i] for i in idx]),
                              "solo_fifo_latency_ms_p50_p99": percentiles([fifo_lat[i] for i in idx])}
    return {
        "rate_per_s": round(rate, 3), "budget_gib": budget_gib,
        "recons_per_s": round(count / span, 3),
        "latency_ms_p50_p99": percentiles(lat),
        "queue_ms_p50_p99": percentiles([(v["t_admit"] - v["t_submit"]) * 1e3 for v in res]),
        "solo_fifo_latency_ms_p50_p99": percentiles(fifo_lat),
        "by_side": by_side,
        "all_ok": all(v["status"] == "ok" for v in res),
        "results_equal_solo": bool(all(torch.equal(a, b) for a, b in zip(outs, S["xs"]))),
    }


def serve_leg(reco, torch, args):
    """The serving mix at fractions of the one-at-a-time saturation throughput,
    and once more under a small device-memory budget."""
    S = serve_setup(reco, torch, args.serve)
    sat = S["saturation"]
    runs = []
    for frac in [float(f) for f in args.serve_fracs.split(",") if f]:
        r = serve_run(reco, torch, S, frac * sat, args.serve_budget_gib, args.serve_slots)
        r["fraction_of_saturation"] = frac
        runs.append(r)
    if args.serve_low_budget_gib > 0:
        r = serve_run(reco, torch, S, 0.7 * sat, args.serve_low_budget_gib, args.serve_slots)
        r["fraction_of_saturation"] = 0.7
        runs.append(r)
    return {
        "workload": f"{args.serve} requests, Poisson arrivals, side 256/512/1024/2048 at "
                    "40/30/20/10%, angles side/2..1.5 side, tol 1e-2 or 1e-3, 1% noise",
        "saturation_recons_per_s": round(sat, 3),
        "geometries_built": S["geometries"],
        "max_slots": args.serve_slots,
        "runs": runs,
        "note": "saturation: the one-at-a-time throughput (request count over the summed solo "
                "service times, geometry build on first use plus the solve); solo FIFO "
                "latency: a one-at-a-time server fed the same arrivals, from those service times",
    }


def solvers_leg(reco, torch, g, sinos):
    """The solvers of the 512^2 workload to rel-res 1e-3 (iteration cap 1000):
    iterations, applications of W^T W and time per reconstruction."""
    out = {}
    x = g.new_image()
    runs = [("cgls", lambda b: g.solve_cgls(b, x=x, tol=1e-3, precond=reco.PRECOND_NONE)),
            ("wmg_cgls", lambda b: g.solve_cgls(b, x=x, tol=1e-3)),
            ("wmg_gmres30", lambda b: g.solve_gmres(b, x=x, tol=1e-3, restart=30)),
            ("bicgstab", lambda b: g.solve_bicgstab(b, x=x, tol=1e-3, precond=reco.PRECOND_NONE)),
            ("wmg_bicgstab", lambda b: g.solve_bicgstab(b, x=x, tol=1e-3)),
            ("sirt", lambda b: g.solve_sirt(b, x=x, tol=1e-3, max_iter=1000))]
    for name, fn in runs:
        fn(sinos[0])
        torch.cuda.synchronize()
        reps = 1 if name == "sirt" else 3
        t0 = time.perf_counter()
        infos = [fn(sinos[i % len(sinos)])[1] for i in range(reps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        out[name] = {"iters": infos[-1]["iters"], "matvecs": infos[-1]["matvecs"],
                     "status": infos[-1]["status"], "relres": round(infos[-1]["relres"], 6),
                     "ms_per_recon": round(ms, 3)}
    return out


def joseph_leg(reco, torch):
    """The 512^2 workload with Joseph's projection kernel (the paper's W) in
    place of exact intersection lengths: its own sinograms (Joseph projections
    of the same phantoms, same noise recipe), solved to rel-res 1e-3.  Errors
    are recorded, not raised."""
    w = WORKLOAD
    out = {}
    try:
        gj = reco.Geometry(w["n"], w["m"], w["nb"], w["levels"], reco.F32,
                           projector=reco.PROJ_JOSEPH)
        sinos = make_inputs(reco, torch, gj, 2)
        x = gj.new_image()
        runs = [("cgls", lambda b: gj.solve_cgls(b, x=x, tol=1e-3, precond=reco.PRECOND_NONE)),
                ("wmg_cgls", lambda b: gj.solve_cgls(b, x=x, tol=1e-3)),
                ("wmg_bicgstab", lambda b: gj.solve_bicgstab(b, x=x, tol=1e-3))]
        for name, fn in runs:
            fn(sinos[0])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = [fn(sinos[i % len(sinos)])[1] for i in range(3)]
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / 3 * 1e3
            out[name] = {"iters": infos[-1]["iters"], "matvecs": infos[-1]["matvecs"],
                         "status": infos[-1]["status"], "relres": round(infos[-1]["relres"], 6),
                         "ms_per_recon": round(ms, 3)}
        gj.close()
    except Exception as e:   # recorded in the output line; the other legs stand
        out["error"] = repr(e)
    return out


SEMICONV_GRIDS = {
    "sirt": [1, 2, 5, 10, 20, 50, 100, 200, 300, 500, 700, 1000, 1500, 2000, 3000, 4000, 6000],
    "bicgstab": [1, 2, 3, 5, 7, 10, 15, 20, 30, 50, 70, 100, 150, 200, 300],
    "wmg_bicgstab": [1, 2, 3, 4, 5, 6, 8, 10, 12, 14, 17, 20, 25, 30, 40, 60, 100],
    "wmg_cgls": [1, 2, 3, 4, 5, 6, 8, 10, 12, 14, 17, 20, 25, 30, 40, 60, 100],
    "wmg_hybrid_bicgstab": [1, 2, 3, 4, 5, 6, 8, 10, 12, 14, 17, 20, 25, 30, 40, 60, 100],
}


def semiconv_leg(reco, torch):
    """The paper's noisy-data experiment (Section 4.3) at its shape: a 160^2
    image, 400 angles x 160 rays, 3-level WMG, 1% uniform white noise
    eps = 0.01 U(-1, 1) max|b|; seeded ellipses stand in for its phantom.  For
    each solver the error ||x_k - x_ex|| / ||x_ex|| (x_0 = 0, so this is
    ||e_k|| / ||e_0||) on a log-spaced grid of iteration counts, each a
    separate fixed-iteration solve; k_opt and the error minimum."""
    import numpy as np
    import inputs
    n, m, nb, lv = 160, 400, 160, 3
    x_ex = inputs.ellipse_phantom(n, 10, 11)
    g = reco.Geometry(n, m, nb, lv, reco.F32)
    b = g.project(torch.from_numpy(x_ex.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    eps = inputs.uniform_noise(m * nb, 12).reshape(m, nb)
    bn = b + torch.from_numpy((0.01 * float(b.abs().max()) * eps).astype(np.float32)).cuda()
    xe = torch.from_numpy(x_ex.astype(np.float32)).cuda()
    nx = float(torch.linalg.vector_norm(xe))
    # Tikhonov weight of the paper's regularized Krylov runs, lambda = 10 in its
    # pixel units; W here measures lengths in units of the domain [-1, 1]^2
    # (pixel side h = 2/n), so W^T W carries a factor h^2 and so does lambda
    lam = 10.0 * (2.0 / n) ** 2
    solve = {"sirt": lambda k: g.solve_sirt(bn, fixed_iters=k),
             "bicgstab": lambda k: g.solve_bicgstab(bn, fixed_iters=k, precond=reco.PRECOND_NONE),
             "wmg_bicgstab": lambda k: g.solve_bicgstab(bn, fixed_iters=k),
             "wmg_cgls": lambda k: g.solve_cgls(bn, fixed_iters=k),
             "bicgstab_reg": lambda k: g.solve_bicgstab(bn, fixed_iters=k, lam=lam,
                                                        precond=reco.PRECOND_NONE),
             "wmg_bicgstab_reg": lambda k: g.solve_bicgstab(bn, fixed_iters=k, lam=lam),
             "wmg_cgls_reg": lambda k: g.solve_cgls(bn, fixed_iters=k, lam=lam),
             "wmg_hybrid_bicgstab": lambda k: g.solve_bicgstab(
                 bn, fixed_iters=k, precond=reco.PRECOND_WMG_HYBRID),
             "wmg_hybrid_bicgstab_reg": lambda k: g.solve_bicgstab(
                 bn, fixed_iters=k, lam=lam, precond=reco.PRECOND_WMG_HYBRID)}
    out = {"workload": "160^2 image, 400 angles x 160 rays, 10 ellipses, 1% uniform noise, "
                       "3-level WMG, float32; error of fixed-iteration solves; wmg_*: the "
                       "additive packet-diagonal cycle, wmg_hybrid_*: the hybrid cycle with "
                       "exact coarsest solves; *_reg: Tikhonov "
                       f"lambda = 10 h^2 = {lam:.6g}"}
    # the hybrid cycle's coarsest Cholesky factors are built on first use per
    # lambda (float64, one Galerkin apply per unknown): timed here as set-up
    setup = {}
    for key, la in (("lambda_0", 0.0), ("lambda_reg", lam)):
        t0 = time.perf_counter()
        g.wmg_hybrid_apply(xe, lam=la)
        torch.cuda.synchronize()
        setup[key] = round((time.perf_counter() - t0) * 1e3, 1)
    out["hybrid_factor_setup_ms"] = setup
    grids = dict(SEMICONV_GRIDS)
    for name in ("bicgstab", "wmg_bicgstab", "wmg_cgls", "wmg_hybrid_bicgstab"):
        grids[name + "_reg"] = SEMICONV_GRIDS[name]
    for name, ks in grids.items():
        errs, done = [], []
        for k in ks:
            x, info = solve[name](k)
            errs.append(float(torch.linalg.vector_norm(x - xe)) / nx)
            done.append(info["iters"])
        i = int(np.argmin(errs))
        out[name] = {"k_opt": ks[i], "err_min": round(errs[i], 5),
                     "curve": [[k, round(e, 5)] for k, e in zip(ks, errs)],
                     "iters_run": done}
    # time per iteration at the error-minimising iteration count (the paper's
    # Table 3 compares whole solves to k_opt)
    for name in ("bicgstab", "wmg_bicgstab", "wmg_hybrid_bicgstab"):
        k = out[name]["k_opt"]
        solve[name](k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve[name](k)
        torch.cuda.synchronize()
        out[name]["ms_at_k_opt"] = round((time.perf_counter() - t0) * 1e3, 3)
    return out


def tiny64_leg(reco, torch):
    """64^2, 90 angles x 64 bins, 10-ellipse noiseless phantom, float64:
    50 iterations each of SIRT, CGLS and 2-level WMG-CGLS, and of BiCGStab
    with the hybrid cycle and exact coarsest solves (its factors built before
    the timing)."""
    import numpy as np
    import inputs
    g = reco.Geometry(64, 90, 64, 2, reco.F64)
    x = torch.from_numpy(inputs.ellipse_phantom(64, 10, 0)).cuda()
    b = g.project(x)
    torch.cuda.synchronize()
    out = {"workload": "tiny64: 64x64, 90 angles x 64 bins, 10-ellipse noiseless phantom, float64, "
                       "50 iterations each"}
    xs = g.new_image()
    for name, fn in [("sirt", lambda: g.solve_sirt(b, x=xs, fixed_iters=50)),
                     ("cgls", lambda: g.solve_cgls(b, x=xs, fixed_iters=50,
                                                   precond=reco.PRECOND_NONE)),
                     ("wmg_cgls", lambda: g.solve_cgls(b, x=xs, fixed_iters=50)),
                     ("wmg_hybrid_bicgstab", lambda: g.solve_bicgstab(
                         b, x=xs, fixed_iters=50, precond=reco.PRECOND_WMG_HYBRID))]:
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            _, info = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        err = float(torch.linalg.norm(xs - x) / torch.linalg.norm(x))
        out[name] = {"ms_median_of_3": round(sorted(ts)[1], 3),
                     "relres": float("%.4g" % info["relres"]), "rel_error_vs_phantom": round(err, 5)}
    return out


def ct2048_leg(reco, torch):
    """2048^2 image, 2048 angles x 2897 bins, 5-level WMG-CGLS to rel-res 1e-3."""
    t0 = time.perf_counter()
    g = reco.Geometry(2048, 2048, 2897, 5, reco.F32)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    nnz = g.count_nnz()
    b = gpu_sinogram(torch, g, 40, 2000, 0.005)
    x = g.new_image()
    g.solve_cgls(b, x=x, tol=1e-3)          # warm-up
    torch.cuda.synchronize()
    reco.timing_reset()
    reco.timing_enable(True)
    t0 = time.perf_counter()
    reps = 2
    infos = [g.solve_cgls(b, x=x, tol=1e-3)[1] for _ in range(reps)]
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    kt = reco.timing_read()
    reco.timing_enable(False)
    it = sum(i["iters"] for i in infos)
    # A and A^T alone: plain projections of the reconstruction and of the data
    q = g.project(x)
    bt = g.backproject(b)
    torch.cuda.synchronize()
    reco.timing_reset()
    reco.timing_enable(True)
    for _ in range(5):
        g.project(x, out=q)
    for _ in range(5):
        g.backproject(b, out=bt)
    torch.cuda.synchronize()
    kt_alone = reco.timing_read()
    reco.timing_enable(False)
    a_ms = kt_alone["forward"][1] / kt_alone["forward"][0]
    at_ms = kt_alone["backward"][1] / kt_alone["backward"][0]
    fwd = nnz * it / (kt["forward"][1] * 1e-3) / 1e9
    bwd = nnz * (it + reps) / (kt["backward"][1] * 1e-3) / 1e9
    roof, _ = roofline_of(kt, {"forward": it, "backward": it + reps}, nnz, "ct2048")
    return roof, {
        "workload": "ct2048: 2048x2048 image, 2048 angles x 2897 bins, 40-ellipse phantom, "
                    "0.5% noise, 5-level WMG-CGLS to rel-res 1e-3",
        "recons_per_s": round(1.0 / t, 4), "ms_per_recon": round(t * 1e3, 2),
        "iters": infos[0]["iters"], "status": infos[0]["status"],
        "A_gupdates_per_s": round(fwd, 2), "AT_gupdates_per_s": round(bwd, 2),
        "A_frac_of_alu_peak": round(fwd / (PEAK_VALU_LANE_OPS / ALG_OPS_PER_UPDATE / 1e9), 4),
        "AT_frac_of_alu_peak": round(bwd / (PEAK_VALU_LANE_OPS / ALG_OPS_PER_UPDATE / 1e9), 4),
        # per launch that did work (launches issued after the device marked a
        # solve finished return at once and are not counted)
        "A_alone": {"ms": round(a_ms, 4), "gupdates_per_s": round(nnz / (a_ms * 1e-3) / 1e9, 2),
                    "frac_of_alu_peak": round(nnz / (a_ms * 1e-3) / 1e9
                                              / (PEAK_VALU_LANE_OPS / ALG_OPS_PER_UPDATE / 1e9), 4)},
        "AT_alone": {"ms": round(at_ms, 4), "gupdates_per_s": round(nnz / (at_ms * 1e-3) / 1e9, 2),
                     "frac_of_alu_peak": round(nnz / (at_ms * 1e-3) / 1e9
                                               / (PEAK_VALU_LANE_OPS / ALG_OPS_PER_UPDATE / 1e9), 4)},
        "kernel_avg_ms_working": {"forward": round(kt["forward"][1] / it, 4),
                                  "backward": round(kt["backward"][1] / (it + reps), 4)},
        "nnz": nnz, "setup_ms": round(setup_ms, 2),
    }


def copy_calibration(torch):
    """Calibration for the HBM byte counters: plain device copies of a known
    size (read COPY_BYTES, write COPY_BYTES) in the same profiled process."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def profile_ct2048(reco, torch, args):
    """The 2048^2 reconstruction alone (for rocprofv3): geometry set-up, then
    warm-up and timed WMG-CGLS solves of one resident sinogram, then the copy
    calibration."""
    g = reco.Geometry(2048, 2048, 2897, 5, reco.F32)
    b = gpu_sinogram(torch, g, 40, 2000, 0.005)
    x = g.new_image()
    for _ in range(args.warmup):
        g.solve_cgls(b, x=x, tol=1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = [g.solve_cgls(b, x=x, tol=1e-3)[1]["iters"] for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    copy_calibration(torch)
    print(json.dumps({"workload": "ct2048", "steps": args.steps, "iters": iters,
                      "seconds": elapsed, "copy_bytes": COPY_BYTES}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(independent reconstructions shard across GPUs with no communication; "
              "see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1310_0956_amd as reco

    torch.cuda.set_device(0)
    if args.profile_only and args.profile_workload == "ct2048":
        profile_ct2048(reco, torch, args)
        return
    w = WORKLOAD
    t0 = time.perf_counter()
    g = reco.Geometry(w["n"], w["m"], w["nb"], w["levels"], reco.F32)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    nnz = g.count_nnz()
    sinos = make_inputs(reco, torch, g, 4)
    x = g.new_image()

    def step(i):
        _, info = g.solve_cgls(sinos[i % len(sinos)], x=x, tol=w["tol"], max_iter=1000)
        return info

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    lat = []
    iters = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        info = step(i)
        lat.append((time.perf_counter() - s0) * 1e3)
        iters.append(info["iters"])
        assert info["status"] == "ok", info
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if args.profile_only:
        copy_calibration(torch)
        print(json.dumps({"steps": args.steps, "seconds": elapsed, "copy_bytes": COPY_BYTES}))
        return

    # Same steps again with per-kernel HIP-event timing on the launch stream.
    reco.timing_reset()
    reco.timing_enable(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    kt = reco.timing_read()
    reco.timing_enable(False)
    work_iters = sum(iters)
    # Launches that did work: the forward projector runs once per iteration,
    # the backprojector once per iteration plus once at the start of a solve.
    # A launch issued after the device marked the solve finished returns at
    # once; its (short) duration still counts in the totals below.
    working = {"forward": work_iters, "backward": work_iters + args.steps}
    avg_ms = {k: (ms / n if n else 0.0) for k, (n, ms) in kt.items()}
    roofline, gups = roofline_of(kt, working, nnz, "ct512")
    N, M = w["n"] ** 2, w["m"] * w["nb"]
    spmv_bytes = 8.0 * nnz + 4.0 * (N + M)
    result = {
        "metric": "WMG-CGLS recons/s at rel-res 1e-3; A/AT Gupdates/s; p50/p99 latency",
        "value": round(args.steps / elapsed, 3),
        "unit": "recons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "ct512: 512x512 image, 360 angles x 725 bins, 20-ellipse phantom, "
                        "1% Gaussian noise, 3-level WMG-CGLS to rel-res 1e-3",
            "image_side": w["n"], "angles": w["m"], "bins": w["nb"], "wmg_levels": w["levels"],
            "tol": w["tol"], "parallelism": "single GPU",
        },
        "iters_per_recon": sorted(set(iters)),
        "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
        "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
        "setup_ms": round(setup_ms, 3),
        "A_gupdates_per_s": round(gups.get("forward", 0.0), 3),
        "AT_gupdates_per_s": round(gups.get("backward", 0.0), 3),
        "A_spmv_equiv_GBs": round(spmv_bytes * gups.get("forward", 0.0) / nnz, 1),
        "kernel_avg_ms": {k: round(v, 5) for k, v in avg_ms.items()},
        "roofline": roofline,
    }
    if not args.no_solvers:
        result["solvers_ct512"] = solvers_leg(reco, torch, g, sinos)
        result["solvers_ct512_joseph"] = joseph_leg(reco, torch)
    if args.batch > 0:
        # the same workload, 8 reconstructions per batched solve (the headline
        # value above is one reconstruction at a time)
        xs8 = [g.new_image() for _ in range(8)]
        bs8 = [sinos[i % len(sinos)] for i in range(8)]
        reco.solve_batch([g] * 8, bs8, xs8, tol=w["tol"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            infos8 = reco.solve_batch([g] * 8, bs8, xs8, tol=w["tol"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        result["ct512_batched8"] = {"recons_per_s": round(8 / dt, 3),
                                    "ms_per_batch": round(dt * 1e3, 3),
                                    "all_ok": all(i["status"] == "ok" for i in infos8)}
    if args.batch > 0:
        result["batch"] = batch_leg(reco, torch, args.batch)
    if args.serve > 0:
        result["serving"] = serve_leg(reco, torch, args)
    if not args.no_ct2048:
        progress("2048^2 reconstruction")
        result["roofline_ct2048"], result["ct2048"] = ct2048_leg(reco, torch)
    if not args.no_tiny64:
        gc.collect()
        torch.cuda.synchronize()
        result["tiny64_f64"] = tiny64_leg(reco, torch)
    if not args.no_semiconv:
        progress("semi-convergence 160^2")
        result["semiconv160"] = semiconv_leg(reco, torch)
    if not args.no_cpu_baseline:
        solved, t_sum, cpu_iters, W = cpu_baseline(args)
        threads = min(16, os.cpu_count() or 1)
        matvec = cpu_matvec(W, threads)
        del W
        result["cpu_baseline"] = {
            "value": round(solved / t_sum, 5),
            "unit": "recons/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"{solved} whole float64 oracle WMG-CGLS reconstructions of the same "
                      f"512^2 workload (scipy CSR matrix, single thread) to rel-res 1e-3 in "
                      f"{t_sum:.2f} s, {cpu_iters} iterations; matrix assembly and packet "
                      f"diagonal excluded as setup",
            "host": host_info(),
            "matvec_ct512": matvec,
            "tiny64_oracle": cpu_config0(),
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
