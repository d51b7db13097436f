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
float64 oracle timed on a bounded sample on the host.
"""
import argparse
import hashlib
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3,
                    help="oracle iterations timed for the CPU baseline sample")
    ap.add_argument("--profile-only", action="store_true",
                    help="only run the timed steps (for rocprofv3)")
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


def source_hash(name):
    p = os.path.join(ROOT, "paper_1310_0956_amd", "csrc", name)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_for(kernel_file, per_launch_default=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source (else None)."""
    p = os.path.join(ROOT, "profiles", "traffic_ct512.json")
    if not os.path.exists(p):
        return per_launch_default
    d = json.load(open(p))
    ent = d.get(kernel_file)
    if not ent or ent.get("source_sha256_16") != source_hash(kernel_file):
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(args):
    """Oracle WMG-CGLS on the host, a bounded sample of the same workload."""
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
    x = inputs.ellipse_phantom(w["n"], w["ellipses"], w["seed"])
    b = W @ x.ravel()
    b = b + w["noise"] * np.abs(b).max() * inputs.standard_normal(b.size, w["seed"] + 500000)
    b = b.astype(np.float32).astype(np.float64)
    M = lambda v: wmg.apply_additive_diag(v, d, L)  # noqa: E731
    t0 = time.perf_counter()
    solvers.pcgls(W, b, fixed_iters=0, precond=M)      # initial W^T b and M^-1
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    solvers.pcgls(W, b, fixed_iters=args.cpu_iters, precond=M)
    t_k = time.perf_counter() - t0
    per_iter = max((t_k - t_init) / args.cpu_iters, 1e-9)
    return W.nnz, t_init, per_iter


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
        print(json.dumps({"steps": args.steps, "seconds": elapsed}))
        return

    # Same steps again with per-kernel HIP-event timing on the launch stream.
    reco.timing_reset()
    reco.timing_enable(True)
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    kt = reco.timing_read()
    reco.timing_enable(False)
    avg_ms = {k: (ms / n if n else 0.0) for k, (n, ms) in kt.items()}
    dom = "forward" if kt["forward"][1] >= kt["backward"][1] else "backward"
    # the solver launches the projector once per iteration on the current direction
    gups = {k: nnz / (avg_ms[k] * 1e-3) / 1e9 for k in ("forward", "backward") if avg_ms[k] > 0}
    peak = {k: PEAK_VALU_LANE_OPS / ALG_OPS_PER_UPDATE / 1e9 for k in ("forward", "backward")}
    N, M = w["n"] ** 2, w["m"] * w["nb"]
    spmv_bytes = 8.0 * nnz + 4.0 * (N + M)
    src = {"forward": "project.hip", "backward": "backproject.hip"}[dom]
    roofline = {
        "bound": "alu",
        "kernel": dom,
        "achieved": round(gups[dom], 3),
        "peak": round(peak[dom], 3),
        "unit": "Gupdate/s",
        "frac": round(gups[dom] / peak[dom], 4),
        "traffic": traffic_for(src),
        "avg_launch_ms": round(avg_ms[dom], 5),
        "launches": kt[dom][0],
        "updates_per_launch": nnz,
        "alg_valu_ops_per_update": ALG_OPS_PER_UPDATE,
    }
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
        "A_spmv_equiv_GBs": round(spmv_bytes / (avg_ms["forward"] * 1e-3) / 1e9, 1) if avg_ms["forward"] else None,
        "kernel_avg_ms": {k: round(v, 5) for k, v in avg_ms.items()},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        nnz_cpu, t_init, per_iter = cpu_baseline(args)
        k = float(np.mean(iters))
        t_recon = t_init + k * per_iter
        result["cpu_baseline"] = {
            "value": round(1.0 / t_recon, 5),
            "unit": "recons/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"float64 scipy-CSR oracle, WMG-CGLS on the same 512^2 workload: initial "
                      f"step + {args.cpu_iters} iterations timed ({t_init:.2f} s + "
                      f"{per_iter:.3f} s/iter), scaled to the GPU's {k:.1f} iterations per "
                      f"reconstruction; matrix assembly and packet diagonal excluded as setup",
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
