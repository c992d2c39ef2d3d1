"""Benchmark: fine-grid Mdof/s of the level-dependent multigrid-preconditioned
GMRES(20) solve to relative residual 1e-6 on one MI355X.

Workload (one step = one full solve of the batch): 2D 1023 x 1023 interior
grid (h = 1/1024), heterogeneous medium k = k0 (1 + 0.3 g) with g a seeded
smooth Gaussian random field (correlation length 0.1, clipped to [-1, 1]) and
max k h = 0.625, ECS absorbing layer of 32 cells on every side, 8 unit point
sources at seeded nodes of the physical region, complex128, V(1,1) cycles with
omega-Jacobi (omega = 2/3), full weighting, bilinear interpolation, shifts
sigma_l = exp(i l pi / (6 L)), 3 x 3 coarsest direct solve, one cycle from a
zero guess per GMRES step.  Inputs are resident in device memory before the
timed region; set-up of the hierarchy is timed separately.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Besides the metric it carries the roofline figure of
the dominant kernel (algorithmic bytes over HIP-event time of its launches in
the timed region) and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-grid Mdof/s to rel. residual 1e-6 (FP64 vs mixed/batched); %HBM peak"
HBM_PEAK_GBS = 8000.0
N_GRID = 1023
NRHS = 8
RTOL = 1e-6
RESTART = 20
MAXIT = 20000          # GMRES steps per solve before it is reported as not converged
FINE_CLASSES = ["smooth_restrict_fine", "prolong_smooth_fine", "residual", "matvec_dot",
                "update_dot", "update_norm", "combine"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1211_4752_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel_class, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this kernel and workload, when it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.md" % (kernel_class, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"sources_sha256_16\s*=\s*([0-9a-f]+)", text)
    m_tr = re.search(r"traffic_bytes_per_launch\s*=\s*([0-9.eE+]+)", text)
    if not m_sha or not m_tr or m_sha.group(1) != sources_sha():
        return None
    return float(m_tr.group(1))


def cpu_baseline(wl, gpu_iters, sample_iters=6):
    """The oracle as it stands, one thread, on a bounded sample: GMRES(20)
    steps of right-hand side 0 of the same workload, extrapolated to the
    number of steps the solve needs."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import cycle as C
    from oracle import helmholtz as H
    from oracle import krylov as K
    with threadpool_limits(limits=1):
        prob = H.Problem(wl.n, wl.h, wl.k2, (wl.ecs,) * 2, (wl.ecs,) * 2, wl.ecs_angle)
        levels = H.build_hierarchy(prob)
        vc = C.VCycle(levels)
        f = wl.f[0].ravel()
        t0 = time.perf_counter()
        K.gmres(levels[0].A, vc.precondition, f, rtol=0.0, restart=RESTART, maxit=sample_iters)
        dt = time.perf_counter() - t0
    per_iter = dt / sample_iters
    est = per_iter * gpu_iters
    dofs = N_GRID * N_GRID
    return {
        "value": dofs / est / 1e6,
        "unit": "Mdof/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("%d GMRES(20) steps (one V(1,1) cycle + MGS Arnoldi each) of rhs 0 on the %dx%d "
                   "workload in %.1f s, single-threaded NumPy/SciPy; extrapolated to the %d steps the "
                   "GPU solve of that rhs needed" % (sample_iters, N_GRID, N_GRID, dt, gpu_iters)),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB four times (counter calibration)")
    ap.add_argument("--maxit", type=int, default=MAXIT,
                    help="cap on GMRES steps per solve (a capped solve is reported as not converged)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the batch of "
              "right-hand sides would shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1211_4752_amd import mg, workloads as W

    dev = torch.device("cuda:0")
    if args.copy_probe:
        # 2^27 float64 = 1 GiB read and 1 GiB written per copy
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read_per_copy": 1 << 30, "copies": 4}), flush=True)
        return
    wl = W.heterogeneous_2d(N_GRID, NRHS)
    k2 = torch.tensor(wl.k2, dtype=torch.float64, device=dev)
    f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=NRHS)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    u = s.empty()
    # load the code objects outside the timed region
    s.solve(u, f, mode="gmres", rtol=RTOL, maxit=2, restart=RESTART)
    for w in range(args.warmup):
        u.zero_()
        s.solve(u, f, mode="gmres", rtol=RTOL, maxit=args.maxit, restart=RESTART)
        log("warmup step %d done" % w)

    torch.cuda.synchronize()
    s.profile(True)
    statuses, iters = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        u.zero_()
        st, its, hists = s.solve(u, f, mode="gmres", rtol=RTOL, maxit=args.maxit, restart=RESTART)
        statuses.append(st)
        iters.append(its)
        log("step %d: %s, GMRES steps per rhs %s" % (k, st, its))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)

    dofs = N_GRID * N_GRID * NRHS
    value = dofs * args.steps / elapsed / 1e6
    # dominant fine-grid kernel of the timed region
    dom = max(FINE_CLASSES, key=lambda c: prof[c][0])
    ms, cnt, by = prof[dom]
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    workload = "grf2d_%d_x%d" % (N_GRID, NRHS)
    traffic = committed_traffic(dom, workload)
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": dom,
        "avg_launch_us": round(1e3 * ms / max(cnt, 1), 2),
        "algorithmic_bytes_per_launch": round(by / max(cnt, 1)),
        "launches": cnt,
    }
    kernels = {c: {"ms": round(v[0], 2), "launches": v[1],
                   "GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 and v[2] > 0 else None}
               for c, v in prof.items() if v[1]}

    # true residual check of the result with the library's own operator
    r = s.apply(u)
    true_res = [float(((f[i] - r[i]).abs().pow(2).sum().sqrt() / f[i].abs().pow(2).sum().sqrt()).item())
                for i in range(NRHS)]

    extra = {"setup_s": round(setup_s, 3), "status": statuses[-1], "gmres_steps": iters[-1],
             "true_rel_residual_max": max(true_res), "kernels": kernels}
    if not args.no_extras:
        # standalone level-dependent multigrid on the same batch (Sec. 4.1 LVL-MG)
        u.zero_()
        t1 = time.perf_counter()
        st, its, hists = s.solve(u, f, mode="standalone", rtol=RTOL, maxit=2000)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t1
        extra["standalone"] = {"status": st, "cycles": its, "seconds": round(dts, 3),
                               "last_ratio": [float(h[-1]) for h in hists]}
        log("standalone:", st, its)
        # mixed precision: complex64 cycle inside FP64 GMRES
        sm = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max,
                       nrhs=NRHS, precision="mixed")
        u.zero_()
        sm.solve(u, f, mode="gmres", rtol=RTOL, maxit=2, restart=RESTART)
        u.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, its, hists = sm.solve(u, f, mode="gmres", rtol=RTOL, maxit=args.maxit, restart=RESTART)
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t1
        extra["mixed"] = {"status": st, "gmres_steps": its, "Mdof_per_s": round(dofs / dtm / 1e6, 3)}
        log("mixed:", st, its)
        sm.close()
    s.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, iters[-1][0])

    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "Mdof/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "grid": "%dx%d" % (N_GRID, N_GRID), "h": "1/1024", "nrhs": NRHS,
                   "mode": "gmres(%d), one V(1,1) per step" % RESTART, "rtol": RTOL, "ecs_cells": wl.ecs,
                   "kh_max": 0.625, "theta_max": "pi/6", "omega": "2/3", "levels": 9, "precision": "c128"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
