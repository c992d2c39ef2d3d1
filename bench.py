"""Benchmark: fine-grid Mdof/s of the level-dependent multigrid-preconditioned
(F)GMRES(20) solve to relative residual 1e-6 on one MI355X.

Workload (one step = one full solve of the batch): 2D 1023 x 1023 interior
grid (h = 1/1024), heterogeneous medium k = k0 (1 + 0.3 g) with g a seeded
smooth Gaussian random field (correlation length 0.1, clipped to [-1, 1]) and
max k h = 0.625, ECS absorbing layer of 32 cells on every side, 8 unit point
sources at seeded nodes of the physical region, complex128, V(1,1) cycles with
the GMRES(3) smoother (the smoother of every experiment in the paper; with
it the cycle is nonlinear and the outer method is flexible GMRES(20)), full
weighting, bilinear interpolation, shifts sigma_l = exp(i l pi / (6 L)),
3 x 3 coarsest direct solve, one cycle from a zero guess per outer step.
The omega-Jacobi (omega = 2/3) form of the same cycle does not reach 1e-6
on this workload; it is run for a capped number of steps and reported in
"extra".  Inputs are resident in device memory before the timed region;
set-up of the hierarchy is timed separately.

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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-grid Mdof/s to rel. residual 1e-6 (FP64 vs mixed/batched); %HBM peak"
HBM_PEAK_GBS = 8000.0
N_GRID = 1023
NRHS = 8
RTOL = 1e-6
RESTART = 20
MAXIT = 5000           # outer steps per solve before it is reported as not converged
JACOBI_MAXIT = 2000    # capped omega-Jacobi GMRES(20) run reported in "extra"
SMOOTHER = "gmres3"
FINE_CLASSES = ["smooth_restrict_fine", "prolong_smooth_fine", "residual", "matvec_dot",
                "update_dot", "update_norm", "combine", "smooth_power_fine", "smooth_gram_fine",
                "smooth_gram_post_fine"]


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
    """The oracle as it stands, one thread, on a bounded sample: FGMRES(20)
    steps with the GMRES(3)-smoothed cycle of right-hand side 0 of the same
    workload, extrapolated to the number of steps the solve needs."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    from oracle import cycle as C
    from oracle import helmholtz as H
    from oracle import krylov as K
    with threadpool_limits(limits=1):
        prob = H.Problem(wl.n, wl.h, wl.k2, (wl.ecs,) * 2, (wl.ecs,) * 2, wl.ecs_angle)
        levels = H.build_hierarchy(prob)
        vc = C.VCycle(levels, smoother="gmres")
        f = wl.f[0].ravel()
        t0 = time.perf_counter()
        K.gmres(levels[0].A, vc.precondition, f, rtol=0.0, restart=RESTART, maxit=sample_iters, flexible=True)
        dt = time.perf_counter() - t0
    per_iter = dt / sample_iters
    est = per_iter * gpu_iters
    dofs = N_GRID * N_GRID
    return {
        "value": dofs / est / 1e6,
        "unit": "Mdof/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("%d FGMRES(20) steps (one GMRES(3)-smoothed V(1,1) cycle + MGS Arnoldi each) of rhs 0 "
                   "on the %dx%d workload in %.1f s, single-threaded NumPy/SciPy; extrapolated to the %d "
                   "steps the GPU solve of that rhs needed" % (sample_iters, N_GRID, N_GRID, dt, gpu_iters)),
    }


def batched(mg, W, torch, dev):
    """64 sources on one 511^2 GRF medium plus 24 uneven constant-kh grids
    (127^2 .. 1023^2), mixed precision, GMRES(3) smoother, one batch: every
    launch of a step covers all of them, the coarse part of each cycle is a
    replayed HIP graph.  Whole-batch fine-grid Mdof/s to 1e-6."""
    wls = W.batched_2d()
    ss = [mg.Solver(w.n, w.h, torch.tensor(w.k2, dtype=torch.float64, device=dev), ecs=w.ecs,
                    ecs_angle=w.ecs_angle, theta_max=w.theta_max, nrhs=w.f.shape[0], precision="mixed",
                    smoother=SMOOTHER) for w in wls]
    fs = [torch.tensor(w.f, dtype=torch.complex128, device=dev) for w in wls]
    us = [s.empty() for s in ss]
    b = mg.Batch(ss)
    b.solve(us, fs, mode="gmres", rtol=RTOL, maxit=2, restart=RESTART)
    for u in us:
        u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, its, hists = b.solve(us, fs, mode="gmres", rtol=RTOL, maxit=MAXIT, restart=RESTART)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dofs = sum(int(w.f.shape[0]) * int(np.prod(w.n)) for w in wls)
    b.close()
    for s in ss:
        s.close()
    log("batched:", st, "%.3f s" % dt)
    return {"status": st, "problems": len(wls), "rhs": sum(w.f.shape[0] for w in wls), "dofs": dofs,
            "seconds": round(dt, 3), "Mdof_per_s": round(dofs / dt / 1e6, 3),
            "max_steps": max(max(r) for r in its), "precision": "mixed"}


# Table 5 of the paper: standalone level-dependent V(1,1) cycles with GMRES(3)
# smoothing, constant k = 30 on n = 128 points, rtol 1e-7, d-theta = theta_max / 7.
TABLE5_THETA_OVER_PI = [1 / 15, 1 / 12, 1 / 10, 1 / 8, 1 / 6, 1 / 5, 1 / 4]
TABLE5_CYCLES = [27, 25, 23, 22, 22, 25, 28]


def theta_sweep(mg, W, torch, dev):
    """The theta_max sweep on the same k h and number of levels (255^2 grid,
    64-cell layers inside it around the 128-point physical region)."""
    wl = W.constant_2d(255, 30.0 / 128, ecs=64)
    k2 = torch.tensor(wl.k2, dtype=torch.float64, device=dev)
    f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
    cycles = []
    for tm in TABLE5_THETA_OVER_PI:
        s = mg.Solver(wl.n, wl.h, k2, ecs=64, theta_max=tm * math.pi, nrhs=1, smoother=SMOOTHER)
        u = s.empty()
        st, its, _ = s.solve(u, f, mode="standalone", rtol=1e-7, maxit=200)
        cycles.append(its[0] if st == "converged" else None)
        s.close()
    log("theta sweep:", cycles)
    return {"theta_max_over_pi": [round(t, 4) for t in TABLE5_THETA_OVER_PI], "gpu_cycles": cycles,
            "paper_cycles": TABLE5_CYCLES, "grid": "255x255, ECS 64, kh 30/128, 7 levels"}


# LVL-MG rows of Tables 6, 7 and 8 (Sec. 4.2 wedge in 2D and 3D, Sec. 4.3
# ionization): standalone V(1,1) cycles with GMRES(3) smoothing, rtol 1e-7.
TABLE6_CYCLES = [30, 47, 72, 83, 101]
TABLE7_CYCLES = [38, 46, 50, 58, 71]
TABLE8_CYCLES = [44, 83, 208, 149, 289]
# MG-FGMRES(10) rows: fixed-shift CSG cycles preconditioning FGMRES(10)
TABLE6_FGMRES10 = [32, 58, 85, 107, 133]
TABLE7_FGMRES10 = [35, 40, 47, 55, 62]
TABLE8_FGMRES10 = [66, 140, 245, 250, 393]


def paper_models(mg, W, torch, dev):
    """Every case of the three tables on the paper's physical grids (plus
    layers of a quarter of the x cell count outside the physical region):
    LVL-MG, and the MG-FGMRES(10) comparator (sigma = 1 + 0.5 i on every
    level, FGMRES restarted every 10 steps)."""
    rows = {}
    cases = ([("wedge_2d_table6", W.wedge_2d(fz, c), p, q)
              for (fz, c), p, q in zip(W.WEDGE_2D_TABLE6, TABLE6_CYCLES, TABLE6_FGMRES10)]
             + [("wedge_3d_table7", W.wedge_3d(fz), p, q)
                for fz, p, q in zip(W.WEDGE_3D_TABLE7, TABLE7_CYCLES, TABLE7_FGMRES10)]
             + [("ionization_table8", W.ionization_2d(k0, c), p, q)
                for (k0, c), p, q in zip(W.IONIZATION_TABLE8, TABLE8_CYCLES, TABLE8_FGMRES10)])
    for table, wl, paper, paper_fg in cases:
        k2 = torch.tensor(wl.k2, dtype=torch.float64, device=dev)
        f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
        s = mg.Solver(wl.n, wl.h, k2, ecs=(wl.ecs_lo, wl.ecs_hi), ecs_angle=wl.ecs_angle,
                      theta_max=wl.theta_max, nrhs=1, smoother=SMOOTHER)
        u = s.empty()
        s.solve(u, f, mode="standalone", rtol=1e-7, maxit=2)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, its, _ = s.solve(u, f, mode="standalone", rtol=1e-7, maxit=1000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nlev = s.num_levels
        s.close()
        sc = mg.Solver(wl.n, wl.h, k2, ecs=(wl.ecs_lo, wl.ecs_hi), ecs_angle=wl.ecs_angle,
                       sigma=[1 + 0.5j] * nlev, nrhs=1, smoother=SMOOTHER)
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stc, itc, _ = sc.solve(u, f, mode="gmres", rtol=1e-7, maxit=2000, restart=10)
        torch.cuda.synchronize()
        dtc = time.perf_counter() - t0
        sc.close()
        rows.setdefault(table, []).append({"case": wl.name, "grid": "x".join(map(str, wl.n)),
                                           "levels": nlev, "status": st, "gpu_cycles": its[0],
                                           "paper_cycles": paper, "seconds": round(dt, 4),
                                           "mg_fgmres10": {"status": stc, "gpu_steps": itc[0],
                                                           "paper_steps": paper_fg, "seconds": round(dtc, 4)}})
        log("%s: LVL-MG %s %d cycles (paper %d), %.3f s; MG-FGMRES(10) %s %d (paper %d), %.3f s"
            % (wl.name, st, its[0], paper, dt, stc, itc[0], paper_fg, dtc))
    return rows


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
    s = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=NRHS,
                  smoother=SMOOTHER)
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
        def timed(solver, uu, mode, maxit):
            uu.zero_()
            solver.solve(uu, f, mode=mode, rtol=RTOL, maxit=2, restart=RESTART)
            uu.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, its, hists = solver.solve(uu, f, mode=mode, rtol=RTOL, maxit=maxit, restart=RESTART)
            torch.cuda.synchronize()
            return st, its, hists, time.perf_counter() - t1

        # standalone level-dependent multigrid on the same batch (Sec. 4.1 LVL-MG)
        st, its, hists, dts = timed(s, u, "standalone", 300)
        extra["standalone"] = {"status": st, "cycles": its, "seconds": round(dts, 3),
                               "last_ratio": [float(h[-1]) for h in hists]}
        log("standalone:", st, its)
        # mixed precision: complex64 cycle inside FP64 FGMRES
        sm = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max,
                       nrhs=NRHS, precision="mixed", smoother=SMOOTHER)
        st, its, hists, dtm = timed(sm, u, "gmres", args.maxit)
        extra["mixed"] = {"status": st, "gmres_steps": its, "Mdof_per_s": round(dofs / dtm / 1e6, 3)}
        log("mixed:", st, its)
        sm.close()
        # the omega-Jacobi cycle, right-preconditioned GMRES(20), capped
        sj = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max,
                       nrhs=NRHS, smoother="jacobi")
        st, its, hists, dtj = timed(sj, u, "gmres", JACOBI_MAXIT)
        extra["omega_jacobi_gmres"] = {"status": st, "gmres_steps": its, "seconds": round(dtj, 3),
                                       "ms_per_step": round(1e3 * dtj / max(its), 3),
                                       "last_ratio": [float(h[-1]) for h in hists]}
        log("omega-jacobi:", st, its)
        sj.close()
        # comparator of Table 3 (MG-FGMRES): the cycle on -Delta - (1 + 0.5 i) k^2
        # on every level, preconditioning the unshifted problem
        L = s.num_levels
        sc = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, sigma=[1 + 0.5j] * L, nrhs=NRHS,
                       smoother=SMOOTHER)
        st, its, hists, dtc = timed(sc, u, "gmres", 2000)
        extra["fixed_shift_csl"] = {"sigma": "1+0.5i on every level", "status": st, "gmres_steps": its,
                                    "seconds": round(dtc, 3), "Mdof_per_s": round(dofs / dtc / 1e6, 3)}
        log("fixed-shift comparator:", st, its)
        sc.close()
        extra["batched"] = batched(mg, W, torch, dev)
        extra["theta_sweep_table5"] = theta_sweep(mg, W, torch, dev)
        extra["paper_models"] = paper_models(mg, W, torch, dev)
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
                   "mode": "fgmres(%d), one V(1,1) per step" % RESTART, "smoother": "gmres(3)", "rtol": RTOL,
                   "ecs_cells": wl.ecs, "kh_max": 0.625, "theta_max": "pi/6", "levels": 9,
                   "precision": "c128"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
