"""Benchmark: fine-grid Mdof/s of the level-dependent multigrid-preconditioned
(F)GMRES(20) solve to relative residual 1e-6 on one MI355X.

Headline workload (one step = one full solve of the batch): 2D 1023 x 1023
interior grid (h = 1/1024), heterogeneous medium k = k0 (1 + 0.3 g) with g a
seeded smooth Gaussian random field (correlation length 0.1, clipped to
[-1, 1]) and max k h = 0.625, ECS absorbing layer of 32 cells on every side,
8 unit point sources at seeded nodes of the physical region, complex128,
V(1,1) cycles with the GMRES(3) smoother (the smoother of every experiment in
the paper; with it the cycle is nonlinear and the outer method is flexible
GMRES(20)), full weighting, bilinear interpolation, shifts
sigma_l = exp(i l pi / (6 L)), 3 x 3 coarsest direct solve, one cycle from a
zero guess per outer step.  Inputs are resident in device memory before the
timed region; set-up of the hierarchy is timed separately.  Every restart
cycle runs as a replayed HIP graph.  Kernel durations come from HIP events
around every launch of the same solves run again launch by launch in this
process (events captured inside a HIP graph cannot be timed).

Errors against FP64: a solve to a relative residual of 1e-6 is itself only
about 1e-5 from the exact discrete solution, in any precision, so each
mixed-precision result is also solved to 1e-9 and compared with the
complex128 solution to 1e-12 (the mixed-precision bar is an error of 1e-6).

Extras: the omega-Jacobi form of the same cycle (it does not reach 1e-6 on
this 2D workload: reported capped), mixed precision with its error against
the FP64 solution, the 3D 255^3 workload (both smoothers, both precisions),
the batched workload (64 sources on 511^2 plus 24 uneven grids, one batch)
with its error against FP64, adjoint gradients per second on 511^2 with 16
shots, the comparator of the paper's Table 3, Table 5's theta sweep and the
models of Tables 6-8.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --only c3_jacobi|c3_gmres3|c4|c5|headline   (one workload, for profilers)

Prints one JSON line.
"""

from __future__ import annotations

import argparse
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
JACOBI_MAXIT = 2000    # capped omega-Jacobi GMRES(20) run on the 2D workload
SMOOTHER = "gmres3"
WORKLOAD = "grf2d_%d_x%d" % (N_GRID, NRHS)
CYCLE_CLASSES = ["smooth_restrict_fine", "prolong_smooth_fine", "coarse_levels", "coarsest_solve",
                 "smooth_gram_fine", "smooth_gram_post_fine", "smooth_power_fine"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def committed_traffic(kernel_class, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary of this workload, with the algorithmic bytes per launch
    of the same counter run (so that their ratio is meaningful)."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.md" % (kernel_class, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_tr = re.search(r"traffic_bytes_per_launch\s*=\s*([0-9.eE+]+)", text)
    m_al = re.search(r"algorithmic_bytes_per_launch\s*=\s*([0-9.eE+]+)", text)
    if not m_tr:
        return None
    out = {"traffic_bytes_per_launch": float(m_tr.group(1))}
    if m_al:
        out["algorithmic_bytes_per_launch"] = float(m_al.group(1))
        out["ratio"] = round(out["traffic_bytes_per_launch"] / out["algorithmic_bytes_per_launch"], 3)
    return out


def hbm_probe(torch, dev):
    """Bandwidth that plain torch kernels reach on this GPU (1 GiB float64
    arrays, HIP events, best of 5): a copy (read + write), a sum (read) and a
    fill (write).  Context for the roofline fractions, which use the
    published 8 TB/s."""
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    nbytes = float(1 << 30)
    out = {}
    for name, fn, moved in (("copy", lambda: b.copy_(a), 2 * nbytes), ("read", lambda: a.sum(), nbytes),
                            ("write", lambda: b.fill_(2.0), nbytes)):
        fn()
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[name + "_GBps"] = round(moved / (best * 1e-3) / 1e9, 1)
    del a, b
    return out


def shapes(s):
    """Tile-shape id in force on each level (ids 3-5: plane sweeps)."""
    return [s.tile_shape(l) for l in range(s.num_levels)]


def per_class(prof):
    """{class: ms, launches, avg launch us, GB/s of algorithmic bytes, frac}."""
    out = {}
    for c, (ms, cnt, by) in prof.items():
        if not cnt:
            continue
        gbs = by / (ms * 1e-3) / 1e9 if ms > 0 and by > 0 else None
        out[c] = {"ms": round(ms, 2), "launches": cnt, "avg_launch_us": round(1e3 * ms / cnt, 2),
                  "algorithmic_bytes_per_launch": round(by / cnt) if by > 0 else None,
                  "GBps": round(gbs, 1) if gbs else None,
                  "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None}
    return out


def cycle_summary(prof):
    """Bytes and time of every cycle kernel (all levels) of a profiled run."""
    ms = sum(prof[c][0] for c in CYCLE_CLASSES if c in prof)
    by = sum(prof[c][2] for c in CYCLE_CLASSES if c in prof)
    gbs = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"ms": round(ms, 2), "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def rel_err(a, b):
    return float(((a - b).abs().pow(2).sum().sqrt() / b.abs().pow(2).sum().sqrt()).item())


def timed_solve(torch, s, u, f, mode, rtol, maxit, restart=RESTART, profile=False, graph_time=True):
    """Warm (records and captures the operations), then one timed solve
    (replayed graphs).  With profile, a further solve launched kernel by
    kernel under HIP events gives the per-class table; u keeps the timed
    solve's result.  graph_time=False (profiler runs): only the profiled
    solve, which is then the timed one."""
    u.zero_()
    s.solve(u, f, mode=mode, rtol=rtol, maxit=min(maxit, 2), restart=restart)
    u.zero_()
    torch.cuda.synchronize()
    if profile and not graph_time:
        s.profile(True)
        t0 = time.perf_counter()
        st, its, hists = s.solve(u, f, mode=mode, rtol=rtol, maxit=maxit, restart=restart)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = s.profile_read()
        s.profile(False)
        return st, its, hists, dt, prof
    t0 = time.perf_counter()
    st, its, hists = s.solve(u, f, mode=mode, rtol=rtol, maxit=maxit, restart=restart)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile:
        keep = u.clone()
        u.zero_()
        s.profile(True)
        s.solve(u, f, mode=mode, rtol=rtol, maxit=maxit, restart=restart)
        torch.cuda.synchronize()
        prof = s.profile_read()
        s.profile(False)
        u.copy_(keep)
        del keep
    return st, its, hists, dt, prof


# ---------------------------------------------------------------------------
# CPU baselines (the oracle as it stands)
# ---------------------------------------------------------------------------
def cpu_baseline(wl, gpu_iters, sample_iters=6):
    """The oracle, one thread, on a bounded sample: FGMRES(20) steps with the
    GMRES(3)-smoothed cycle of right-hand side 0 of the headline workload,
    extrapolated to the number of steps the GPU solve of that rhs needed."""
    from threadpoolctl import threadpool_limits
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
    est = dt / sample_iters * gpu_iters
    return {
        "value": N_GRID * N_GRID / est / 1e6, "unit": "Mdof/s", "cores": 1, "kind": "oracle",
        "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
        "sample": ("%d FGMRES(20) steps (one GMRES(3)-smoothed V(1,1) cycle + MGS Arnoldi each) of rhs 0 "
                   "on the %dx%d workload in %.1f s, single-threaded NumPy/SciPy (its elementwise work is "
                   "single-threaded), extrapolated to the %d steps the GPU solve of that rhs needed"
                   % (sample_iters, N_GRID, N_GRID, dt, gpu_iters)),
    }


def _oracle_steps(args):
    """Worker: oracle FGMRES steps on one right-hand side of a batch problem."""
    n, kind, idx, steps = args
    os.environ["OMP_NUM_THREADS"] = "1"
    from threadpoolctl import threadpool_limits
    from oracle import cycle as C
    from oracle import helmholtz as H
    from oracle import krylov as K
    from paper_1211_4752_amd import workloads as W
    with threadpool_limits(limits=1):
        wl = W.heterogeneous_2d(n, 64, source_seed=4) if kind == "grf" else W.uneven_batch()[idx]
        prob = H.Problem(wl.n, wl.h, wl.k2, (wl.ecs,) * 2, (wl.ecs,) * 2, wl.ecs_angle)
        vc = C.VCycle(H.build_hierarchy(prob), smoother="gmres")
        f = wl.f[idx if kind == "grf" else 0].ravel()
        A = H.operator(prob)
        t0 = time.perf_counter()
        K.gmres(A, vc.precondition, f, rtol=0.0, restart=RESTART, maxit=steps, flexible=True)
        return time.perf_counter() - t0


def cpu_baseline_batched(gpu_steps, workers=None, sample_steps=3):
    """The oracle over all host cores (one process per right-hand side of the
    511^2 GRF member, a bounded sample of FGMRES steps each), extrapolated to
    the steps the GPU batch needed per right-hand side; the uneven grids are
    counted at the rate of the 511^2 member."""
    import multiprocessing as mp
    workers = workers or min(os.cpu_count() or 1, 16)
    jobs = [(511, "grf", r, sample_steps) for r in range(workers)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        times = pool.map(_oracle_steps, jobs)
    wall = time.perf_counter() - t0
    per_step = float(np.mean(times)) / sample_steps
    # every process works on its own rhs: aggregate dof-steps per second
    rate = workers * 511 * 511 / per_step
    dofs_steps = sum(gpu_steps)
    return {"value": rate / gpu_steps_mean(gpu_steps) / 1e6, "unit": "Mdof/s", "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
            "sample": ("%d processes x %d FGMRES(20) steps of one 511^2 GRF source each (%.1f s wall, %.2f s "
                       "per step per process); rate extrapolated to the GPU batch's mean of %.0f steps per "
                       "right-hand side" % (workers, sample_steps, wall, per_step, gpu_steps_mean(gpu_steps))),
            "dof_steps_gpu": dofs_steps}


def gpu_steps_mean(steps):
    return float(np.mean(steps)) if len(steps) else 1.0


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def c3(mg, W, torch, dev, smoothers=("gmres3", "jacobi")):
    """3D 255^3, constant k h = 0.5, ECS 16, centre source: FGMRES/GMRES(20)
    to 1e-6 in complex128 and mixed; the mixed result's error against the
    FP64 solution of the same solver (complex128, solved to 1e-12)."""
    wl = W.constant_3d(255, 0.5, 16)
    k2 = torch.tensor(wl.k2, dtype=torch.float64, device=dev)
    f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
    dofs = int(np.prod(wl.n))
    out = {}
    for sm in smoothers:
        ref = None
        for prec in ("c128", "mixed"):
            s = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=1,
                          precision=prec, smoother=sm)
            u = s.empty()
            st, its, hists, dt, prof = timed_solve(torch, s, u, f, "gmres", RTOL, 3000, profile=True)
            row = {"status": st, "steps": its[0], "seconds": round(dt, 4), "Mdof_per_s": round(dofs / dt / 1e6, 3),
                   "ms_per_step": round(1e3 * dt / max(1, its[0]), 3), "cycle_kernels": cycle_summary(prof),
                   "shapes": shapes(s), "kernels": per_class(prof)}
            if prec == "c128":
                ref = s.empty()
                s.solve(ref, f, mode="gmres", rtol=1e-12, maxit=6000, restart=RESTART)
            row["error_at_rtol_1e-6_vs_fp64_1e-12"] = rel_err(u, ref)
            r = s.apply(u)
            row["true_rel_residual"] = rel_err(r, f)
            if prec == "mixed":
                u.zero_()
                st9, its9, _ = s.solve(u, f, mode="gmres", rtol=1e-9, maxit=6000, restart=RESTART)
                row["error_at_rtol_1e-9_vs_fp64_1e-12"] = rel_err(u, ref)
                row["rtol_1e-9"] = {"status": st9, "steps": its9[0]}
            out["%s_%s" % (sm, prec)] = row
            log("c3 %s %s: %s %d steps %.3f s %.2f Mdof/s" % (sm, prec, st, its[0], dt, dofs / dt / 1e6))
            s.close()
            del u
        del ref
    return out


def batched(mg, W, torch, dev, precision="mixed", profile=True):
    """64 sources on one 511^2 GRF medium plus 24 uneven constant-kh grids
    (127^2 .. 1023^2), GMRES(3) smoother, one batch: every launch covers all
    88 right-hand sides, each restart cycle of the whole batch is one graph.
    Whole-batch fine-grid Mdof/s to 1e-6; every result's error against the
    complex128 batch solved to 1e-12."""
    wls = W.batched_2d()
    mk = lambda prec: [mg.Solver(w.n, w.h, torch.tensor(w.k2, dtype=torch.float64, device=dev), ecs=w.ecs,
                                 ecs_angle=w.ecs_angle, theta_max=w.theta_max, nrhs=w.f.shape[0], precision=prec,
                                 smoother=SMOOTHER) for w in wls]
    fs = [torch.tensor(w.f, dtype=torch.complex128, device=dev) for w in wls]
    ss = mk(precision)
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
    prof = None
    if profile:
        # the kernel table: a further solve launched kernel by kernel with
        # HIP events (the timed solve above replays graphs)
        u_keep = [u.clone() for u in us]
        for u in us:
            u.zero_()
        ss[0].profile(True)
        b.solve(us, fs, mode="gmres", rtol=RTOL, maxit=MAXIT, restart=RESTART)
        torch.cuda.synchronize()
        prof = ss[0].profile_read()
        ss[0].profile(False)
        for u, v in zip(us, u_keep):
            u.copy_(v)
    dofs = sum(int(w.f.shape[0]) * int(np.prod(w.n)) for w in wls)
    u6 = [u.clone() for u in us]
    for u in us:
        u.zero_()
    st9, its9, _ = b.solve(us, fs, mode="gmres", rtol=1e-9, maxit=MAXIT, restart=RESTART)
    b.close()
    # FP64 reference: the same batch in complex128, to 1e-12
    rs = mk("c128")
    refs = [s.empty() for s in rs]
    rb = mg.Batch(rs)
    rb.solve(refs, fs, mode="gmres", rtol=1e-12, maxit=MAXIT, restart=RESTART)
    rb.close()
    errs, errs6 = [], []
    for u, v, r in zip(us, u6, refs):
        for i in range(u.shape[0]):
            errs.append(rel_err(u[i], r[i]))
            errs6.append(rel_err(v[i], r[i]))
    for s in ss + rs:
        s.close()
    steps = [x for row in its for x in row]
    log("batched:", st, "%.3f s" % dt)
    out = {"status": st, "problems": len(wls), "rhs": len(steps), "dofs": dofs, "seconds": round(dt, 3),
           "Mdof_per_s": round(dofs / dt / 1e6, 3), "max_steps": max(steps), "mean_steps": round(float(np.mean(steps)), 1),
           "precision": precision, "graph_launches": "one per restart cycle of the whole batch",
           "timing": "wall clock of one solve replaying the recorded graphs; kernel table from a further solve "
                     "launched kernel by kernel",
           "error_at_rtol_1e-6_vs_fp64_1e-12": {"max": max(errs6), "median": float(np.median(errs6))},
           "error_at_rtol_1e-9_vs_fp64_1e-12": {"max": max(errs), "median": float(np.median(errs)),
                                                "status": st9, "max_steps": max(x for row in its9 for x in row)},
           "errors_per_result_note": "every one of the 88 results compared; max and median shown"}
    if prof:
        out["kernels"] = per_class(prof)
        out["cycle_kernels"] = cycle_summary(prof)
    return out, [x for row in its for x in row]


def c5(mg, W, torch, dev, reps=2):
    """Adjoint gradients on 511^2 (GRF medium), 16 shots, 128 receivers on
    the row y = 0.9, L = 0.5 sum ||P u - d||^2 with data from a 5 % perturbed
    medium: one gradient = 16 forward and 16 adjoint (F)GMRES solves to 1e-10
    plus the pointwise dL/dk^2 pass.  Gradients per second (set-up excluded)."""
    n, nshots, nrec = 511, 16, 128
    ecs = (n + 1) // 32
    k2n = W.heterogeneous_k2(n, 2, seed=2)
    k2t = W.perturbed_k2(k2n, seed=7)
    nodes = W.source_nodes(n, 2, nshots, seed=6, lo=ecs, hi=n - 1 - ecs, max_y=int(0.8 * (n + 1)))
    f = torch.tensor(W.point_sources((n, n), nodes), dtype=torch.complex128, device=dev)
    rec = W.receiver_nodes(n, nrec, 460)
    idx = torch.tensor(rec[:, 1] * n + rec[:, 0], device=dev)
    h = 1.0 / (n + 1)
    st_true = mg.Solver((n, n), h, torch.tensor(k2t, dtype=torch.float64, device=dev), ecs=ecs, nrhs=nshots,
                        smoother=SMOOTHER)
    ut = st_true.empty()
    st_true.solve(ut, f, mode="gmres", rtol=1e-10, maxit=5000)
    d = ut.reshape(nshots, -1)[:, idx].clone()
    st_true.close()
    k2 = torch.tensor(k2n, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    s = mg.Solver((n, n), h, k2, ecs=ecs, nrhs=nshots, smoother=SMOOTHER)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    u, lam = s.empty(), s.empty()
    g = torch.zeros_like(k2)

    def gradient():
        u.zero_()
        lam.zero_()
        g.zero_()
        st, its, _ = s.solve(u, f, mode="gmres", rtol=1e-10, maxit=5000)
        r = torch.zeros_like(u).reshape(nshots, -1)
        r[:, idx] = u.reshape(nshots, -1)[:, idx] - d
        sta, itsa, _ = s.solve_adjoint(lam, r.reshape(u.shape).contiguous(), mode="gmres", rtol=1e-10, maxit=5000)
        s.grad_k2(u, lam, g)
        return st, sta, its, itsa

    gradient()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st, sta, its, itsa = gradient()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    s.close()
    log("c5: %.3f s per gradient" % dt)
    return {"gradients_per_s": round(1.0 / dt, 3), "seconds_per_gradient": round(dt, 4),
            "shot_gradients_per_s": round(nshots / dt, 2), "setup_s": round(setup, 3),
            "forward": {"status": st, "max_steps": max(its)}, "adjoint": {"status": sta, "max_steps": max(itsa)},
            "Mdof_per_s_forward_plus_adjoint": round(2 * nshots * n * n / dt / 1e6, 3)}


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
        st, its, _, dt, _ = timed_solve(torch, s, u, f, "standalone", 1e-7, 1000)
        nlev = s.num_levels
        s.close()
        sc = mg.Solver(wl.n, wl.h, k2, ecs=(wl.ecs_lo, wl.ecs_hi), ecs_angle=wl.ecs_angle,
                       sigma=[1 + 0.5j] * nlev, nrhs=1, smoother=SMOOTHER)
        stc, itc, _, dtc, _ = timed_solve(torch, sc, u, f, "gmres", 1e-7, 2000, restart=10)
        sc.close()
        rows.setdefault(table, []).append({"case": wl.name, "grid": "x".join(map(str, wl.n)),
                                           "levels": nlev, "status": st, "gpu_cycles": its[0],
                                           "paper_cycles": paper, "seconds": round(dt, 4),
                                           "mg_fgmres10": {"status": stc, "gpu_steps": itc[0],
                                                           "paper_steps": paper_fg, "seconds": round(dtc, 4)}})
        log("%s: LVL-MG %s %d cycles (paper %d), %.3f s; MG-FGMRES(10) %s %d (paper %d), %.3f s"
            % (wl.name, st, its[0], paper, dt, stc, itc[0], paper_fg, dtc))
    return rows


def force_shapes(s, arg):
    """--shapes a,b,c: set the tile shape of each level (so that separate
    profiler runs of one workload use the same kernels)."""
    if not arg:
        return
    for l, sh in enumerate(int(x) for x in arg.split(",")):
        if l < s.num_levels:
            s.tile_shape(l, sh)


def only(args, mg, W, torch, dev):
    """A single workload, for profiler runs: one solve after the warm-up."""
    res = {}
    if args.only == "headline":
        wl = W.heterogeneous_2d(N_GRID, NRHS)
        s = mg.Solver(wl.n, wl.h, torch.tensor(wl.k2, dtype=torch.float64, device=dev), ecs=wl.ecs,
                      ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=NRHS, smoother=SMOOTHER,
                      precision=args.precision)
        f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
        force_shapes(s, args.shapes)
        u = s.empty()
        st, its, _, dt, prof = timed_solve(torch, s, u, f, "gmres", RTOL, args.maxit, profile=True,
                                           graph_time=False)
        res = {"status": st, "steps": its, "seconds": dt, "shapes": shapes(s), "kernels": per_class(prof)}
    elif args.only.startswith("c3_") and args.light:
        wl = W.constant_3d(255, 0.5, 16)
        s = mg.Solver(wl.n, wl.h, torch.tensor(wl.k2, dtype=torch.float64, device=dev), ecs=wl.ecs,
                      ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=1, smoother=args.only[3:],
                      precision=args.precision)
        f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
        force_shapes(s, args.shapes)
        u = s.empty()
        st, its, _, dt, prof = timed_solve(torch, s, u, f, "gmres", RTOL, args.maxit, profile=True,
                                           graph_time=False)
        res = {"status": st, "steps": its, "seconds": dt, "shapes": shapes(s), "kernels": per_class(prof)}
    elif args.only.startswith("c3_"):
        res = c3(mg, W, torch, dev, smoothers=(args.only[3:],))
    elif args.only == "c4":
        res, _ = batched(mg, W, torch, dev, profile=False)
    elif args.only == "c4_jacobi_511":
        # the omega-Jacobi cycle on the 64-source 511^2 member
        wl = W.heterogeneous_2d(511, 64, source_seed=4)
        s = mg.Solver(wl.n, wl.h, torch.tensor(wl.k2, dtype=torch.float64, device=dev), ecs=wl.ecs,
                      ecs_angle=wl.ecs_angle, theta_max=wl.theta_max, nrhs=64, smoother="jacobi",
                      precision=args.precision)
        f = torch.tensor(wl.f, dtype=torch.complex128, device=dev)
        force_shapes(s, args.shapes)
        u = s.empty()
        st, its, _, dt, prof = timed_solve(torch, s, u, f, "gmres", RTOL, args.maxit, profile=True,
                                           graph_time=False)
        res = {"status": st, "max_steps": max(its), "seconds": dt, "shapes": shapes(s), "kernels": per_class(prof)}
    elif args.only == "c5":
        res = c5(mg, W, torch, dev, reps=1)
    print(json.dumps({"only": args.only, "result": res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", default=None,
                    help="run one workload only (headline, c3_gmres3, c3_jacobi, c4, c4_jacobi_511, c5)")
    ap.add_argument("--precision", default="c128", help="with --only headline / c4_jacobi_511 / --light c3_*")
    ap.add_argument("--light", action="store_true", help="with --only c3_*: one solve, no FP64 references")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 1 GiB four times (counter calibration)")
    ap.add_argument("--shapes", default=None, help="with --only: tile shape per level, comma-separated")
    ap.add_argument("--maxit", type=int, default=MAXIT,
                    help="cap on GMRES steps per solve (a capped solve is reported as not converged)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the batch of "
              "right-hand sides would shard across GPUs without communication).", file=sys.stderr)
        sys.exit(2)

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
    if args.only:
        only(args, mg, W, torch, dev)
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
    # records and captures the operations outside the timed region
    s.solve(u, f, mode="gmres", rtol=RTOL, maxit=2, restart=RESTART)
    for w in range(args.warmup):
        u.zero_()
        s.solve(u, f, mode="gmres", rtol=RTOL, maxit=args.maxit, restart=RESTART)
        log("warmup step %d done" % w)

    torch.cuda.synchronize()
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
    # kernel timing: the same solves again, launch by launch with HIP events
    # around every launch on the library's stream (events captured inside a
    # HIP graph cannot be timed)
    s.profile(True)
    tp = time.perf_counter()
    for k in range(args.steps):
        u.zero_()
        s.solve(u, f, mode="gmres", rtol=RTOL, maxit=args.maxit, restart=RESTART)
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - tp
    prof = s.profile_read()
    s.profile(False)

    dofs = N_GRID * N_GRID * NRHS
    value = dofs * args.steps / elapsed / 1e6
    kernels = per_class(prof)
    # dominant class of the timed region (every class, coarse levels included)
    dom = max(kernels, key=lambda c: kernels[c]["ms"])
    kd = kernels[dom]
    tr = committed_traffic(dom, WORKLOAD)
    roofline = {
        "bound": "hbm", "achieved": kd["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kd["frac"],
        "traffic": tr["traffic_bytes_per_launch"] if tr else None,
        "kernel": dom, "avg_launch_us": kd["avg_launch_us"],
        "algorithmic_bytes_per_launch": kd["algorithmic_bytes_per_launch"], "launches": kd["launches"],
        "timing": ("HIP events around every launch of %d further solves of the same workload in this process, "
                   "launched one by one (%.1f ms per solve, against %.1f ms per solve as replayed graphs)"
                   % (args.steps, 1e3 * elapsed_prof / args.steps, 1e3 * elapsed / args.steps)),
    }
    if tr and "ratio" in tr:
        roofline["traffic_counter_run"] = tr

    # true residual and the FP64 reference of the mixed run
    r = s.apply(u)
    true_res = [rel_err(r[i], f[i]) for i in range(NRHS)]
    ref = s.empty()
    s.solve(ref, f, mode="gmres", rtol=1e-12, maxit=args.maxit, restart=RESTART)
    extra = {"setup_s": round(setup_s, 3), "status": statuses[-1], "gmres_steps": iters[-1],
             "true_rel_residual_max": max(true_res),
             "error_at_rtol_1e-6_vs_fp64_1e-12_max": max(rel_err(u[i], ref[i]) for i in range(NRHS)),
             "kernels": kernels, "cycle_kernels_all_levels": cycle_summary(prof)}
    cpu = None
    if not args.no_extras:
        # standalone level-dependent multigrid on the same batch (Sec. 4.1 LVL-MG)
        st, its, hists, dts, _ = timed_solve(torch, s, u, f, "standalone", RTOL, 300)
        extra["standalone"] = {"status": st, "cycles": its, "seconds": round(dts, 3),
                               "last_ratio": [float(h[-1]) for h in hists]}
        log("standalone:", st, its)
        # mixed precision: complex64 cycle inside FP64 FGMRES
        sm = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max,
                       nrhs=NRHS, precision="mixed", smoother=SMOOTHER)
        um = sm.empty()
        st, its, hists, dtm, profm = timed_solve(torch, sm, um, f, "gmres", RTOL, args.maxit, profile=True)
        err6 = [rel_err(um[i], ref[i]) for i in range(NRHS)]
        um.zero_()
        st9, its9, _ = sm.solve(um, f, mode="gmres", rtol=1e-9, maxit=args.maxit, restart=RESTART)
        extra["mixed"] = {"status": st, "gmres_steps": its, "seconds": round(dtm, 3),
                          "Mdof_per_s": round(dofs / dtm / 1e6, 3),
                          "error_at_rtol_1e-6_vs_fp64_1e-12": err6,
                          "error_at_rtol_1e-9_vs_fp64_1e-12": [rel_err(um[i], ref[i]) for i in range(NRHS)],
                          "rtol_1e-9": {"status": st9, "gmres_steps": its9},
                          "cycle_kernels_all_levels": cycle_summary(profm), "kernels": per_class(profm)}
        log("mixed:", st, its)
        sm.close()
        del um
        # the omega-Jacobi cycle, right-preconditioned GMRES(20), capped
        sj = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, theta_max=wl.theta_max,
                       nrhs=NRHS, smoother="jacobi")
        st, its, hists, dtj, profj = timed_solve(torch, sj, u, f, "gmres", RTOL, JACOBI_MAXIT, profile=True)
        extra["omega_jacobi_gmres"] = {"status": st, "gmres_steps": its, "seconds": round(dtj, 3),
                                       "ms_per_step": round(1e3 * dtj / max(its), 3),
                                       "last_ratio": [float(h[-1]) for h in hists],
                                       "cycle_kernels_all_levels": cycle_summary(profj), "shapes": shapes(sj),
                                       "kernels": per_class(profj)}
        log("omega-jacobi:", st, its)
        sj.close()
        # comparator of Table 3 (MG-FGMRES): the cycle on -Delta - (1 + 0.5 i) k^2
        # on every level, preconditioning the unshifted problem
        L = s.num_levels
        sc = mg.Solver(wl.n, wl.h, k2, ecs=wl.ecs, ecs_angle=wl.ecs_angle, sigma=[1 + 0.5j] * L, nrhs=NRHS,
                       smoother=SMOOTHER)
        st, its, hists, dtc, _ = timed_solve(torch, sc, u, f, "gmres", RTOL, 2000)
        extra["fixed_shift_csl"] = {"sigma": "1+0.5i on every level", "status": st, "gmres_steps": its,
                                    "seconds": round(dtc, 3), "Mdof_per_s": round(dofs / dtc / 1e6, 3)}
        log("fixed-shift comparator:", st, its)
        sc.close()
        s.close()
        del u, ref
        torch.cuda.empty_cache()
        extra["c3_255"] = c3(mg, W, torch, dev)
        extra["batched"], bsteps = batched(mg, W, torch, dev)
        extra["adjoint_c5"] = c5(mg, W, torch, dev)
        extra["theta_sweep_table5"] = theta_sweep(mg, W, torch, dev)
        extra["paper_models"] = paper_models(mg, W, torch, dev)
        if not args.no_cpu_baseline:
            extra["cpu_baseline_batched"] = cpu_baseline_batched(bsteps)
    else:
        s.close()

    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, iters[-1][0])

    probe = hbm_probe(torch, dev)
    roofline["hbm_probe"] = probe
    if roofline["achieved"]:
        roofline["frac_of_copy"] = round(roofline["achieved"] / probe["copy_GBps"], 4)
    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "Mdof/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": "%dx%d" % (N_GRID, N_GRID), "h": "1/1024", "nrhs": NRHS,
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
