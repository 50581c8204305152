"""Benchmark: cell-updates/s of the full predictor-corrector step.

Headline workload: the 3D triply periodic 2*pi box at 256^3, FP64,
random-mode temperature (|k| <= 6, density ratio 6) and solenoidal velocity
(rms 0.1), Re = 400, Pr = 0.7, CFL 0.3, Poisson solved to relative residual
1e-10 in both stages (seeded synthetic input). A step is one
predictor-corrector pass with two multigrid-preconditioned CG solves. The
same workload is timed with the mixed-precision preconditioner beside it.
Its working set (about 2.7 GB) streams from HBM, so its kernels carry the
HBM roofline. The 2D 1024^2 workload follows with an effective-bandwidth
figure for its finest-level kernel: its working set (about 100 MB) stays in
the 256 MB last-level cache (MALL), so that figure is not an HBM rate.

Prints one JSON line. With --summarize-trace / --summarize-pmc it instead
reads rocprofv3 output databases and prints the per-kernel summaries kept
with the profiles (no GPU needed for those).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2603_01727_amd", "csrc", f)
                  for f in ("lm_mg_kernels.h", "lm_mg3d.h", "lm_solver.hip")]

# Kernel classes timed inside the step (lm_kernel_timing) and their
# algorithmic HBM bytes per finest-level cell (FP64 build, mixed build):
#  0 finest down: 3D reads b = r (8 B), writes the pre-smoothed correction
#    (8 B FP64 / 4 B FP32) and the coarse right-hand side (one value per 8
#    cells); 2D additionally carries the single-reduction CG update: reads
#    r, w, s, u, p, x (6 x 8 B), writes p, s, x, r, correction (5 x 8 B) and
#    the coarse right-hand side (8 B per 4 cells).
#  1 finest 3D up: reads the pre-smoothed correction and the coarse
#    correction (one per 8 cells), b = r (8 B), writes u = M r and w = A u
#    (8 B each; u in FP32 for mixed).
#  2 single-reduction CG update (3D): reads x, r, p, s, w (5 x 8 B) and u
#    (8 B / 4 B), writes x, r, p, s (4 x 8 B). Iteration 1 has no old p, s
#    and is left out of the timed set.
KCLASS_3D = {
    0: ("k_mg_down3d finest (two red-black sweeps from zero + restriction)", 8 + 8 + 1, 8 + 4 + 0.5),
    1: ("k_mg_up3d finest (prolongation + two red-black sweeps + w = A u + CG partial sums)",
        8 + 1 + 8 + 8 + 8, 4 + 0.5 + 8 + 4 + 8),
    2: ("k_cgcg_update (single-reduction CG: p, s, x, r)", 10 * 8, 9 * 8 + 4),
}
KCLASS_2D = {
    0: ("k_mg_down2d finest (fused CG update + two red-black sweeps + restriction)", 6 * 8 + 5 * 8 + 2,
        None),
}
TRAFFIC_C4 = os.path.join(ROOT, "profiles", "c4_256_fp64_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per side of the 3D headline box")
    ap.add_argument("--timed-steps", type=int, default=10,
                    help="further steps per kernel class with in-step event timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the 2D 1024^2 workload")
    ap.add_argument("--no-vc", action="store_true", help="skip the beta = 1 vs beta = 1/rho solve comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the 64^2, slot-flame and 512^2 workloads")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 512^2 200-step and 128^3 gradients")
    ap.add_argument("--small", choices=("c1", "c2", "adjoint"),
                    help="only the 64^2 (c1) or 1024^2 (c2) FP64 steps, or only the 512^2 200-step gradient "
                    "and the 128^3 40-step gradients (adjoint), for kernel traces of those paths")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a device copy of known size (for HBM counter calibration)")
    ap.add_argument("--summarize-trace", metavar="DB", help="summarise a rocprofv3 kernel-trace database")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="summarise two rocprofv3 --pmc databases (FETCH_SIZE, then WRITE_SIZE)")
    ap.add_argument("--traffic-out", metavar="JSON", help="with --summarize-pmc: write the C4 traffic record")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


PARAM_KEYS = ("Re", "Pr", "sigma", "inv_Fr2", "reacting", "S", "qs", "eps", "tol", "Le_F", "Le_O", "Da_ib",
              "p0", "dt", "cfl", "poisson_rtol")


def make_solver(case, precision):
    """Solver for a seeded workload (any sides, immersed body, inflow data)."""
    from paper_2603_01727_amd import Solver
    nd = case.ndim
    kw = {k: case.params[k] for k in PARAM_KEYS if k in case.params}
    s = Solver(case.n[:nd], case.L[:nd], bc=case.bc, precision=precision, poisson_maxit=200,
               with_ib=case.ib is not None, device="cuda:0", **kw)
    for (d, side), data in (case.bnd or {}).items():
        s.set_side(d, side, v=data.get("v"), Z=data.get("Z"), H=data.get("H"), F=data.get("F"),
                   wall=data.get("wall"))
    s.set(T=case.T, H=case.H if case.T is None else None, v=case.v, Z=case.Z, ib=case.ib)
    return s


def time_solver(case, precision, steps, warmup):
    import torch
    s = make_solver(case, precision)
    if warmup:
        s.step(warmup)
    torch.cuda.synchronize()
    it0 = s.stats["total_poisson_iters"] if s.stats else 0
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    iters = (s.stats["total_poisson_iters"] - it0) / (2.0 * steps)
    sec = t1 - t0
    return dict(sec=sec, ms_per_step=1e3 * sec / steps, value=case.ncells * steps / sec,
                poisson_iters_per_solve=iters, dt=s.dt, solver=s, steps_taken=warmup + steps)


def time_class(s, which, steps):
    """Mean event-measured duration (us) of one kernel class over its
    full-work launches in `steps` further steps, and the launch count."""
    import ctypes as C
    ms = C.c_double()
    cnt = C.c_int()
    if s.lib.lm_kernel_timing(s.ctx, which, 64 * steps) != 0:
        return None
    s.step(steps)
    st = s.lib.lm_kernel_timing_read(s.ctx, C.byref(ms), C.byref(cnt))
    s.lib.lm_kernel_timing(s.ctx, which, 0)
    if st != 0 or cnt.value == 0:
        return None
    return ms.value * 1e3, cnt.value


def load_traffic(path):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    return t if t.get("kernel_source_hash") == kernel_source_hash() else None


def class_rooflines(s, ncells, classes, steps, mixed=False):
    """Each kernel class timed inside the step (start/stop HIP events bound
    to its dispatches on the solver's stream), priced at its algorithmic
    bytes; the class with the largest time per step is the dominant one."""
    rows = []
    for which, (name, b64, bmx) in classes.items():
        bpc = bmx if mixed else b64
        t = time_class(s, which, steps)
        if t is None or bpc is None:
            continue
        us, cnt = t
        achieved = bpc * ncells / (us * 1e-6) / 1e9
        rows.append(dict(kernel=name, timing_class=which, avg_us=round(us, 3), launches_timed=cnt,
                         launches_per_step=round(cnt / steps, 2), us_per_step=round(us * cnt / steps, 1),
                         bytes_per_cell=bpc, algorithmic_bytes_per_launch=bpc * ncells,
                         achieved=round(achieved, 1), frac=round(achieved / HBM_PEAK_GBS, 4)))
    return rows


def c4_roofline(s, ncells, steps):
    rows = class_rooflines(s, ncells, KCLASS_3D, steps)
    if not rows:
        return None
    dom = max(rows, key=lambda r: r["us_per_step"])
    t = load_traffic(TRAFFIC_C4)
    traffic = None
    if t is not None:
        traffic = t.get("bytes_per_launch", {}).get(str(dom["timing_class"]))
    return dict(bound="hbm", achieved=dom["achieved"], peak=HBM_PEAK_GBS, unit="GB/s", frac=dom["frac"],
                traffic=traffic, kernel=dom["kernel"], avg_us=dom["avg_us"], launches_timed=dom["launches_timed"],
                timed_steps=steps, bytes_per_cell=dom["bytes_per_cell"],
                algorithmic_bytes_per_launch=dom["algorithmic_bytes_per_launch"],
                dominant_by="event-timed time per step among the timed classes",
                classes=rows)


def field_differences(s_a, s_b):
    import numpy as np
    fa = s_a.get(("rho", "v", "H", "T", "P"), device=False)
    fb = s_b.get(("rho", "v", "H", "T", "P"), device=False)
    out = {}
    for k in ("rho", "H", "T", "P"):
        out[k] = float(np.linalg.norm(fa[k] - fb[k]) / np.linalg.norm(fb[k]))
    for d in range(len(fb["v"])):
        out[f"v{d}"] = float(np.linalg.norm(fa["v"][d] - fb["v"][d]) / np.linalg.norm(fb["v"][d]))
    return out


def precision_block(case, ref, steps, warmup, precision):
    """Another preconditioner precision on the same workload and step count,
    with its per-field relative L2 difference from the FP64 state once both
    have taken the same number of steps."""
    r = time_solver(case, precision, steps, warmup)
    out = dict(value=r["value"], ms_per_step=round(r["ms_per_step"], 4),
               poisson_iters_per_solve=r["poisson_iters_per_solve"],
               speedup_vs_fp64=round(r["value"] / ref["value"], 3))
    extra = ref["steps_taken"] - r["steps_taken"]
    if extra >= 0:
        if extra:
            r["solver"].step(extra)
        out["rel_l2_vs_fp64"] = field_differences(r["solver"], ref["solver"])
        out["compared_after_steps"] = ref["steps_taken"]
    r["solver"].close()
    return out


def c2_block(steps=100, warmup=5, timed=20):
    """The 2D doubly periodic 1024^2 workload (random modes |k| <= 8,
    density ratio 4, Re 500), FP64, mixed and mixed-flexible."""
    from workloads import c2_case
    case = c2_case()
    r64 = time_solver(case, "fp64", steps, warmup)
    out = {"workload": "2D periodic 2pi box 1024x1024, random modes |k|<=8, density ratio 4, Re=500, Pr=0.7, "
                       "CFL 0.3, Poisson rtol 1e-10", "steps": steps, "warmup": warmup,
           "fp64": dict(value=r64["value"], ms_per_step=round(r64["ms_per_step"], 4),
                        poisson_iters_per_solve=r64["poisson_iters_per_solve"])}
    rows = class_rooflines(r64["solver"], case.ncells, KCLASS_2D, timed)
    r64["steps_taken"] += timed * len(rows)
    if rows:
        r = rows[0]
        out["effective_bandwidth"] = dict(
            kind="mall-assisted effective bandwidth (the ~100 MB working set stays in the 256 MB MALL); "
                 "not an HBM rate", kernel=r["kernel"], avg_us=r["avg_us"], bytes_per_cell=r["bytes_per_cell"],
            effective_GBs=r["achieved"], frac_of_hbm_peak=r["frac"], launches_timed=r["launches_timed"])
    out["mixed"] = precision_block(case, r64, steps, warmup, "mixed")
    out["mixed_flexible"] = precision_block(case, r64, steps, warmup, "mixed-flexible")
    r64["solver"].close()
    return out


def poisson_forms(n=1024, reps=10):
    """The pressure solve alone at n^2 in its two forms: beta = 1 (the
    step's operator) and beta = 1/rho_f (div(grad P / rho) = b), FP64 and
    mixed, on a seeded random-mode density (ratio 4, |k| <= 8) and
    right-hand side, Poisson rtol 1e-10, from a zero start. Device arrays;
    per solve: wall time between device synchronisations, including the
    variable-coefficient set-up (density copy, coarse densities, coarsest
    inverse)."""
    import math
    import numpy as np
    import torch
    from paper_2603_01727_amd import Solver
    from workloads import variable_coefficient_problem
    L = (2 * math.pi, 2 * math.pi)
    rho, b = variable_coefficient_problem((n, n), L, seed=2)
    out = {"workload": f"pressure solve {n}x{n} periodic, random-mode density ratio 4 and right-hand side, "
                       f"rtol 1e-10, zero start", "solves": reps}
    for prec in ("fp64", "mixed"):
        s = Solver((n, n), L, Re=100.0, dt=1e-3, precision=prec, poisson_rtol=1e-10, variable_coefficient=True)
        bt = torch.tensor(b, device="cuda:0")
        rt = torch.tensor(rho, device="cuda:0")
        z = torch.zeros_like(bt)
        res = {}
        for form, kw in (("beta_one", {}), ("beta_inv_rho", {"rho": rt})):
            for _ in range(3):
                s.project(bt, **kw)
            ts = []
            for _ in range(reps):
                s.project(z)    # zero right-hand side: P = 0, the next solve starts cold
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = s.project(bt, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            res[form] = dict(ms_per_solve=round(1e3 * float(np.median(ts)), 4), iters=info["iters"],
                             relres=info["relres"])
        res["inv_rho_over_one"] = round(res["beta_inv_rho"]["ms_per_solve"] / res["beta_one"]["ms_per_solve"], 3)
        out[prec] = res
        s.close()
    return out


def bench_configs(steps=20, warmup=3):
    """The other workloads at their full sizes, FP64 and mixed: 64^2 hot
    spot (Poisson 1e-12), 768x1536 slot flame, 512^2 random modes (the
    adjoint workload's forward step); same steps for both precisions."""
    from workloads import c1_case, c3_case, c5_case
    out = {}
    for name, mk in (("c1_64", c1_case), ("c3_slot_flame_768x1536", c3_case), ("c5_512", c5_case)):
        case = mk()
        res = {}
        for prec in ("fp64", "mixed"):
            r = time_solver(case, prec, steps, warmup)
            res[prec] = dict(value=r["value"], ms_per_step=round(r["ms_per_step"], 4),
                             poisson_iters_per_solve=r["poisson_iters_per_solve"])
            r["solver"].close()
        res["mixed_speedup_vs_fp64"] = round(res["mixed"]["value"] / res["fp64"]["value"], 3)
        res["steps"], res["warmup"] = steps, warmup
        out[name] = res
    return out


def adjoint_block(every=20):
    """The adjoint workload: 512^2 periodic random modes, its full length
    (200 steps), checkpoints every 20 steps: the gradient of the final
    kinetic energy with respect to T0 (the checkpointed forward run, then
    the reverse sweep, which replays each segment forward to tape its states
    and runs the adjoint steps back through it), against the same steps
    forward only. Fixed time step (the CFL step of the initial state), the
    Poisson solves of both sweeps to 1e-10."""
    import torch
    from paper_2603_01727_amd import Solver
    from paper_2603_01727_amd.adjoint import Trajectory, final_kinetic_energy
    from workloads import c5_case
    case = c5_case()
    nsteps = case.nsteps
    kw = dict(bc=case.bc, Re=case.params["Re"], Pr=case.params["Pr"], poisson_rtol=1e-10, poisson_maxit=400)
    probe = Solver(case.n[:2], case.L[:2], cfl=case.params["cfl"], **kw)
    probe.set(T=case.T, v=case.v)
    dt = probe.dt
    probe.close()
    s = Solver(case.n[:2], case.L[:2], dt=dt, with_adjoint=True, **kw)
    T0 = torch.tensor(case.T, dtype=torch.float64, device="cuda", requires_grad=True)
    v0 = [torch.tensor(x, dtype=torch.float64, device="cuda") for x in case.v]
    J = final_kinetic_energy(s, T0, v0, 4, 2)      # warm-up of both sweeps
    J.backward()
    T0.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = final_kinetic_energy(s, T0, v0, nsteps, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.set(T=case.T, v=case.v)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    s.step(nsteps)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    # the same gradient with every step taped in the forward pass (no
    # replay: 200 states and step levels, about 11 GB of HBM)
    traj = Trajectory(s, nsteps, every, tape_all=True)
    traj.forward(T0.detach(), v0)
    traj.backward()
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    traj.forward(T0.detach(), v0)
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    g_all = traj.backward()[0]
    torch.cuda.synchronize()
    t7 = time.perf_counter()
    same = bool(torch.equal(g_all, T0.grad))
    del traj
    s.close()
    fwd = t4 - t3
    return dict(workload=f"2D periodic 2pi box 512^2, random modes |k|<=8, density ratio 4, Re=300, Pr=0.7, "
                         f"{nsteps} steps of dt={dt:.6g}, gradient of the final kinetic energy w.r.t. T0",
                checkpoint_every=every, gradient_s=round(t2 - t0, 4),
                forward_with_checkpoints_s=round(t1 - t0, 4), reverse_sweep_s=round(t2 - t1, 4),
                forward_only_s=round(fwd, 4), gradient_over_forward=round((t2 - t0) / fwd, 3),
                reverse_ms_per_step=round((t2 - t1) / nsteps * 1e3, 4),
                J=float(J.item()), grad_norm=float(T0.grad.norm().item()),
                tape_all=dict(gradient_s=round(t7 - t5, 4), forward_with_tape_s=round(t6 - t5, 4),
                              reverse_sweep_s=round(t7 - t6, 4), gradient_over_forward=round((t7 - t5) / fwd, 3),
                              same_gradient_bits=same))


def adjoint3d_block(n=128, nsteps=40, every=10):
    """The adjoint in 3D: the headline's triply periodic random-mode box at
    n^3 (same seeded fields as the 256^3 workload's generator at this size),
    nsteps steps of the initial state's CFL step, checkpoints every
    ``every``: the gradient of the final kinetic energy with respect to T0
    against the same steps forward only."""
    import torch
    from paper_2603_01727_amd import Solver
    from paper_2603_01727_amd.adjoint import final_kinetic_energy
    from workloads import c4_case
    case = c4_case(n=n)
    kw = dict(bc=case.bc, Re=case.params["Re"], Pr=case.params["Pr"], poisson_rtol=1e-10, poisson_maxit=400)
    probe = Solver(case.n, case.L, cfl=case.params["cfl"], **kw)
    probe.set(T=case.T, v=case.v)
    dt = probe.dt
    probe.close()
    s = Solver(case.n, case.L, dt=dt, with_adjoint=True, **kw)
    T0 = torch.tensor(case.T, dtype=torch.float64, device="cuda", requires_grad=True)
    v0 = [torch.tensor(x, dtype=torch.float64, device="cuda") for x in case.v]
    J = final_kinetic_energy(s, T0, v0, 2, 1)      # warm-up of both sweeps
    J.backward()
    T0.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = final_kinetic_energy(s, T0, v0, nsteps, every)
    J.backward()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.set(T=case.T, v=case.v)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.step(nsteps)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    s.close()
    return dict(workload=f"3D triply periodic 2pi box {n}^3, random modes |k|<=6, density ratio 6, Re=400, "
                         f"Pr=0.7, {nsteps} steps of dt={dt:.6g}, gradient of the final kinetic energy w.r.t. T0",
                checkpoint_every=every, gradient_s=round(t1 - t0, 4), forward_only_s=round(t3 - t2, 4),
                gradient_over_forward=round((t1 - t0) / (t3 - t2), 3), J=float(J.item()),
                grad_norm=float(T0.grad.norm().item()))


ORACLE_KEYS = ("Re", "Pr", "sigma", "inv_Fr2", "reacting", "S", "qs", "eps", "tol", "Le_F", "Le_O", "Da_ib",
               "p0", "dt", "cfl")


def cpu_baseline(case, budget_s=10.0):
    """The FP64 oracle on the host cores: after one untimed warm-up step
    (the Heun start), AB2/AM2 steps of the same workload until about
    budget_s seconds have passed (at least 2). Its Poisson solve is the
    exact FFT transform solve on all usable cores; the stencils are NumPy on
    one thread."""
    from oracle import Grid, Oracle, Params
    from oracle.poisson import FFT_WORKERS
    nd = case.ndim
    g = Grid(case.n[:nd], case.L[:nd], bc=case.bc, bnd=case.bnd)
    o = Oracle(g, Params(**{k: case.params[k] for k in ORACLE_KEYS if k in case.params}), ib=case.ib)
    st = o.initial_state(case.T, case.v, Z=case.Z, H=case.H)
    st = o.step(st)
    n = 0
    t0 = time.perf_counter()
    while n < 2 or time.perf_counter() - t0 < budget_s:
        st = o.step(st)
        n += 1
    sec = time.perf_counter() - t0
    shape = "x".join(str(x) for x in case.n[:nd])
    return dict(value=case.ncells * n / sec, unit="cell-updates/s", cores=FFT_WORKERS, kind="oracle",
                sample=f"{n} steps of the {shape} workload after one warm-up step, {sec:.1f} s: FFT Poisson "
                       f"solves on {FFT_WORKERS} threads (scipy.fft workers), NumPy stencils on one thread",
                host_cpus=os.cpu_count(), host_cpus_usable=FFT_WORKERS)


def copy_calibration():
    """Device-to-device copy of 512 MiB, twice (reference for the HBM
    byte counters: 512 MiB read + 512 MiB written per copy)."""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()


# --- rocprofv3 output summaries (host only) --------------------------------

COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 512 * 1024 * 1024


def _groups(rows):
    """rows: (name, grid, value) -> {(name, grid): [values]}"""
    g = {}
    for name, grid, v in rows:
        g.setdefault((name, grid), []).append(v)
    return g


def _full_work(vals):
    """Launches that did a full pass: at least half the group's 90th
    percentile (launches queued after a solve converged return at once)."""
    s = sorted(vals)
    cut = 0.5 * s[int(0.9 * (len(s) - 1))]
    return [v for v in vals if v >= cut]


def summarize_trace(db_path):
    import sqlite3
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, grid_x * grid_y * grid_z, end - start, vgpr_count, lds_size, "
                      "scratch_size from kernels").fetchall()
    res = {}
    for name, grid, dur, vgpr, lds, scr in rows:
        r = res.setdefault((name.split("(")[0], grid), dict(d=[], vgpr=vgpr, lds=lds, scratch=scr))
        r["d"].append(dur * 1e-3)
    tot = sum(sum(r["d"]) for r in res.values())
    print(f"kernel-trace summary of {os.path.basename(db_path)}: {len(rows)} dispatches, {tot / 1e3:.2f} ms kernel "
          f"time. Columns: launches, mean (all), full-work launches and their mean (us; full work = at least "
          f"half the group's 90th percentile), total ms, VGPRs, LDS bytes, scratch bytes.")
    for (name, grid), r in sorted(res.items(), key=lambda kv: -sum(kv[1]["d"])):
        d = r["d"]
        fw = _full_work(d)
        print(f"{name[:58]:58s} grid {grid:9d} n {len(d):5d} mean {sum(d) / len(d):9.2f}  full {len(fw):5d} "
              f"mean {sum(fw) / len(fw):9.2f}  total {sum(d) / 1e3:8.3f}  vgpr {r['vgpr']:3d} lds {r['lds']:6d} "
              f"scratch {r['scratch']}")
    # the single-reduction CG update by iteration: the first launch after a
    # solve's initialisation kernel is iteration 1 (no old p, s: fewer bytes)
    seq = db.execute("select name, end - start from kernels order by start").fetchall()
    it, by_k = 0, {}
    for name, dur in seq:
        if "k_cg_init" in name:
            it = 0
        elif "k_cgcg_update" in name:
            it += 1
            by_k.setdefault(min(it, 2), []).append(dur * 1e-3)
    for k, d in sorted(by_k.items()):
        fw = _full_work(d)
        print(f"k_cgcg_update iteration {'1' if k == 1 else '>= 2'}: n {len(d)}, full-work n {len(fw)} "
              f"mean {sum(fw) / len(fw):.2f} us")
    # time between consecutive dispatches (end of one to start of the next)
    # inside the runs of work, i.e. leaving out pauses of 1 ms and more
    # (set-up, host work between workloads)
    tl = db.execute("select start, end from kernels order by start").fetchall()
    gaps = [(tl[i + 1][0] - tl[i][1]) * 1e-3 for i in range(len(tl) - 1)]
    gaps = [g for g in gaps if g < 1000.0]
    if gaps:
        gs = sorted(gaps)
        busy = sum((e - b) * 1e-3 for b, e in tl)
        print(f"dispatch gaps inside runs of work: n {len(gs)}, median {gs[len(gs) // 2]:.2f} us, mean "
              f"{sum(gs) / len(gs):.2f} us, total {sum(gs) / 1e3:.3f} ms against {busy / 1e3:.3f} ms of kernel time "
              f"(under the profiler, which lengthens both)")


def _pmc_rows(db_path, counter):
    import sqlite3
    db = sqlite3.connect(db_path)
    q = ("select kernel_name, grid_size, dispatch_id, sum(value) from counters_collection "
         "where counter_name = ? group by dispatch_id")
    return [(n.split("(")[0], g, v) for n, g, _, v in db.execute(q, (counter,)).fetchall()]


def summarize_pmc(fetch_db, write_db, traffic_out=None):
    f = _groups(_pmc_rows(fetch_db, "FETCH_SIZE"))
    w = _groups(_pmc_rows(write_db, "WRITE_SIZE"))
    # the calibration copy: the copy-kernel dispatch group that moved the
    # most (other copies of the run are small staging transfers)
    def calib(groups):
        cand = [vs for (n, _), vs in groups.items() if n.startswith(COPY_KERNEL)]
        return max(cand, key=lambda vs: sum(vs) / len(vs)) if cand else []
    cf, cw = calib(f), calib(w)
    if not cf or not cw:
        raise SystemExit("no copy-calibration dispatch in the databases (run bench.py with --copy-calibration)")
    kib = COPY_BYTES / 1024
    fs, ws = kib / (sum(cf) / len(cf)), kib / (sum(cw) / len(cw))
    print(f"HBM-side byte counters per dispatch, two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE). "
          f"Calibration: a 512 MiB device copy ({COPY_KERNEL}) reads and writes 512 MiB; it reads "
          f"FETCH {sum(cf) / len(cf):.1f} KiB and WRITE {sum(cw) / len(cw):.1f} KiB, so FETCH is scaled by {fs:.4f} "
          f"and WRITE by {ws:.4f}. Columns: full-work dispatches (FETCH at least half its 90th percentile), "
          f"scaled KiB per dispatch, MB per dispatch.")
    out = {}
    for key in sorted(f, key=lambda k: -sum(f[k])):
        if key not in w:
            continue
        fv, wv = _full_work(f[key]), _full_work(w[key])
        fk, wk = fs * sum(fv) / len(fv), ws * sum(wv) / len(wv)
        tot = (fk + wk) * 1024
        out[key] = tot
        print(f"{key[0][:58]:58s} grid {key[1]:9d} n {len(fv):4d}/{len(wv):4d} fetch {fk:11.1f} KiB "
              f"write {wk:11.1f} KiB total {tot / 1e6:9.2f} MB")
    if traffic_out:
        # timing class -> the finest-level dispatch group of that kernel
        pick = {}
        for (name, grid), tot in out.items():
            for which, tag in ((0, "k_mg_down3d<double"), (1, "k_mg_up3d<double, 2, 1"),
                               (2, "k_cgcg_update<3, double")):
                if tag in name and (which not in pick or grid > pick[which][1]):
                    pick[which] = (name, grid, tot)
        rec = {"workload": "3D periodic 256^3 FP64 step", "fetch_scale": round(fs, 4), "write_scale": round(ws, 4),
               "kernels": {str(k): f"{v[0]} grid {v[1]}" for k, v in pick.items()},
               "bytes_per_launch": {str(k): int(v[2]) for k, v in pick.items()},
               "kernel_source_hash": kernel_source_hash()}
        with open(traffic_out, "w") as fh:
            json.dump(rec, fh, indent=1)


def main():
    a = parse()
    if a.summarize_trace:
        summarize_trace(a.summarize_trace)
        return
    if a.summarize_pmc:
        summarize_pmc(a.summarize_pmc[0], a.summarize_pmc[1], a.traffic_out)
        return
    if a.small == "adjoint":
        print(json.dumps({"adjoint_c5": adjoint_block(), "adjoint_3d_128": adjoint3d_block()}))
        return
    if a.small:
        from workloads import c1_case, c2_case
        case = c1_case() if a.small == "c1" else c2_case()
        r = time_solver(case, "fp64", a.steps, a.warmup)
        r["solver"].close()
        print(json.dumps({"workload": case.name, "steps": a.steps, "warmup": a.warmup,
                          "ms_per_step": round(r["ms_per_step"], 4),
                          "poisson_iters_per_solve": r["poisson_iters_per_solve"]}))
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: --gpus must be 1 (the step has no "
                                   "multi-GPU path)"}))
        sys.exit(2)
    from workloads import c4_case
    case = c4_case(n=a.n)
    if a.copy_calibration:
        copy_calibration()
    r64 = time_solver(case, "fp64", a.steps, a.warmup)
    roof = c4_roofline(r64["solver"], case.ncells, a.timed_steps)
    if roof is not None:
        r64["steps_taken"] += a.timed_steps * len(roof["classes"])
    mixed = None
    if not a.no_mixed:
        mixed = precision_block(case, r64, a.steps, a.warmup, "mixed")
        mixed["flexible_cg"] = precision_block(case, r64, a.steps, a.warmup, "mixed-flexible")
    cfg = {"workload": f"3D triply periodic 2pi box {a.n}^3, random modes |k|<=6, density ratio 6, Re=400, "
                       f"Pr=0.7, CFL 0.3, Poisson rtol 1e-10", "cells": case.ncells, "dt": r64["dt"],
           "poisson_iters_per_solve": r64["poisson_iters_per_solve"]}
    r64["solver"].close()
    c2 = None if a.no_c2 else c2_block()
    forms = None if a.no_vc else poisson_forms()
    configs = None if a.no_configs else bench_configs()
    adj = None if a.no_adjoint else adjoint_block()
    adj3 = None if a.no_adjoint else adjoint3d_block()
    cpu = None if a.no_cpu else cpu_baseline(case)
    out = {
        "metric": "cell-updates/s per full time step (Poisson to 1e-10), FP64 vs mixed; HBM GB/s",
        "value": r64["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random-mode temperature and solenoidal velocity)",
        "config": cfg,
        "mixed": mixed,
        "c2_1024": c2,
        "poisson_forms": forms,
        "other_workloads": configs,
        "adjoint_c5": adj,
        "adjoint_3d_128": adj3,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
