"""Benchmark: cell-updates/s of the full predictor-corrector step.

Workload: the 2D doubly periodic 2*pi box at 1024^2, FP64, random-mode
temperature (density ratio up to 4) and solenoidal velocity, Re = 500,
Pr = 0.7, CFL 0.3, Poisson solved to relative residual 1e-10 in both stages
(seeded synthetic input). A step is one predictor-corrector pass with two
multigrid-preconditioned CG solves. The same workload is also timed with the
mixed-precision preconditioner. Prints one JSON line.
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
# Dominant kernel: the finest-level multigrid down kernel, which also carries
# the single-reduction CG update. Algorithmic bytes per cell (FP64): reads
# r, w, s, u, p, x (6 x 8 B), writes p, s, x, r and the pre-smoothed
# correction (5 x 8 B), and the coarse right-hand side (8 B per 4 cells).
DOMINANT = "k_mg_down2d (finest level, fused CG update + 2 red-black sweeps + restriction)"
BYTES_PER_CELL = 6 * 8 + 5 * 8 + 8 / 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_mg_down2d_finest_c2_1024_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2603_01727_amd", "csrc", f)
                  for f in ("lm_mg_kernels.h", "lm_solver.hip")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a device copy of known size (for HBM counter calibration)")
    ap.add_argument("--no-3d", action="store_true", help="skip the 256^3 FP64-vs-mixed comparison")
    ap.add_argument("--no-vc", action="store_true", help="skip the beta = 1 vs beta = 1/rho solve comparison")
    ap.add_argument("--no-configs", action="store_true", help="skip the 64^2, slot-flame and 512^2 workloads")
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
                poisson_iters_per_solve=iters, dt=s.dt, solver=s)


def kernel_roofline(s, ncells, steps=20):
    """Average duration of the dominant kernel as launched inside the step:
    each of its launches in `steps` further steps of the same run carries a
    start and a stop HIP event bound to the dispatch on the solver's stream
    (lm_kernel_timing); priced at its algorithmic bytes. The same kernel
    timed back to back in isolation (lm_bench_kernel) is reported beside it."""
    import ctypes as C
    ms = C.c_double()
    cnt = C.c_int()
    if s.lib.lm_kernel_timing(s.ctx, 64 * steps) != 0:
        return None
    s.step(steps)
    st = s.lib.lm_kernel_timing_read(s.ctx, C.byref(ms), C.byref(cnt))
    s.lib.lm_kernel_timing(s.ctx, 0)
    if st != 0 or cnt.value == 0:
        return None
    iso = C.c_double()
    iso_us = None
    if s.lib.lm_bench_kernel(s.ctx, 0, 200, C.byref(iso)) == 0:
        iso_us = round(iso.value * 1e3, 3)
    per_launch_s = ms.value * 1e-3
    achieved = BYTES_PER_CELL * ncells / per_launch_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if t.get("kernel_source_hash") == kernel_source_hash():
            traffic = t.get("bytes_per_launch")
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=DOMINANT,
                avg_us=round(per_launch_s * 1e6, 3), launches_timed=cnt.value, timed_steps=steps,
                isolated_avg_us=iso_us, bytes_per_cell=BYTES_PER_CELL,
                algorithmic_bytes_per_launch=BYTES_PER_CELL * ncells)


def bench_3d(steps=10, warmup=3):
    """The 3D triply periodic 256^3 workload (random modes |k| <= 6,
    density ratio 6, Re 400), FP64 against mixed precision on the same
    device, same steps; not the headline metric."""
    from workloads import c4_case
    case = c4_case()
    out = {"workload": "3D periodic 2pi box 256^3, random modes |k|<=6, density ratio 6, Re=400, Pr=0.7, "
                       "CFL 0.3, Poisson rtol 1e-10", "steps": steps, "warmup": warmup}
    res = {}
    for prec in ("fp64", "mixed"):
        r = time_solver(case, prec, steps, warmup)
        res[prec] = r
        out[prec] = dict(value=r["value"], ms_per_step=round(r["ms_per_step"], 3),
                         poisson_iters_per_solve=r["poisson_iters_per_solve"])
    out["mixed_speedup_vs_fp64"] = round(res["mixed"]["value"] / res["fp64"]["value"], 3)
    out["mixed_rel_l2_vs_fp64"] = field_differences(res["mixed"]["solver"], res["fp64"]["solver"])
    for r in res.values():
        r["solver"].close()
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


def cpu_baseline(case, budget_s=12.0):
    """The FP64 oracle on the host: one warm-up step, then steps until about
    budget_s seconds have passed (at least 2)."""
    from oracle import Grid, Oracle, Params
    p = case.params
    g = Grid(case.n[:2], case.L[:2])
    o = Oracle(g, Params(Re=p["Re"], Pr=p["Pr"], cfl=p["cfl"]))
    st = o.initial_state(case.T, case.v)
    st = o.step(st)
    t0 = time.perf_counter()
    n = 0
    while n < 2 or time.perf_counter() - t0 < budget_s:
        st = o.step(st)
        n += 1
    sec = time.perf_counter() - t0
    return dict(value=case.ncells * n / sec, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{n} steps of the {case.n[0]}x{case.n[1]} workload after one warm-up step "
                       f"(NumPy FP64, FFT Poisson, single thread), {sec:.1f} s",
                host_cpus=os.cpu_count(), host_cpus_usable=len(os.sched_getaffinity(0)))


def copy_calibration():
    """Device-to-device copy of 512 MiB, twice (reference for the HBM
    byte counters: 512 MiB read + 512 MiB written per copy)."""
    import torch
    a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1"}))
        sys.exit(2)
    from workloads import c2_case
    case = c2_case(n=a.n)
    if a.copy_calibration:
        copy_calibration()
    r64 = time_solver(case, "fp64", a.steps, a.warmup)
    roof = kernel_roofline(r64["solver"], case.ncells)
    mixed = None
    if not a.no_mixed:
        rmx = time_solver(case, "mixed", a.steps, a.warmup)
        mixed = dict(value=rmx["value"], ms_per_step=round(rmx["ms_per_step"], 4),
                     poisson_iters_per_solve=rmx["poisson_iters_per_solve"],
                     speedup_vs_fp64=round(rmx["value"] / r64["value"], 3))
        if roof is not None:
            # both runs at the same step count: per-field relative L2
            # difference of the mixed-precision state from the FP64 one
            rmx["solver"].step(roof["timed_steps"])
            mixed["rel_l2_vs_fp64"] = field_differences(rmx["solver"], r64["solver"])
            mixed["compared_after_steps"] = a.warmup + a.steps + roof["timed_steps"]
        rfl = time_solver(case, "mixed-flexible", a.steps, a.warmup)
        mixed["flexible_cg"] = dict(value=rfl["value"], ms_per_step=round(rfl["ms_per_step"], 4),
                                    poisson_iters_per_solve=rfl["poisson_iters_per_solve"],
                                    speedup_vs_fp64=round(rfl["value"] / r64["value"], 3))
        del rfl
    three_d = None if a.no_3d else bench_3d()
    forms = None if a.no_vc else poisson_forms(a.n)
    configs = None if a.no_configs else bench_configs()
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
        "config": {"workload": f"2D periodic 2pi box {a.n}x{a.n}, random modes |k|<=8, density ratio 4, "
                               f"Re=500, Pr=0.7, CFL 0.3, Poisson rtol 1e-10",
                   "cells": case.ncells, "dt": r64["dt"],
                   "poisson_iters_per_solve": r64["poisson_iters_per_solve"]},
        "mixed": mixed,
        "c4_3d": three_d,
        "poisson_forms": forms,
        "other_workloads": configs,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
