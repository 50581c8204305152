"""Differentially heated cavity (section 4.4) marched to the paper's steady
state criterion on one GPU: prints p0 and the mean Nusselt numbers of the
hot wall, the mid-plane and the cold wall (Eq 4.14-4.15) as the run goes.

    python tests/run_cavity_steady.py --ra 1e7 --n 512

Not collected by pytest (a long validation run; the test suite runs the
Ra = 10^2 case on 32^2 and 64^2). The state can be saved at the end and
given back with --resume to continue a run."""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ra", type=float, default=1e2)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--chunk", type=int, default=2000, help="steps between reports")
    ap.add_argument("--tol", type=float, default=1e-6, help="steady when |d p0/dt| over a chunk is below")
    ap.add_argument("--max-seconds", type=float, default=3600.0)
    ap.add_argument("--save", default=None, help="write the final state (.npz)")
    ap.add_argument("--resume", default=None, help="start from a saved state (.npz)")
    a = ap.parse_args()
    import torch
    from workloads import heated_cavity_case
    from _cases import gpu_for
    from test_gpu_cavity import _nusselt
    case = heated_cavity_case(n=a.n, Ra=a.ra)
    s = gpu_for(case, rtol=1e-10)
    if a.resume:
        s.load_state(torch.tensor(np.load(a.resume)["state"], device="cuda"))
    Pe = case.params["Re"] * case.params["Pr"]
    print(f"Ra {a.ra:g} n {a.n} dt {s.dt:.6g}", flush=True)
    t0 = time.time()
    p_prev = None
    while time.time() - t0 < a.max_seconds:
        st = s.step(a.chunk)
        rate = None if p_prev is None else (st["p0"] - p_prev) / (a.chunk * st["dt"])
        p_prev = st["p0"]
        nu = _nusselt(case, s.get(("T", "F"), device=False), Pe)
        print(f"t {st['time']:.4f} p0 {st['p0']:.7f} dp0dt {rate} Nu {nu[0]:.5f} {nu[1]:.5f} {nu[2]:.5f} "
              f"wall {time.time() - t0:.0f}", flush=True)
        if rate is not None and abs(rate) < a.tol:
            print("steady", flush=True)
            break
    if a.save:
        np.savez_compressed(a.save, state=s.save_state().cpu().numpy())


if __name__ == "__main__":
    main()
