"""The stage-kernel forms that the default does not pick, forced with
LM_STAGE_KERNEL when the solver is created: "lds" (z-marching LDS planes in
3D, halo tiles in 2D) and "direct" (one thread per cell, in 2D), against
the FP64 oracle on grids whose planes tile by 64 x 4: periodic boxes,
walls with gravity, Sutherland's law and the enclosed-system p0, the flame
sheet, and the immersed-body slot flame with its inflow and outflow sides
(2D)."""
import pytest

from workloads import c2_case, c3_case, c4_case
from _cases import oracle_for, gpu_for, compare
from test_gpu_cavity import _cavity_3d
from test_gpu_edges import _reacting_3d_case

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True)
def _lds_stage(monkeypatch):
    monkeypatch.setenv("LM_STAGE_KERNEL", "lds")


def _run(case, steps, precision="fp64"):
    o, st = oracle_for(case)
    for _ in range(steps):
        st = o.step(st)
    s = gpu_for(case, precision=precision)
    s.step(steps)
    errs = compare(st, s.get(device=False))
    print(case.name, errs, s.stats, flush=True)
    bad = {k: v for k, v in errs.items() if not (v <= TOL)}
    assert not bad, f"fields above {TOL:g}: {bad} (all: {errs})"


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tiled_2d_random_modes(precision):
    print("lds 2d random modes 128", precision, flush=True)
    _run(c2_case(n=128), 3, precision)


def test_tiled_2d_slot_flame():
    print("lds 2d slot flame 128x256", flush=True)
    _run(c3_case(nx=128, ny=256), 3)


def test_marching_3d_random_modes():
    print("lds 3d random modes 64^3", flush=True)
    _run(c4_case(n=64), 2)


@pytest.mark.parametrize("slip", [False, True], ids=["noslip", "slip"])
def test_marching_3d_cavity(slip):
    print("lds 3d cavity 64x8x12 slip", slip, flush=True)
    _run(_cavity_3d(n=(64, 8, 12), slip=slip), 3)


def test_marching_3d_flame_sheet():
    print("lds 3d reacting 64x8x16", flush=True)
    _run(_reacting_3d_case((64, 8, 16)), 3)


@pytest.mark.parametrize("case", ["random", "flame"])
def test_direct_2d_on_tiled_grids(case, monkeypatch):
    """LM_STAGE_KERNEL=direct: the one-thread-per-cell kernel on 2D grids
    that the default would give to the halo-tile kernel."""
    monkeypatch.setenv("LM_STAGE_KERNEL", "direct")
    print("direct 2d", case, flush=True)
    _run(c2_case(n=128) if case == "random" else c3_case(nx=128, ny=256), 3)
