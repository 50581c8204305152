"""Reverse-mode gradients of the step behind ``torch.autograd.Function``:
of the final kinetic energy with respect to the initial temperature
(``FinalKineticEnergy``), and of the whole final state (T, v) with respect
to the initial (T, v) (``StepFn``).

J(T0) = sum_cells 1/2 rho |v|^2 dV after ``nsteps`` predictor-corrector
steps from (T0, v0) with a fixed time step. The forward pass stores a full
state checkpoint every ``checkpoint_every`` steps. The backward pass walks
the segments from last to first: it restores the segment's checkpoint,
replays the segment forward while storing each step's state and the
step's predicted and new levels (the segment tape), then steps back from
the last step of the segment to its first with ``lm_step_adjoint_levels``,
which reads the taped levels instead of recomputing the step (one forward
step per step of the reverse sweep). Peak storage is (nsteps / k + k)
states and k step levels. Every step of the forward and reverse sweeps
runs in the HIP library; this module only sequences the calls.
"""
from __future__ import annotations

import math

import torch


def _on_device(x, device, mask: bool):
    """A body array (or list of arrays) as a tensor on the solver's device,
    so that it travels with device-resident initial fields in one call."""
    if x is None:
        return None
    if isinstance(x, (list, tuple)):
        return [_on_device(y, device, mask) for y in x]
    return torch.as_tensor(x, dtype=torch.uint8 if mask else torch.float64, device=device)


class Trajectory:
    """Checkpointed forward run of a ``Solver`` built with ``with_adjoint``
    and a fixed ``dt`` (the gradient is taken at fixed dt). ``ib``: the
    immersed-body arrays handed to ``Solver.set`` with the initial state
    (constants of the run)."""

    def __init__(self, solver, nsteps: int, checkpoint_every: int = 20, ib=None, tape_levels: bool = True,
                 tape_all: bool = False):
        if nsteps < 0 or checkpoint_every < 1:
            raise ValueError("nsteps >= 0 and checkpoint_every >= 1 required")
        if not solver.params.with_adjoint:
            raise ValueError("the solver needs with_adjoint=True")
        if not solver.params.dt > 0:
            raise ValueError("the gradient is taken at a fixed time step: give the solver dt > 0")
        self.solver = solver
        self.nsteps = int(nsteps)
        self.k = int(checkpoint_every)
        self.ib = None if ib is None else {k: _on_device(x, solver.device, k == "chi") for k, x in ib.items()}
        self.tape_levels = bool(tape_levels)   # False: lm_step_adjoint recomputes each step
        # True: the forward pass itself tapes every step's state and levels
        # (nsteps of each in device memory), so the reverse sweep replays
        # nothing; checkpoint_every is then unused
        self.tape_all = bool(tape_all)
        self.ckpt = {}
        self.tape = []
        self.levels = []
        self.final = None

    def forward(self, T0, v0, Z0=None) -> float:
        """Runs from (T0, v0), and the mixture fraction Z0 in reacting flow."""
        s = self.solver
        s.set(T=T0, v=v0, Z=Z0, ib=self.ib)
        if self.tape_all:
            size, lsize = s.state_size(), s.step_levels_size()
            while len(self.tape) < self.nsteps:
                self.tape.append(torch.empty(size, dtype=torch.uint8, device=s.device))
                self.levels.append(torch.empty(lsize, dtype=torch.uint8, device=s.device))
            self.ckpt = {0: s.save_state()}
            for n in range(self.nsteps):
                s.save_state(self.tape[n])
                s.step(1)
                s.save_step_levels(self.levels[n])
            self.final = s.save_state()
            return s.kinetic_energy()
        self.ckpt = {0: s.save_state()}
        done = 0
        while done < self.nsteps:
            m = min(self.k, self.nsteps - done)
            s.step(m)
            done += m
            if done < self.nsteps:
                self.ckpt[done] = s.save_state()
        self.final = s.save_state()
        return s.kinetic_energy()

    def backward(self, seed=None):
        """Returns (T0_bar, [v0_bar...]) as device tensors, and Z0_bar as a
        third entry in reacting flow. ``seed``: the
        cotangents of the final state as keyword arguments of
        ``Solver.adjoint_set`` (None: the gradient of the final kinetic
        energy)."""
        s = self.solver
        s.load_state(self.final)
        if seed is None:
            s.adjoint_seed_ke()
        else:
            s.adjoint_set(**seed)
        if self.tape_all:
            for n in reversed(range(self.nsteps)):
                s.load_state(self.tape[n])
                s.step_adjoint(self.levels[n])
            if self.nsteps == 0:
                s.load_state(self.ckpt[0])
            return s.adjoint_initial()
        size = s.state_size()
        nseg = math.ceil(self.nsteps / self.k)
        for q in reversed(range(nseg)):
            a = q * self.k
            b = min(a + self.k, self.nsteps)
            while len(self.tape) < b - a:
                self.tape.append(torch.empty(size, dtype=torch.uint8, device=s.device))
            s.load_state(self.ckpt[a])
            if self.tape_levels:
                while len(self.levels) < b - a:
                    self.levels.append(torch.empty(s.step_levels_size(), dtype=torch.uint8, device=s.device))
                for n in range(a, b):
                    s.save_state(self.tape[n - a])
                    s.step(1)
                    s.save_step_levels(self.levels[n - a])
                for n in reversed(range(a, b)):
                    s.load_state(self.tape[n - a])
                    s.step_adjoint(self.levels[n - a])
            else:
                s.save_state(self.tape[0])
                for n in range(a + 1, b):
                    s.step(1)
                    s.save_state(self.tape[n - a])
                for n in reversed(range(a, b)):
                    s.load_state(self.tape[n - a])
                    s.step_adjoint()
        if self.nsteps == 0:
            s.load_state(self.ckpt[0])
        return s.adjoint_initial()


class FinalKineticEnergy(torch.autograd.Function):
    """J = kinetic energy after ``nsteps`` steps from (T0, v0); gradient
    with respect to T0 (v0 is held fixed)."""

    @staticmethod
    def forward(ctx, T0, v0, solver, nsteps, checkpoint_every, ib, Z0):
        traj = Trajectory(solver, nsteps, checkpoint_every, ib)
        J = traj.forward(T0.detach(), [x.detach() for x in v0], Z0)
        ctx.traj = traj
        return torch.tensor(J, dtype=torch.float64, device=T0.device)

    @staticmethod
    def backward(ctx, gJ):
        Tb = ctx.traj.backward()[0]
        return Tb * gJ.to(Tb.device), None, None, None, None, None, None


def final_kinetic_energy(solver, T0: torch.Tensor, v0, nsteps: int, checkpoint_every: int = 20,
                         ib=None, Z0=None) -> torch.Tensor:
    """Differentiable J(T0); ``T0`` is a float64 tensor on the solver's
    device; ``ib``: immersed-body arrays as for ``Solver.set``; ``Z0``: the
    initial mixture fraction of a reacting run (held fixed)."""
    return FinalKineticEnergy.apply(T0, list(v0), solver, nsteps, checkpoint_every, ib, Z0)


class StepFn(torch.autograd.Function):
    """(T_n, v_n) after ``nsteps`` steps from (T0, v0), differentiable in
    T0 and v0: the backward pass seeds the adjoint state with the
    cotangents of T_n (which the library folds into that of H) and of v_n,
    and walks the checkpointed trajectory back
    (``Trajectory``). Outputs are float64 tensors on the solver's device."""

    @staticmethod
    def forward(ctx, T0, *args):
        v0, (solver, nsteps, checkpoint_every) = list(args[:-3]), args[-3:]
        traj = Trajectory(solver, nsteps, checkpoint_every)
        traj.forward(T0.detach(), [x.detach() for x in v0])
        g = solver.get(("T", "v"))
        ctx.traj = traj
        ctx.nv = len(v0)
        return (g["T"],) + tuple(g["v"])

    @staticmethod
    def backward(ctx, gT, *gv):
        s = ctx.traj.solver
        zero = lambda g: torch.zeros(s.shape, dtype=torch.float64, device=s.device) if g is None else \
            g.to(torch.float64).contiguous()
        seed = {"T": zero(gT), "v": [zero(g) for g in gv]}
        Tb, vb = ctx.traj.backward(seed)[:2]
        return (Tb,) + tuple(vb) + (None, None, None)


def step_fn(solver, T0: torch.Tensor, v0, nsteps: int, checkpoint_every: int = 20):
    """Differentiable (T_n, [v_n...]) from (T0, v0): float64 tensors on the
    solver's device (a Solver built with with_adjoint=True and dt > 0)."""
    out = StepFn.apply(T0, *list(v0), solver, nsteps, checkpoint_every)
    return out[0], list(out[1:])
