"""MI355X (gfx950) low-Mach predictor-corrector step (Severino et al., section 3).

``Solver`` wraps the C ABI of ``liblowmach.so``: PyTorch provides the device
workspace and the stream; every step of the method runs in the HIP library.
Arrays are float64, C order, x fastest: (ny, nx) or (nz, ny, nx); face fluxes
F_d carry n_d + 1 entries along d.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import lib as _L

__all__ = ["Solver", "LowMachError", "project", "project_static"]
LowMachError = _L.LowMachError


def _check(lib, ctx, status):
    if status != _L.LM_OK:
        msg = lib.lm_last_error(ctx).decode()
        raise _L.LowMachError(status, msg)


class _Marshal:
    """Keeps the arrays of one call alive and yields (pointer, mem)."""

    def __init__(self, torch, device):
        self.torch = torch
        self.device = device
        self.keep = []
        self.mem = None

    def ptr(self, a, dtype=np.float64):
        if a is None:
            return None
        t = self.torch
        if isinstance(a, t.Tensor):
            if a.device.type != "cuda":
                a = a.detach().numpy()
            else:
                tt = t.float64 if dtype == np.float64 else t.uint8
                a = a.detach().to(device=self.device, dtype=tt).contiguous()
                self._mem(_L.LM_DEVICE)
                self.keep.append(a)
                return a.data_ptr()
        arr = np.ascontiguousarray(a, dtype=dtype)
        self._mem(_L.LM_HOST)
        self.keep.append(arr)
        return arr.ctypes.data

    def _mem(self, m):
        if self.mem is None:
            self.mem = m
        elif self.mem != m:
            raise ValueError("mix of host and device arrays in one call")


class Solver:
    """One simulation context on one GPU.

    Parameters follow ``lm_params`` of include/lowmach.h. ``bc`` is a list per
    direction of (low, high) side kinds: "periodic", "slip", "noslip",
    "inflow", "outflow". ``faces`` (optional) gives per direction None or the
    n + 1 face coordinates of a stretched direction (``lm_grid.faces``).
    """

    def __init__(self, n: Sequence[int], L: Sequence[float], bc=None, *, Re: float, Pr: float = 0.7,
                 sigma: float = 0.7, inv_Fr2: float = 0.0, reacting: bool = False, S: float = 1.0,
                 qs: float = 1.0, eps: float = 0.5, tol: float = 1e-3, Le_F: float = 1.0, Le_O: float = 1.0,
                 Da_ib: float = 1.0, p0: float = 1.0, dt: float = 0.0, cfl: float = 0.2,
                 precision: str = "fp64", poisson_rtol: float = 1e-10, poisson_maxit: int = 200,
                 mg_nu: int = 2, with_ib: bool = False, with_adjoint: bool = False,
                 variable_coefficient: bool = False, p0_closed: bool = False, gamma: float = 1.4,
                 sutherland_C: float = 0.0, dt_tol: float = 0.0, faces=None, device: str = "cuda:0",
                 stream=None):
        import torch
        self.torch = torch
        self.lib = _L.load()
        ndim = len(n)
        self.ndim = ndim
        self.n = tuple(int(q) for q in n)
        self.shape = tuple(reversed(self.n))
        if bc is None:
            bc = [("periodic", "periodic")] * ndim
        g = _L.lm_grid()
        g.ndim = ndim
        for d in range(3):
            g.n[d] = self.n[d] if d < ndim else 1
            g.L[d] = float(L[d]) if d < ndim else 1.0
            for s in range(2):
                g.bc[d][s] = _L.SIDE[bc[d][s]] if d < ndim else 0
        self._faces = []                  # host copies alive through lm_init_grid
        for d in range(ndim):
            f = None if faces is None else faces[d]
            if f is not None:
                f = np.ascontiguousarray(f, dtype=np.float64)
                self._faces.append(f)
                g.faces[d] = f.ctypes.data
        p = _L.lm_params(Re=Re, Pr=Pr, sigma=sigma, inv_Fr2=inv_Fr2, reacting=int(reacting), S=S, qs=qs,
                         eps=eps, tol=tol, Le_F=Le_F, Le_O=Le_O, Da_ib=Da_ib, p0=p0, dt=dt, cfl=cfl,
                         precision=_L.PRECISION[precision],
                         poisson_rtol=poisson_rtol, poisson_maxit=poisson_maxit, mg_nu=mg_nu,
                         with_ib=int(with_ib), with_adjoint=int(with_adjoint),
                         poisson_beta=_L.LM_BETA_INV_RHO if variable_coefficient else _L.LM_BETA_ONE,
                         p0_closed=int(p0_closed), gamma=gamma, sutherland_C=sutherland_C,
                         dt_tol=dt_tol)
        self.grid, self.params = g, p
        self.device = torch.device(device)
        size = C.c_size_t()
        _check(self.lib, None, self.lib.lm_workspace_size(C.byref(g), C.byref(p), C.byref(size)))
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        _check(self.lib, None, self.lib.lm_init_grid(C.byref(g), C.byref(p), C.c_void_p(self.workspace.data_ptr()),
                                                     size.value, C.c_void_p(self.stream.cuda_stream),
                                                     C.byref(ctx)))
        self.ctx = ctx
        self.stats = None

    # ------------------------------------------------------------------
    def set(self, T=None, v=None, Z=None, H=None, P=None, F=None, ib: Optional[dict] = None, level: int = 0):
        """Set the state (level 0, time n), or after it the fields of time
        n - 1 (level 1: T or H, v, optionally Z and F), from which the
        library forms the history of the next AB2 / BDF2 step."""
        m = _Marshal(self.torch, self.device)
        f = _L.lm_fields()
        f.T = m.ptr(T)
        f.H = m.ptr(H)
        f.Z = m.ptr(Z)
        f.P = m.ptr(P)
        for d in range(self.ndim):
            f.v[d] = m.ptr(v[d])
            if F is not None:
                f.F[d] = m.ptr(F[d])
        ibs = None
        if ib is not None:
            ibs = _L.lm_ib()
            ibs.chi = m.ptr(ib.get("chi"), np.uint8)
            for d in range(self.ndim):
                vib = ib.get("v_ib")
                ibs.v_ib[d] = m.ptr(vib[d]) if vib is not None else None
            ibs.Z_ib = m.ptr(ib.get("Z_ib"))
            ibs.H_ib = m.ptr(ib.get("H_ib"))
            ibs.S_m = m.ptr(ib.get("Sm"))
        mem = m.mem if m.mem is not None else _L.LM_HOST
        _check(self.lib, self.ctx, self.lib.lm_set_fields(self.ctx, int(level), C.byref(f),
                                                          C.byref(ibs) if ibs is not None else None, mem))

    def set_side(self, d: int, side: int, v=None, Z=None, H=None, F=None, wall=None):
        """Boundary data of an inflow side (``wall`` flags the cells of the
        side under a solid footprint: zero-gradient Z and H there), or the
        wall value H of an isothermal slip / no-slip wall."""
        m = _Marshal(self.torch, self.device)
        s = _L.lm_side_data()
        if v is not None:
            for q in range(self.ndim):
                s.v[q] = m.ptr(v[q])
        s.Z, s.H, s.F = m.ptr(Z), m.ptr(H), m.ptr(F)
        s.wall = m.ptr(wall, np.uint8)
        mem = m.mem if m.mem is not None else _L.LM_HOST
        _check(self.lib, self.ctx, self.lib.lm_set_side(self.ctx, d, side, C.byref(s), mem))

    def step(self, nsteps: int = 1) -> dict:
        st = _L.lm_step_stats()
        _check(self.lib, self.ctx, self.lib.lm_step(self.ctx, nsteps, C.byref(st)))
        self.stats = dict(steps=st.steps, dt=st.dt, time=st.time, poisson_iters=list(st.poisson_iters),
                          poisson_relres=list(st.poisson_relres), compat=list(st.compat),
                          total_poisson_iters=st.total_poisson_iters, p0=st.p0, pc_err=st.pc_err,
                          pc_err_used=bool(st.pc_err_used))
        return self.stats

    def get(self, names=("rho", "v", "H", "T", "P", "F", "Z"), device: bool = True, predicted: bool = False) -> dict:
        """Fields of the current level, or with ``predicted`` those of the
        last step's predicted level (its starred fields and P*)."""
        t = self.torch
        out = {}
        f = _L.lm_fields()
        keep = []

        def alloc(shape):
            a = t.empty(shape, dtype=t.float64, device=self.device) if device else np.empty(shape)
            keep.append(a)
            return a, (a.data_ptr() if device else a.ctypes.data)

        for name in names:
            if name == "v":
                vs = []
                for d in range(self.ndim):
                    a, p = alloc(self.shape)
                    f.v[d] = p
                    vs.append(a)
                out["v"] = vs
            elif name == "F":
                fs = []
                for d in range(self.ndim):
                    shp = list(self.shape)
                    shp[self.ndim - 1 - d] += 1
                    a, p = alloc(tuple(shp))
                    f.F[d] = p
                    fs.append(a)
                out["F"] = fs
            elif name == "Z" and not self.params.reacting:
                continue
            else:
                a, p = alloc(self.shape)
                setattr(f, name, p)
                out[name] = a
        level = _L.LM_LEVEL_PREDICTED if predicted else 0
        _check(self.lib, self.ctx, self.lib.lm_get_fields(self.ctx, level, C.byref(f),
                                                          _L.LM_DEVICE if device else _L.LM_HOST))
        return out

    @property
    def dt(self) -> float:
        v = C.c_double()
        _check(self.lib, self.ctx, self.lib.lm_get_dt(self.ctx, C.byref(v)))
        return v.value

    def project(self, b, rtol: float = 0.0, rho=None):
        """Solve A P = b (zero-mean P, mean(b) removed) on this grid; with
        ``rho`` the variable-coefficient form div(grad P / rho) = b (needs
        ``variable_coefficient=True``). ``rho`` lives where ``b`` does."""
        m = _Marshal(self.torch, self.device)
        a = _L.lm_project_args()
        a.b = m.ptr(b)
        if rho is not None:
            a.rho = m.ptr(rho)
        if m.mem == _L.LM_DEVICE:
            P = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
            a.P = P.data_ptr()
        else:
            P = np.empty(self.shape)
            a.P = P.ctypes.data
        a.mem = m.mem
        a.rtol = rtol
        _check(self.lib, self.ctx, self.lib.lm_project(self.ctx, C.byref(a)))
        if m.mem == _L.LM_DEVICE:
            self.torch.cuda.current_stream(self.device).synchronize()
        return P, dict(iters=a.iters, relres=a.relres, mean_b=a.mean_b)

    # ------------------------------------------------------------------
    # checkpoint / restart
    def state_size(self) -> int:
        n = C.c_size_t()
        _check(self.lib, self.ctx, self.lib.lm_state_size(self.ctx, C.byref(n)))
        return n.value

    def save_state(self, buf=None):
        """Copy the complete state into a device byte tensor (allocated when
        ``buf`` is None) and return it."""
        if buf is None:
            buf = self.torch.empty(self.state_size(), dtype=self.torch.uint8, device=self.device)
        _check(self.lib, self.ctx, self.lib.lm_save_state(self.ctx, C.c_void_p(buf.data_ptr())))
        return buf

    def load_state(self, buf):
        _check(self.lib, self.ctx, self.lib.lm_load_state(self.ctx, C.c_void_p(buf.data_ptr())))

    # ------------------------------------------------------------------
    # adjoint (2D or 3D; periodic, wall, inflow and high-side outflow sides; FP64; needs with_adjoint=True)
    def kinetic_energy(self) -> float:
        v = C.c_double()
        _check(self.lib, self.ctx, self.lib.lm_kinetic_energy(self.ctx, C.byref(v)))
        return v.value

    def adjoint_seed_ke(self):
        _check(self.lib, self.ctx, self.lib.lm_adjoint_seed_ke(self.ctx))

    def adjoint_set(self, H=None, v=None, F=None, rho_prev=None, R_H=None, R_v=None, T=None, Z=None, R_Z=None):
        """Set the adjoint state; ``T``, a cotangent of the temperature, is
        folded into those of H (and Z in reacting flow) by the library."""
        m = _Marshal(self.torch, self.device)
        a = _L.lm_adjoint()
        a.H, a.rho_prev, a.R_H, a.T = m.ptr(H), m.ptr(rho_prev), m.ptr(R_H), m.ptr(T)
        a.Z, a.R_Z = m.ptr(Z), m.ptr(R_Z)
        for d in range(self.ndim):
            a.v[d] = m.ptr(v[d]) if v is not None else None
            a.F[d] = m.ptr(F[d]) if F is not None else None
            a.R_v[d] = m.ptr(R_v[d]) if R_v is not None else None
        mem = m.mem if m.mem is not None else _L.LM_HOST
        _check(self.lib, self.ctx, self.lib.lm_adjoint_set(self.ctx, C.byref(a), mem))

    def adjoint_get(self, device: bool = True) -> dict:
        """Current adjoint state: H, v, F (faces as in ``get``; the low face
        of cell 0 of a periodic direction is the duplicate of face n and
        reads 0), rho_prev, R_H, R_v, and Z, R_Z in reacting flow."""
        t = self.torch
        keep = []

        def alloc(shape):
            x = t.empty(shape, dtype=t.float64, device=self.device) if device else np.empty(shape)
            keep.append(x)
            return x, (x.data_ptr() if device else x.ctypes.data)

        a = _L.lm_adjoint()
        out = {}
        names = ("H", "rho_prev", "R_H") + (("Z", "R_Z") if self.params.reacting else ())
        for name in names:
            x, p = alloc(self.shape)
            setattr(a, name, p)
            out[name] = x
        out["v"], out["F"], out["R_v"] = [], [], []
        for d in range(self.ndim):
            x, a.v[d] = alloc(self.shape)
            out["v"].append(x)
            x, a.R_v[d] = alloc(self.shape)
            out["R_v"].append(x)
            shp = list(self.shape)
            shp[self.ndim - 1 - d] += 1
            x, a.F[d] = alloc(tuple(shp))
            out["F"].append(x)
        _check(self.lib, self.ctx, self.lib.lm_adjoint_get(self.ctx, C.byref(a),
                                                           _L.LM_DEVICE if device else _L.LM_HOST))
        return out

    def step_adjoint(self, levels=None):
        """One step back; ``levels``: the buffer ``save_step_levels`` filled
        right after stepping from the current state (no recompute)."""
        if levels is None:
            _check(self.lib, self.ctx, self.lib.lm_step_adjoint(self.ctx))
        else:
            _check(self.lib, self.ctx, self.lib.lm_step_adjoint_levels(self.ctx, C.c_void_p(levels.data_ptr())))

    def step_levels_size(self) -> int:
        n = C.c_size_t()
        _check(self.lib, self.ctx, self.lib.lm_step_levels_size(self.ctx, C.byref(n)))
        return n.value

    def save_step_levels(self, buf=None):
        """The last step's predicted and new levels into a device uint8
        tensor of ``step_levels_size()`` bytes (allocated when not given)."""
        if buf is None:
            buf = self.torch.empty(self.step_levels_size(), dtype=self.torch.uint8, device=self.device)
        _check(self.lib, self.ctx, self.lib.lm_save_step_levels(self.ctx, C.c_void_p(buf.data_ptr())))
        return buf

    def adjoint_initial(self, device: bool = True):
        """Cotangents (T0_bar, [v0_bar...]) of the initial fields given to
        ``set(T=..., v=...)``, and Z0_bar as a third entry in reacting flow
        (``set(T=..., v=..., Z=...)``); the forward state must be that
        initial state."""
        t = self.torch
        mk = (lambda: t.empty(self.shape, dtype=t.float64, device=self.device)) if device else \
            (lambda: np.empty(self.shape))
        Tb = mk()
        vb = [mk() for _ in range(self.ndim)]
        Zb = mk() if self.params.reacting else None
        ptr = (lambda x: x.data_ptr()) if device else (lambda x: x.ctypes.data)
        arr = (C.c_void_p * 3)(*([ptr(x) for x in vb] + [None] * (3 - self.ndim)))
        _check(self.lib, self.ctx, self.lib.lm_adjoint_initial(self.ctx, C.c_void_p(ptr(Tb)), arr,
                                                               C.c_void_p(ptr(Zb)) if Zb is not None else None,
                                                               _L.LM_DEVICE if device else _L.LM_HOST))
        return (Tb, vb) if Zb is None else (Tb, vb, Zb)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def project(b, L, bc=None, rho=None, rtol: float = 1e-12, precision: str = "fp64", maxit: int = 400,
            device: str = "cuda:0"):
    """One-off pressure solve: the zero-mean P with A P = b on a grid of
    b's shape (C order, x fastest) and lengths L, sides ``bc`` as for
    ``Solver``; with ``rho`` the variable-coefficient form
    div(grad P / rho) = b. Builds a context for the call (use
    ``Solver.project`` for repeated solves). Returns (P, info)."""
    shape = tuple(np.shape(b))
    n = tuple(reversed(shape))
    s = Solver(n, L, bc=bc, Re=1.0, dt=1.0, precision=precision, poisson_rtol=rtol, poisson_maxit=maxit,
               variable_coefficient=rho is not None, device=device)
    try:
        return s.project(b, rho=rho)
    finally:
        s.close()


def project_static(b, L, P=None, bc=None, rtol: float = 1e-12, precision: str = "fp64", maxit: int = 400,
                   mg_nu: int = 2, stream=None):
    """The pressure solve of ``project`` through ``lm_project_static``: no
    context and no device allocation by the library (its arrays live in a
    static 64 MiB device buffer per GPU; calls on one GPU must not overlap).
    ``b`` and ``P`` (the caller's output, same shape; None: only the info)
    are both device tensors or both host arrays. Returns the info dict."""
    lib = _L.load()
    shape = tuple(np.shape(b))
    ndim = len(shape)
    n = tuple(reversed(shape))
    if bc is None:
        bc = [("periodic", "periodic")] * ndim
    g = _L.lm_grid()
    g.ndim = ndim
    for d in range(3):
        g.n[d] = n[d] if d < ndim else 1
        g.L[d] = float(L[d]) if d < ndim else 1.0
        for q in range(2):
            g.bc[d][q] = _L.SIDE[bc[d][q]] if d < ndim else 0
    p = _L.lm_params(Re=1.0, Pr=0.7, sigma=0.7, qs=1.0, S=1.0, eps=0.5, tol=1e-3, Le_F=1.0, Le_O=1.0, Da_ib=1.0,
                     p0=1.0, dt=1.0, cfl=0.2, precision=_L.PRECISION[precision], poisson_rtol=rtol,
                     poisson_maxit=maxit, mg_nu=mg_nu)
    a = _L.lm_project_args()
    import torch
    if isinstance(b, torch.Tensor) and b.device.type == "cuda":
        if not (b.dtype == torch.float64 and b.is_contiguous()):
            raise ValueError("b must be a contiguous float64 tensor")
        if P is not None and not (P.device == b.device and P.dtype == torch.float64 and P.is_contiguous()
                                  and tuple(P.shape) == shape):
            raise ValueError("P must be a contiguous float64 tensor of b's shape on b's device")
        a.b, a.P, a.mem = b.data_ptr(), (P.data_ptr() if P is not None else None), _L.LM_DEVICE
        st = stream if stream is not None else torch.cuda.current_stream(b.device)
        sp = st.cuda_stream
    else:
        b = np.ascontiguousarray(b, dtype=np.float64)
        if P is not None and not (isinstance(P, np.ndarray) and P.dtype == np.float64 and P.flags.c_contiguous
                                  and P.shape == shape):
            raise ValueError("P must be a C-contiguous float64 array of b's shape")
        a.b, a.P, a.mem = b.ctypes.data, (P.ctypes.data if P is not None else None), _L.LM_HOST
        sp = stream.cuda_stream if stream is not None else None
    a.rtol = rtol
    status = lib.lm_project_static(C.byref(g), C.byref(p), C.c_void_p(sp), C.byref(a))
    _check(lib, None, status)
    return dict(iters=a.iters, relres=a.relres, mean_b=a.mean_b)
