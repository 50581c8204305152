"""Plain FP64 CPU oracle of the low-Mach predictor-corrector step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, links or runs
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark do. It shares no code with the HIP library; the two meet only in the
seeded input generators of ``workloads``.

Scope: one full time step of the fractional-step method of Severino et al.
(section 3): AB2 predictor and AM2 corrector for mixture fraction Z, excess
enthalpy H and momentum (section 3.1, Eq 3.1-3.19), the collocated flux
discretisation (section 3.2, Eq 3.20-3.26), the zero-mean pressure Poisson
problem (section 3.3), the penalised immersed boundary with a mass source
(section 3.4, Eq 3.29-3.33), the regularised flame-sheet temperature (section
3.5, Eq 3.34-3.42) and ghost-cell boundary conditions (section 3.6,
Eq 3.43-3.46), on uniform grids or on grids stretched per direction (the
operators of Eq 3.20-3.22 with local spacings; the tanh stretching of
Eq 4.18). The Poisson problem is solved exactly (Fourier / cosine transforms
on uniform grids whose sides are periodic or zero-flux, sparse LU of the
augmented matrix otherwise, volume-weighted on stretched grids), which gives
the zero-mean solution of the augmented-matrix method of section 3.3.

Arrays are float64 in C order, x fastest: (ny, nx) or (nz, ny, nx).
Face arrays along direction d have n_d + 1 entries along that axis: entry f is
the face between cells f-1 and f.
"""
from .flame import FlameParams, theta_eps, le_eps, n_eps, f_eps, f_tilde, temperature, enthalpy_from_T  # noqa: F401
from .grid import Grid, fill_ghosts, tanh_faces  # noqa: F401
from .poisson import PoissonSolver, beta_inv_rho, laplacian  # noqa: F401
from .step import Params, State, Oracle  # noqa: F401
