"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the bench.

This module only draws random numbers and evaluates initial-condition formulas
(hot spots, Fourier-mode fields, solenoidal velocity, burner geometry). It holds
none of the time-stepping arithmetic: no residuals, no equation of state, no
Poisson solve. Every array is float64 in C order with x the fastest axis, i.e.
shape (ny, nx) in 2D and (nz, ny, nx) in 3D.
"""
from .ics import (  # noqa: F401
    Case, cell_centres, taylor_green, hot_spot_tg, fourier_temperature,
    solenoidal_velocity, c1_case, c2_case, c3_case, c4_case, c5_case, make_case,
    fd_directions, variable_coefficient_problem, taylor_couette_case,
    heated_cavity_case, double_tsuji_case, tanh_stretched_faces, sine_stretched_faces,
    reacting_periodic_case,
)
