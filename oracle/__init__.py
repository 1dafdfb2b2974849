"""CPU oracle for the nested-mesh convolution method (FP64, NumPy/SciPy).

TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  It shares no code with the HIP library and
never imports it.

Parity pins: every function here is checked in tests/test_oracle_*.py
against facts fixed by the paper or by mathematics (brute force, closed
forms, invariants, an independent quadrature); see those tests.
"""
from .nested import (BETA, cell_centres, child_region, green_periodic, hole,  # noqa: F401
                     kernel_value, level_spacing, potential_at, potential_direct,
                     potential_fft, prolong, prolong_trilinear, restrict_cascade,
                     solve, solve_points, acceleration,
                     doubled_potential, quadrupled_potential, scaled_potential_at,
                     solve_modified)
from . import analytic  # noqa: F401
