"""Plain, slow, FP64 CPU oracle of the Wave-ADR cycle (test infrastructure only).

This package is the independent reference that the HIP path is checked against.
Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import it; the library never does.  It shares no code with the HIP path: the
two meet only through the seeded inputs of ``helm_inputs``.

Everything is torch CPU float64 / complex128 written with slicing, so that the
oracle is differentiable by autograd (the reference gradient of the unrolled
cycles) and each function can be checked against the paper by eye.

Notation: k is the paper's angular frequency omega, n2 = 1/c^2 is the squared
slowness s^2, phi is the paper's phase tau, sigma = +1 selects the carrier
e^{+i k phi} (sigma = -1 gives the paper's printed signs, which are the complex
conjugate of every operator).

Grids are n_x columns by n_y rows of nodes (powers of two; square domains have
n_x = n_y), spacing h = 1/max(n_x, n_y) on both axes, each axis halved per level
(the non-square domains of Section 4.3.2 use the same method on such grids).

Modules
-------
grid      levels, damping, Helmholtz operator, full weighting, bilinear prolongation
smooth    damped Jacobi, Chebyshev semi-iteration on the normal equations, default weights
adr       ADR coefficients, upwind ADR operator, GMRES(m), ADR V-cycle, ADR correction
cycle     the Wave-ADR cycle (Algorithm 1) and the problem container
solve     FGMRES(20) right-preconditioned by one cycle
grad      loss after K unrolled cycles and its gradient (autograd and finite differences)
eikonal   factored eikonal travel time (plain C, fast sweeping) and the product-rule
          phase derivatives of the ADR coefficients

Dense assemblies of A, R and M used by the pins live in the tests themselves, so
that they stay independent of this package.
"""
from .grid import (level_size, damping_rho, kappa_level, apply_A, apply_Astar, restrict_fw,
                   prolong_bilinear, inject, cnorm, cdot)
from .smooth import (jacobi, chebyshev, lambda_gershgorin, default_jacobi_weight, alpha_median_rule,
                     alpha_median_rule_1d)
from .adr import (phase_derivatives, adr_coefficients, apply_M, gmres, adr_vcycle, adr_step)
from .cycle import Problem, wave_adr_cycle
from .solve import fgmres
from .grad import loss_after_cycles, grad_autograd

__all__ = [
    "level_size", "damping_rho", "kappa_level", "apply_A", "apply_Astar", "restrict_fw",
    "prolong_bilinear", "inject", "cnorm", "cdot", "jacobi", "chebyshev", "lambda_gershgorin",
    "default_jacobi_weight", "alpha_median_rule", "alpha_median_rule_1d", "phase_derivatives",
    "adr_coefficients", "apply_M", "gmres", "adr_vcycle", "adr_step", "Problem",
    "wave_adr_cycle", "fgmres", "loss_after_cycles", "grad_autograd",
]
