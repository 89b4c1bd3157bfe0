"""The Wave-ADR cycle (Algorithm 1) and the problem container.

Test infrastructure only (see the package docstring).

Readings of the paper used here (each also listed in the design notes):
* levels: l = 1 finest ... L coarsest, each axis halves per level; coarse operators are
  re-discretised with h_l = 2^(l-1) h_1 (h_1 = 1/max(n_x, n_y)) and injected n^2 and
  damping;
* smoothers: one damped Jacobi sweep before and after on level 1 (weight w[0]);
  Chebyshev(5) before and after on levels 2 and 4..L-1 (parameter alpha_l = w[l-1]);
  Chebyshev(10) on level L and return; level 3 has no smoothing, following the
  description of the wave cycle in Section 3.1 (Algorithm 1 read literally would
  run a Chebyshev post-smoother there; that form is available with
  level3_literal=True);
* the branch order of Algorithm 1 is kept (l == 1, then l == L, then l == 3);
* after the level-2 post-smoother, adr_steps ADR corrections (r, demodulate,
  ADR V-cycle, modulate-add) are applied; only the correction repeats;
* the ADR V-cycle spans adr_levels levels from level 2 down (default 3) with
  GMRES(3) smoothing on each, also the coarsest (gmres_coarse_m = 3).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .adr import adr_coefficients, adr_step
from .grid import apply_A, damping_rho, inject, kappa_level, level_size, prolong_bilinear, restrict_fw
from .smooth import (alpha_median_rule, chebyshev, default_jacobi_weight, jacobi, lambda_gershgorin)

F64 = torch.float64
C128 = torch.complex128


class Problem:
    """Discrete damped Helmholtz problem and the parameters of the Wave-ADR cycle.

    velocity: (n_y, n_x) array c(x) > 0 (n^2 = 1/c^2 on the fine grid); n_x and n_y are
              powers of two, h_1 = 1/max(n_x, n_y) (``n`` below is that maximum).
    weights:  length-L vector, w[0] = Jacobi weight, w[l-1] = Chebyshev alpha_l.
    shift:    relative imaginary shift s0 of the shifted equation (Section 4.3.2).
    cycle_shift: relative imaginary shift added inside the cycle only, so that the cycle
              is a V-cycle for a complex-shifted operator while the system keeps
              kappa (the CSL preconditioner of the comparison in Section 4.3.1 is
              cycle_shift = 0.5 with adr_steps = 0).
    phi:      fine-grid phase (n, n); may be a tensor that requires grad."""

    def __init__(self, velocity, k: float, levels: int, damping_cells: int = 16,
                 damping_strength: float = 0.5, sigma: int = 1, adr_steps: int = 8,
                 cheb_pre: int = 5, cheb_post: int = 5, cheb_coarse: int = 10,
                 gmres_m: int = 3, gmres_coarse_m: int = 3, level3_literal: bool = False,
                 weights=None, phi=None, adr_levels=3, shift: float = 0.0, cycle_shift: float = 0.0):
        vel = torch.as_tensor(np.asarray(velocity, dtype=np.float64))
        self.ny, self.nx = int(vel.shape[0]), int(vel.shape[1])
        for m in (self.nx, self.ny):
            if m & (m - 1) or m < 8:
                raise ValueError("grid sides must be powers of two >= 8")
        self.n = max(self.nx, self.ny)
        if not 2 <= levels <= int(np.log2(min(self.nx, self.ny))) - 1:
            raise ValueError("bad number of levels")
        self.k = float(k)
        self.L = int(levels)
        self.W = int(damping_cells)
        self.strength = float(damping_strength)
        self.sigma = int(sigma)
        self.shift = float(shift)
        self.cycle_shift = float(cycle_shift)
        self.adr_steps = int(adr_steps)
        self.cheb_pre, self.cheb_post, self.cheb_coarse = cheb_pre, cheb_post, cheb_coarse
        self.gmres_m, self.gmres_coarse_m = gmres_m, gmres_coarse_m
        self.level3_literal = bool(level3_literal)
        # ADR V-cycle on levels 2..LA (LA = L unless fewer ADR levels are requested)
        self.LA = self.L if adr_levels is None else min(self.L, 1 + int(adr_levels))
        if self.L >= 3 and self.LA < 2:
            raise ValueError("adr_levels must be >= 1")
        self.n2_fine = 1.0 / (vel * vel)
        self.h, self.n2, self.rho, self.kappa, self.lam = {}, {}, {}, {}, {}
        for l in range(1, self.L + 1):
            self.h[l] = float(1 << (l - 1)) / self.n
            self.n2[l] = inject(self.n2_fine, l)
            self.rho[l] = damping_rho(self.nx, l, self.W, self.ny)
            self.kappa[l] = kappa_level(self.n2[l], self.rho[l], self.k, self.strength, self.sigma,
                                        self.shift + self.cycle_shift)
            self.lam[l] = lambda_gershgorin(self.kappa[l], self.h[l])
        # the operator of the linear system (level 1); the cycle's operators add cycle_shift
        self.kappa_sys = kappa_level(self.n2[1], self.rho[1], self.k, self.strength, self.sigma, self.shift)
        self.weights = self.default_weights() if weights is None else torch.as_tensor(weights, dtype=F64)
        self.adr = {}
        self.phase_sets = []
        if phi is not None:
            self.set_phase(phi)

    def default_weights(self) -> torch.Tensor:
        """w[0] = (4-K)/(5-K) with K = k^2 max(n^2) h_1^2; w[l-1] = alpha_l by the
        median rule (lower end of the Chebyshev interval at the median of the
        constant-coefficient spectrum of A^*A with the level's mean n^2)."""
        w = np.zeros(self.L)
        w[0] = default_jacobi_weight(self.k, float(self.n2[1][1:, 1:].max()), self.h[1])
        for l in range(2, self.L + 1):
            w[l - 1] = alpha_median_rule(self.k, float(self.n2[l][1:, 1:].mean()), level_size(self.nx, l),
                                         self.lam[l], level_size(self.ny, l), self.h[l])
        return torch.as_tensor(w, dtype=F64)

    def set_weights(self, w):
        self.weights = w if isinstance(w, torch.Tensor) else torch.as_tensor(np.asarray(w, dtype=np.float64))

    def set_phase(self, phi):
        """Inject phi to the ADR levels 2..L, build their coefficients, and the
        level-2 carrier e^{+- i sigma k phi_2}."""
        phi = phi if isinstance(phi, torch.Tensor) else torch.as_tensor(np.asarray(phi))
        self.phase_sets = [self._phase_set(phi.to(F64))]
        self.use_phase(0)

    def _phase_set(self, phi):
        adr = {}
        for l in range(2, self.LA + 1):
            adr[l] = adr_coefficients(inject(phi, l), self.n2[l], self.rho[l], self.k,
                                      self.strength, self.sigma, self.h[l], self.shift + self.cycle_shift)
        arg = (self.sigma * self.k) * inject(phi, 2)
        return adr, torch.complex(torch.cos(arg), torch.sin(arg)), torch.complex(torch.cos(arg), -torch.sin(arg))

    def set_phase_factored(self, tau1, src):
        """The travel time tau = tau0 tau1 of one point source (Section 3.2.1) as the
        phase: ADR coefficients from the product-rule derivatives of
        ``eikonal.factored_derivatives`` on each ADR level (tau1 injected), and the
        carrier of tau on level 2."""
        from .eikonal import factored_adr_coefficients
        t1 = tau1 if isinstance(tau1, torch.Tensor) else torch.as_tensor(np.asarray(tau1))
        t1 = t1.to(F64)
        adr = {}
        for l in range(2, self.LA + 1):
            adr[l] = factored_adr_coefficients(inject(t1, l), src, self.n2[l], self.rho[l], self.k, self.strength,
                                               self.sigma, self.h[l], self.shift + self.cycle_shift)
        t2 = inject(t1, 2)
        Y, X = torch.meshgrid(torch.arange(t2.shape[0], dtype=F64) * self.h[2],
                              torch.arange(t2.shape[1], dtype=F64) * self.h[2], indexing="ij")
        phi2 = torch.sqrt((X - src[0]) ** 2 + (Y - src[1]) ** 2) * t2
        arg = (self.sigma * self.k) * phi2
        self.phase_sets = [(adr, torch.complex(torch.cos(arg), torch.sin(arg)),
                            torch.complex(torch.cos(arg), -torch.sin(arg)))]
        self.use_phase(0)

    def use_phase(self, m: int):
        """Makes phase set m the one the ADR correction uses (ADR coefficients and carrier)."""
        self.adr, self.carrier, self.carrier_conj = self.phase_sets[m]

    def set_rays(self, count: int = 8):
        """Wave-Ray phases (Section 3.2, the plane-wave basis of the Wave-Ray method):
        phi_m = nbar (cos theta_m x + sin theta_m y), theta_m = 2 pi (m - 1)/count,
        m = 1..count, with nbar^2 the mean of n^2 over the fine unknowns (reading: the
        paper's rays have unit slowness, |grad phi_m| = 1 on its unit-slowness medium).
        The m-th ADR correction of a cycle uses ray (m - 1) mod count; the ray equation
        is eq. ADR with phi_m (for n = nbar its reaction term is the damping term alone,
        the paper's ray equation)."""
        nbar = math.sqrt(float(self.n2_fine[1:, 1:].mean()))
        Y, X = torch.meshgrid(torch.arange(self.ny, dtype=F64) * self.h[1],
                              torch.arange(self.nx, dtype=F64) * self.h[1], indexing="ij")
        sets = []
        for m in range(count):
            th = 2.0 * math.pi * m / count
            sets.append(self._phase_set(nbar * (math.cos(th) * X + math.sin(th) * Y)))
        self.phase_sets = sets
        self.use_phase(0)

    # convenience
    def A(self, u, level: int = 1):
        """The system operator on level 1; the cycle's (re-discretised) operator below."""
        return apply_A(u, self.kappa_sys if level == 1 else self.kappa[level], self.h[level])

    def zeros(self, level: int = 1):
        return torch.zeros((level_size(self.ny, level), level_size(self.nx, level)), dtype=C128)


def wave_adr_cycle(P: Problem, level: int, g: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """One Wave-ADR cycle on level ``level`` (Algorithm 1)."""
    kap, h, w = P.kappa[level], P.h[level], P.weights
    L = P.L
    # pre-smoothing
    if level == 1:
        u = jacobi(u, g, kap, h, w[0])
    elif level == L:
        return chebyshev(u, g, kap, h, w[L - 1], P.cheb_coarse, P.lam[L])
    elif level == 3:
        pass
    else:
        u = chebyshev(u, g, kap, h, w[level - 1], P.cheb_pre, P.lam[level])
    # coarse-grid correction with zero initial guess
    rc = restrict_fw(g - apply_A(u, kap, h))
    ec = wave_adr_cycle(P, level + 1, rc, torch.zeros_like(rc))
    u = u + prolong_bilinear(ec)
    # post-smoothing
    if level == 1:
        u = jacobi(u, g, kap, h, w[0])
    elif level == 2:
        u = chebyshev(u, g, kap, h, w[1], P.cheb_post, P.lam[2])
        if P.adr_steps > 0 and L >= 3:
            if not P.phase_sets:
                raise RuntimeError("phase not set")
            for s in range(P.adr_steps):
                P.use_phase(s % len(P.phase_sets))
                u = adr_step(P, g, u)
            P.use_phase(0)
    elif level == 3 and not P.level3_literal:
        pass
    else:
        u = chebyshev(u, g, kap, h, w[level - 1], P.cheb_post, P.lam[level])
    return u


def cycle(P: Problem, g: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """C(u, g): one cycle from the fine-grid iterate u."""
    return wave_adr_cycle(P, 1, g, u)
