"""Smoothers of the wave cycle: damped Jacobi and Chebyshev semi-iteration.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .grid import apply_A, apply_Astar


def jacobi(u, g, kappa, h, w0):
    """One damped Jacobi sweep, error matrix I - w0 D^{-1} A (Section 3.1.1, eq. sjac).

    D = 4/h^2 - kappa is the diagonal of A; the ring stays zero because the
    residual is zero there."""
    d = 4.0 / (h * h) - kappa
    return u + w0 * (g - apply_A(u, kappa, h)) / d


def lambda_gershgorin(kappa, h) -> float:
    """Upper bound of the spectrum of A^* A: (max |4/h^2 - kappa| + 4/h^2)^2 over the
    unknowns (row-sum bound on |A|).  The paper leaves lambda_max unspecified."""
    d = torch.abs(4.0 / (h * h) - kappa[1:, 1:])
    return float((d.max().item() + 4.0 / (h * h)) ** 2)


def chebyshev(u, g, kappa, h, alpha, m, lam):
    """m steps of Chebyshev semi-iteration on the normal equations A^*A u = A^*g
    (Section 3.1.1, eq. cheb): the degree-m error polynomial p with p(0) = 1 that
    minimises max |p| on [lam/alpha, lam].

    Three-term form (Chebyshev acceleration, Saad, Iterative Methods for Sparse
    Linear Systems, Alg. 12.1) with theta = (lam + lam/alpha)/2 (centre) and
    dc = (lam - lam/alpha)/2 (half-width); the rho recursion is written as
    rho' = dc/(2 theta - dc rho), so that alpha = 1 (dc = 0) gives m Richardson
    steps u += A^*(g - A u)/lam, the limit of the same polynomial.
    ``alpha`` may be a float or a 0-d tensor (autograd)."""
    b = lam
    a = lam / alpha
    theta = 0.5 * (b + a)
    dc = 0.5 * (b - a)
    r = apply_Astar(g - apply_A(u, kappa, h), kappa, h)
    rho = dc / theta
    d = r / theta
    for t in range(1, m + 1):
        u = u + d
        if t < m:
            r = r - apply_Astar(apply_A(d, kappa, h), kappa, h)
            den = 2.0 * theta - dc * rho
            rho_new = dc / den
            d = (rho_new * rho) * d + (2.0 / den) * r
            rho = rho_new
    return u


def default_jacobi_weight(k: float, n2max: float, h: float) -> float:
    """2-D analogue of the paper's optimal 1-D damping (2 - k^2h^2)/(3 - k^2h^2)
    (Section 3.1.1): balancing the extreme high-frequency multipliers of the 2-D
    symbol gives (4 - K)/(5 - K), K = k^2 max(n^2) h^2."""
    K = k * k * n2max * h * h
    return (4.0 - K) / (5.0 - K)


def alpha_median_rule_1d(k: float, N: int) -> float:
    """alpha such that lambda_max/alpha is the median eigenvalue of A^*A for the
    1-D model problem with N interior nodes, h = 1/(N+1) (Section 3.1.1; the
    eigenvalues are those of eq. eigs)."""
    h = 1.0 / (N + 1)
    j = np.arange(1, N + 1)
    lam = 4.0 / h**2 * np.sin(j * np.pi * h / 2) ** 2 - k * k
    l2 = lam**2
    return float(l2.max() / np.median(l2))


def alpha_median_rule(k: float, n2mean: float, nl: int, lam_bound: float, nly: int | None = None,
                      h: float | None = None) -> float:
    """2-D default for the Chebyshev parameter on a level with n_l columns and nly rows
    of nodes (nly = n_l by default) and spacing h (1/max(n_l, nly) by default):
    alpha = lam_bound / median |sigma_ab|^2 where sigma_ab = (4/h^2)(sin^2(pi a/(2 n_l))
    + sin^2(pi b/(2 nly))) - k^2 n2mean over the Dirichlet sine modes 1 <= a < n_l,
    1 <= b < nly, so that the lower end lam_bound/alpha of the interval sits at the
    median of the spectrum of A^*A (the paper's criterion for alpha, Section 3.1.1).
    ``lam_bound`` is the Gershgorin bound actually used as the upper end."""
    nly = nl if nly is None else nly
    h = 1.0 / max(nl, nly) if h is None else h
    sx = np.sin(np.arange(1, nl) * math.pi / (2.0 * nl)) ** 2
    sy = np.sin(np.arange(1, nly) * math.pi / (2.0 * nly)) ** 2
    sig = 4.0 / (h * h) * (sy[:, None] + sx[None, :]) - k * k * n2mean
    med = float(np.median((sig * sig).ravel()))
    return max(1.0, lam_bound / med)
