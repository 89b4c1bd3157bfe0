"""Grids, damping, the discrete Helmholtz operator and the transfer operators.

Test infrastructure only (see the package docstring).

Grid: level l has n_l = n / 2^(l-1) stored nodes per side and h_l = 1/n_l.
Stored node (i, j) is at (x, y) = (j h_l, i h_l); unknowns are 1 <= i, j <= n_l - 1,
the ring i or j in {0, n_l} is a zero Dirichlet boundary (index n_l is not
stored).  Coarse node (I, J) coincides with fine node (2I, 2J).
"""
from __future__ import annotations

import torch

F64 = torch.float64
C128 = torch.complex128


def level_size(n: int, level: int) -> int:
    """n_l = n / 2^(l-1), l = 1 is the finest level (Algorithm 1)."""
    return n >> (level - 1)


def inject(fine: torch.Tensor, level: int) -> torch.Tensor:
    """Injection of a fine-grid field to level l: value at fine node (2^(l-1) I, 2^(l-1) J)."""
    s = 1 << (level - 1)
    return fine[::s, ::s].clone()


def damping_rho(n: int, level: int, cells: int) -> torch.Tensor:
    """Sponge ramp rho in [0, 1] at the nodes of level l.

    The damping mask grows from 0 inside the domain to its full value at the
    boundary over a layer of ``cells`` fine cells (Section 2, the damped
    equation).  Reading: linear ramp r(t) = max(0, 1 - min(t, n - t)/W) in fine
    index units per axis, combined by max over the two axes, injected to coarse
    levels."""
    nl = level_size(n, level)
    t = torch.arange(nl, dtype=F64) * (n // nl)
    r = torch.clamp(1.0 - torch.minimum(t, n - t) / cells, min=0.0)
    return torch.maximum(r[:, None], r[None, :])


def kappa_level(n2_l: torch.Tensor, rho_l: torch.Tensor, k: float, strength: float,
                sigma: int, shift: float = 0.0) -> torch.Tensor:
    """kappa = k^2 n^2 (1 + i sigma (delta + s0)), delta = strength * rho^2.

    The damped equation (Section 2) adds i*omega*gamma/c^2 to -Delta - omega^2/c^2;
    with gamma/omega = delta this is -kappa with sigma = -1 (paper's sign) or the
    conjugate with sigma = +1.  The shifted equation (Section 4.3.2) adds
    i gamma_0 u with gamma_0 = 0.01 k(x)^2; reading: k(x) = k n(x) is the local
    wavenumber, so the shift is the relative term s0 = gamma_0 / k(x)^2 (0.01 there)."""
    delta = strength * rho_l * rho_l + shift
    return (k * k) * n2_l * (1.0 + 1j * sigma * delta)


def _shift(u: torch.Tensor, di: int, dj: int) -> torch.Tensor:
    """v[i, j] = u[i + di, j + dj], zero outside the stored array (the index-n ring)."""
    n0, n1 = u.shape
    out = torch.zeros_like(u)
    i0, i1 = max(0, -di), min(n0, n0 - di)
    j0, j1 = max(0, -dj), min(n1, n1 - dj)
    out[i0:i1, j0:j1] = u[i0 + di:i1 + di, j0 + dj:j1 + dj]
    return out


def _mask_ring(v: torch.Tensor) -> torch.Tensor:
    m = torch.ones(v.shape, dtype=F64)
    m[0, :] = 0.0
    m[:, 0] = 0.0
    return v * m


def laplacian(u: torch.Tensor, h: float) -> torch.Tensor:
    """-Delta_h u with the 5-point stencil (1/h^2)[0 -1 0; -1 4 -1; 0 -1 0] (Section 2)."""
    nb = _shift(u, -1, 0) + _shift(u, 1, 0) + _shift(u, 0, -1) + _shift(u, 0, 1)
    return _mask_ring((4.0 * u - nb) / (h * h))


def apply_A(u: torch.Tensor, kappa: torch.Tensor, h: float) -> torch.Tensor:
    """A u = -Delta_h u - kappa u at the unknowns, zero on the ring (Section 2 stencil)."""
    return laplacian(u, h) - _mask_ring(kappa * u)


def apply_Astar(u: torch.Tensor, kappa: torch.Tensor, h: float) -> torch.Tensor:
    """A^* u: A is complex symmetric, so A^* is the same stencil with conj(kappa)."""
    return laplacian(u, h) - _mask_ring(torch.conj(kappa) * u)


def restrict_fw(r: torch.Tensor) -> torch.Tensor:
    """Full weighting (1/16)[1 2 1; 2 4 2; 1 2 1] at stride 2 (Section 3.1.2, Section 3.3).

    r_c(I, J) = (1/16)[4 r(2I,2J) + 2 (r(2I+-1,2J) + r(2I,2J+-1)) + sum r(2I+-1,2J+-1)]
    for 1 <= I, J <= n_c - 1; zero on the coarse ring."""
    n = r.shape[0]
    nc = n // 2
    ev = slice(2, n, 2)       # fine rows/cols 2I,   I = 1..nc-1
    lo = slice(1, n - 1, 2)   # fine rows/cols 2I-1
    hi = slice(3, n, 2)       # fine rows/cols 2I+1
    c = r[ev, ev]
    ud = r[lo, ev] + r[hi, ev] + r[ev, lo] + r[ev, hi]
    dg = r[lo, lo] + r[lo, hi] + r[hi, lo] + r[hi, hi]
    out = torch.zeros((nc, nc), dtype=r.dtype)
    out[1:, 1:] = (4.0 * c + 2.0 * ud + dg) / 16.0
    return out


def prolong_bilinear(ec: torch.Tensor) -> torch.Tensor:
    """Bilinear interpolation, the stride-2 transposed convolution with
    (1/4)[1 2 1; 2 4 2; 1 2 1] (Section 3.3); equals 4 R^T.

    Even-even fine nodes copy the coarse value, edge midpoints average 2 coarse
    neighbours, cell centres average 4.  Coarse ring values are zero."""
    nc = ec.shape[0]
    n = 2 * nc
    ep = torch.zeros((nc + 1, nc + 1), dtype=ec.dtype)
    ep[:nc, :nc] = ec
    ep[0, :] = 0.0
    ep[:, 0] = 0.0
    a = ep[:nc, :nc]
    b = ep[1:, :nc]  # (I+1, J)
    c = ep[:nc, 1:]  # (I, J+1)
    d = ep[1:, 1:]  # (I+1, J+1)
    out = torch.zeros((n, n), dtype=ec.dtype)
    out[0::2, 0::2] = a
    out[1::2, 0::2] = 0.5 * (a + b)
    out[0::2, 1::2] = 0.5 * (a + c)
    out[1::2, 1::2] = 0.25 * (a + b + c + d)
    return out


def cdot(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """<a, b> = sum conj(a) b."""
    return torch.sum(torch.conj(a) * b)


def cnorm(a: torch.Tensor) -> torch.Tensor:
    """Euclidean 2-norm over all stored entries (the ring is zero)."""
    return torch.sqrt(torch.sum(a.real * a.real + a.imag * a.imag))
