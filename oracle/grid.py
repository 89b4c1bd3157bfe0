"""Grids, damping, the discrete Helmholtz operator and the transfer operators.

Test infrastructure only (see the package docstring).

Grid: the fine grid has n_x = 2^a columns and n_y = 2^b rows of stored nodes (square
domains: n_x = n_y = n), spacing h_1 = 1/max(n_x, n_y) in both directions, so the longer
side of the domain has unit length.  Level l has n_x/2^(l-1) x n_y/2^(l-1) stored nodes
and h_l = 2^(l-1) h_1.  Stored node (i, j) is at (x, y) = (j h_l, i h_l); unknowns are
1 <= i <= n_y,l - 1 and 1 <= j <= n_x,l - 1, the ring i in {0, n_y,l} or j in {0, n_x,l}
is a zero Dirichlet boundary (the last index of each axis is not stored).  Arrays are
(rows, columns) = (n_y,l, n_x,l).  Coarse node (I, J) coincides with fine node (2I, 2J).
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


def damping_rho(n: int, level: int, cells: int, ny: int | None = None) -> torch.Tensor:
    """Sponge ramp rho in [0, 1] at the nodes of level l of a fine grid with n columns
    and ny rows (ny = n by default).

    The damping mask grows from 0 inside the domain to its full value at the
    boundary over a layer of ``cells`` fine cells (Section 2, the damped
    equation).  Reading: linear ramp r(t) = max(0, 1 - min(t, N - t)/W) in fine
    index units along each axis (N the fine node count of that axis), combined by
    max over the two axes, injected to coarse levels."""
    ny = n if ny is None else ny

    def ramp(nf):
        nl = level_size(nf, level)
        t = torch.arange(nl, dtype=F64) * (nf // nl)
        return torch.clamp(1.0 - torch.minimum(t, nf - t) / cells, min=0.0)

    return torch.maximum(ramp(ny)[:, None], ramp(n)[None, :])


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
    at the coarse unknowns; zero on the coarse ring.  Each axis halves."""
    ny, nx = r.shape
    eyi, exj = slice(2, ny, 2), slice(2, nx, 2)          # fine rows/cols 2I, 2J
    lyi, lxj = slice(1, ny - 1, 2), slice(1, nx - 1, 2)  # 2I-1, 2J-1
    hyi, hxj = slice(3, ny, 2), slice(3, nx, 2)          # 2I+1, 2J+1
    c = r[eyi, exj]
    ud = r[lyi, exj] + r[hyi, exj] + r[eyi, lxj] + r[eyi, hxj]
    dg = r[lyi, lxj] + r[lyi, hxj] + r[hyi, lxj] + r[hyi, hxj]
    out = torch.zeros((ny // 2, nx // 2), dtype=r.dtype)
    out[1:, 1:] = (4.0 * c + 2.0 * ud + dg) / 16.0
    return out


def prolong_bilinear(ec: torch.Tensor) -> torch.Tensor:
    """Bilinear interpolation, the stride-2 transposed convolution with
    (1/4)[1 2 1; 2 4 2; 1 2 1] (Section 3.3); equals 4 R^T.

    Even-even fine nodes copy the coarse value, edge midpoints average 2 coarse
    neighbours, cell centres average 4.  Coarse ring values are zero.  Each axis
    doubles."""
    ncy, ncx = ec.shape
    ep = torch.zeros((ncy + 1, ncx + 1), dtype=ec.dtype)
    ep[:ncy, :ncx] = ec
    ep[0, :] = 0.0
    ep[:, 0] = 0.0
    a = ep[:ncy, :ncx]
    b = ep[1:, :ncx]  # (I+1, J)
    c = ep[:ncy, 1:]  # (I, J+1)
    d = ep[1:, 1:]  # (I+1, J+1)
    out = torch.zeros((2 * ncy, 2 * ncx), dtype=ec.dtype)
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
