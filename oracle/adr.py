"""ADR correction: phase derivatives, upwind ADR operator, GMRES(m), ADR V-cycle.

Test infrastructure only (see the package docstring).

Substituting v = a e^{i sigma k phi} into the damped Helmholtz operator gives the
advection-diffusion-reaction operator on the amplitude a (Section 3.2, eq. ADR):

    M a = -Delta a - 2 i sigma k grad(phi).grad(a) + c0 a,
    c0  = -i sigma k Delta(phi) + k^2 (|grad phi|^2 - n^2) - i sigma k^2 n^2 delta.

With sigma = -1 this is eq. ADR as printed (omega = k, tau = phi, s^2 = n^2,
gamma = k delta).  grad(phi).grad(a) is discretised with the first-order upwind
rule of eq. upwind; the phase derivatives use second-order central differences
inside and first-order one-sided differences at the open edge (Section 3.2.1).
"""
from __future__ import annotations

import torch

from .grid import _mask_ring, _shift, apply_A, cnorm, cdot, laplacian, prolong_bilinear, restrict_fw

F64 = torch.float64


def phase_derivatives(phi: torch.Tensor, h: float):
    """phi_x, phi_y and the 5-point Laplacian of phi at the unknowns of one level.

    Interior (1 <= j <= n-2): central (phi[j+1] - phi[j-1])/(2h) and
    (phi[j+1] - 2 phi[j] + phi[j-1])/h^2.  At the last unknown j = n-1 (the node
    x = 1 is not stored) the one-sided first-order forms (phi[j] - phi[j-1])/h and
    (phi[j] - 2 phi[j-1] + phi[j-2])/h^2.  Same along y (n the node count of the
    axis).  Zero on the ring."""

    def d1(p):  # derivative along the last axis
        n = p.shape[1]
        out = torch.zeros_like(p)
        out[:, 1:n - 1] = (p[:, 2:n] - p[:, 0:n - 2]) / (2.0 * h)
        out[:, n - 1] = (p[:, n - 1] - p[:, n - 2]) / h
        return out

    def d2(p):
        n = p.shape[1]
        out = torch.zeros_like(p)
        out[:, 1:n - 1] = (p[:, 2:n] - 2.0 * p[:, 1:n - 1] + p[:, 0:n - 2]) / (h * h)
        out[:, n - 1] = (p[:, n - 1] - 2.0 * p[:, n - 2] + p[:, n - 3]) / (h * h)
        return out

    px = d1(phi)
    py = d1(phi.transpose(0, 1)).transpose(0, 1)
    lap = d2(phi) + d2(phi.transpose(0, 1)).transpose(0, 1)
    return _mask_ring(px), _mask_ring(py), _mask_ring(lap)


def adr_coefficients(phi_l, n2_l, rho_l, k, strength, sigma, h, shift: float = 0.0):
    """Per-level coefficients of M: phi_x, phi_y and the reaction term c0 (eq. ADR);
    the relative shift s0 of the shifted equation enters c0 like the sponge term."""
    px, py, lap = phase_derivatives(phi_l, h)
    delta = strength * rho_l * rho_l + shift
    c0 = (-1j * sigma * k) * lap + (k * k) * (px * px + py * py - n2_l) \
        - 1j * sigma * (k * k) * n2_l * delta
    return dict(px=px, py=py, c0=_mask_ring(c0), h=h, k=k, sigma=sigma)


def upwind_grad(a: torch.Tensor, px: torch.Tensor, py: torch.Tensor, h: float) -> torch.Tensor:
    """First-order upwind approximation of grad(phi).grad(a) (eq. upwind):
    phi_x (a_j - a_{j-1})/h where phi_x > 0 and phi_x (a_{j+1} - a_j)/h where
    phi_x < 0, i.e. the 5-point stencil (1/2h)[centre 2(|phi_x|+|phi_y|),
    west -(phi_x+|phi_x|), east phi_x-|phi_x|, south -(phi_y+|phi_y|),
    north phi_y-|phi_y|] of Section 3.3 (south/north = row i-1 / i+1)."""
    ax, ay = torch.abs(px), torch.abs(py)
    w = _shift(a, 0, -1)
    e = _shift(a, 0, 1)
    s = _shift(a, -1, 0)
    nn = _shift(a, 1, 0)
    return ((2.0 * (ax + ay)) * a - (px + ax) * w + (px - ax) * e - (py + ay) * s + (py - ay) * nn) / (2.0 * h)


def apply_M(a: torch.Tensor, coef: dict) -> torch.Tensor:
    """Upwind ADR operator M a = -Delta_h a - 2 i sigma k U_h[a] + c0 a, zero on the ring."""
    h, k, sigma = coef["h"], coef["k"], coef["sigma"]
    u = upwind_grad(a, coef["px"], coef["py"], h)
    return laplacian(a, h) + _mask_ring((-2j * sigma * k) * u + coef["c0"] * a)


def gmres(op, b: torch.Tensor, x0, m: int, breakdown_tol: float = 1e-14):
    """GMRES(m) from x0 (None means 0): x = x0 + argmin over z in K_m(op, r0) of
    ||b - op(x0 + z)||_2 (used as the ADR smoother, Section 3.2.2).

    Arnoldi with modified Gram-Schmidt; stops early when h_{j+1,j} <= 1e-14 beta
    (the Krylov space is invariant); the small least-squares problem is solved by
    a library least-squares routine."""
    r0 = b if x0 is None else b - op(x0)
    beta = cnorm(r0)
    if beta.item() == 0.0:
        return torch.zeros_like(b) if x0 is None else x0
    V = [r0 / beta]
    cols = []  # Hessenberg columns, column j has j + 2 entries
    for j in range(m):
        w = op(V[j])
        col = []
        for i in range(j + 1):
            hij = cdot(V[i], w)
            col.append(hij)
            w = w - hij * V[i]
        hn = cnorm(w)
        col.append(hn.to(b.dtype))
        cols.append(col)
        if hn.item() <= breakdown_tol * beta.item():
            break
        if j + 1 < m:
            V.append(w / hn)
    mm = len(cols)
    zero = torch.zeros((), dtype=b.dtype)
    H = torch.stack([torch.stack(c + [zero] * (mm + 1 - len(c))) for c in cols], dim=1)
    rhs = torch.zeros((mm + 1, 1), dtype=b.dtype)
    rhs[0, 0] = 1.0
    y = torch.linalg.lstsq(H, rhs * beta.to(b.dtype)).solution[:, 0]
    z = torch.zeros_like(b)
    for i in range(mm):
        z = z + y[i] * V[i]
    return z if x0 is None else x0 + z


def adr_vcycle(P, level: int, b: torch.Tensor, x):
    """One V-cycle for M on ADR levels level..LA (Section 3.2.2: one V-cycle with
    GMRES(3) pre- and post-smoothing).  Reading: on the coarsest ADR level LA the
    cycle applies GMRES(gmres_coarse_m) and returns."""
    coef = P.adr[level]
    op = lambda v: apply_M(v, coef)
    if level == P.LA:
        return gmres(op, b, x, P.gmres_coarse_m)
    x = gmres(op, b, x, P.gmres_m)
    rc = restrict_fw(b - op(x))
    ec = adr_vcycle(P, level + 1, rc, None)
    x = x + prolong_bilinear(ec)
    return gmres(op, b, x, P.gmres_m)


def adr_step(P, g2: torch.Tensor, u2: torch.Tensor) -> torch.Tensor:
    """One ADR correction on level 2 (Algorithm 1, post-smoothing at level 2):
    r = g - A u, r_hat = r e^{-i sigma k phi}, a = ADR V-cycle(r_hat, 0),
    u += a e^{+i sigma k phi}  (eq. Rytov and eq. ADR)."""
    r = g2 - apply_A(u2, P.kappa[2], P.h[2])
    rhat = r * P.carrier_conj
    a = adr_vcycle(P, 2, rhat, None)
    return u2 + a * P.carrier
