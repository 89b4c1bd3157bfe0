"""Outer solver: FGMRES(restart) right-preconditioned by one Wave-ADR cycle.

Test infrastructure only (see the package docstring).

The paper uses every preconditioner inside FGMRES with restart 20, a zero
initial guess and the stopping test ||r_k|| / ||g|| < 1e-6 (Section 4.3.1).
The preconditioner is z = C(0, v), one cycle from a zero iterate; since the
cycle is nonlinear in v (GMRES inside), the flexible variant is required.
Reading: the Givens estimate of the residual ends an inner cycle; the true
residual is then checked and the method restarts if it is not yet below tol.
"""
from __future__ import annotations

import math

import torch

from .cycle import Problem, cycle
from .grid import apply_A, cdot, cnorm


def _givens(a: complex, b: complex):
    """c (real), s with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    rho = math.hypot(abs(a), abs(b))
    c = abs(a) / rho
    s = (a / abs(a)) * b.conjugate() / rho
    return c, s


def fgmres(P: Problem, g: torch.Tensor, x0=None, tol: float = 1e-6, restart: int = 20,
           maxit: int = 500, precond=None, history=None):
    """Returns (x, iterations, true relative residual, converged)."""
    prec = precond if precond is not None else (lambda v: cycle(P, v, torch.zeros_like(v)))
    x = torch.zeros_like(g) if x0 is None else x0.clone()
    gnorm = cnorm(g).item()
    if gnorm == 0.0:
        return torch.zeros_like(g), 0, 0.0, True
    its = 0
    while True:
        r = g - apply_A(x, P.kappa_sys, P.h[1])
        beta = cnorm(r).item()
        if beta / gnorm < tol:
            return x, its, beta / gnorm, True
        if its >= maxit:
            return x, its, beta / gnorm, False
        V = [r / beta]
        Z = []
        H = [[0j] * restart for _ in range(restart + 1)]
        cs, sn = [], []
        e = [0j] * (restart + 1)
        e[0] = complex(beta)
        j_used = 0
        for j in range(restart):
            z = prec(V[j])
            Z.append(z)
            w = apply_A(z, P.kappa_sys, P.h[1])
            for i in range(j + 1):
                hij = cdot(V[i], w)
                H[i][j] = complex(hij.item())
                w = w - hij * V[i]
            hn = cnorm(w).item()
            H[j + 1][j] = complex(hn)
            for i in range(j):
                t1 = cs[i] * H[i][j] + sn[i] * H[i + 1][j]
                t2 = -sn[i].conjugate() * H[i][j] + cs[i] * H[i + 1][j]
                H[i][j], H[i + 1][j] = t1, t2
            c, s = _givens(H[j][j], H[j + 1][j])
            cs.append(c)
            sn.append(s)
            H[j][j] = c * H[j][j] + s * H[j + 1][j]
            H[j + 1][j] = 0j
            e[j + 1] = -s.conjugate() * e[j]
            e[j] = c * e[j]
            its += 1
            j_used = j + 1
            est = abs(e[j + 1]) / gnorm
            if history is not None:
                history.append(est)
            if est < tol or hn == 0.0 or its >= maxit:
                break
            V.append(w / hn)
        y = [0j] * j_used
        for i in range(j_used - 1, -1, -1):
            acc = e[i]
            for q in range(i + 1, j_used):
                acc -= H[i][q] * y[q]
            y[i] = acc / H[i][i]
        for i in range(j_used):
            x = x + y[i] * Z[i]
