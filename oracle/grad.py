"""Loss after K unrolled cycles and its reference gradient.

Test infrastructure only (see the package docstring).

The training loss of the paper is the squared relative residual after K cycles
from a zero iterate (Section 3.3, eq. loss).  The loss here is the unnormalised
||g - A u_K||^2 (FP64); its gradient with respect to the fine-grid phase phi and
the per-level weights w is what the hand-written adjoint must reproduce.  The
reference gradient is torch autograd through this oracle, with one checkpoint
per cycle.
"""
from __future__ import annotations

import numpy as np
import torch
from torch.utils.checkpoint import checkpoint

from .cycle import Problem, cycle
from .grid import apply_A

F64 = torch.float64


def loss_after_cycles(P: Problem, g, K: int, phi=None, w=None, u0=None, use_checkpoint: bool = False):
    """L = ||g - A u_K||^2 with u_{k+1} = C(u_k, g) and u_0 = 0 (or u0)."""
    if phi is not None:
        P.set_phase(phi)
    if w is not None:
        P.set_weights(w)
    g = torch.as_tensor(g)
    u = torch.zeros_like(g) if u0 is None else torch.as_tensor(u0)
    for _ in range(K):
        if use_checkpoint:
            u = checkpoint(lambda uu: cycle(P, g, uu), u, use_reentrant=False)
        else:
            u = cycle(P, g, u)
    r = g - apply_A(u, P.kappa_sys, P.h[1])
    return torch.sum(r.real * r.real + r.imag * r.imag), u


def grad_autograd(P: Problem, g, K: int, phi, w, use_checkpoint: bool = True):
    """(L, dL/dphi (n x n float64), dL/dw (L float64)) by autograd."""
    phi_t = torch.tensor(np.asarray(phi, dtype=np.float64), requires_grad=True)
    w_t = torch.tensor(np.asarray(w, dtype=np.float64), requires_grad=True)

    def run(phi_in, w_in):
        return loss_after_cycles(P, g, K, phi=phi_in, w=w_in, use_checkpoint=False)[0]

    if use_checkpoint:
        # rebuild the phase-dependent coefficients inside each checkpointed cycle
        g_t = torch.as_tensor(g)

        def one(uu, phi_in, w_in):
            P.set_phase(phi_in)
            P.set_weights(w_in)
            return cycle(P, g_t, uu)

        u = torch.zeros_like(g_t)
        for _ in range(K):
            u = checkpoint(one, u, phi_t, w_t, use_reentrant=False)
        r = g_t - apply_A(u, P.kappa_sys, P.h[1])
        L = torch.sum(r.real * r.real + r.imag * r.imag)
    else:
        L = run(phi_t, w_t)
    L.backward()
    return float(L.item()), phi_t.grad.detach().numpy(), w_t.grad.detach().numpy()
