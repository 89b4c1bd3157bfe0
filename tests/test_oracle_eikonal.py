"""Pins of the factored eikonal oracle (Section 3.2.1, eq. eikeq and eq. eikonal_cons).

CPU only.  The discrete scheme is the oracle's reading (first-order Godunov upwind
form of the factored equation, solved by fast sweeping); these tests fix it to
what the mathematics fixes: the exact solution for a constant medium, first-order
convergence to the closed-form travel time of a linear velocity gradient, mirror
symmetry, a true fixed point at convergence, and the product rule of the phase
derivatives against automatic differentiation.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

from oracle import eikonal as E
from oracle.adr import phase_derivatives


def _grid(n):
    x = np.arange(n) / n
    return np.meshgrid(x, x)  # X (varies along j), Y (varies along i)


@pytest.mark.parametrize("src", [(0.5, 0.5), (0.31, 0.47), (0.0, 0.0), (0.984375, 0.125)])
@pytest.mark.parametrize("s0", [0.5, 1.3])
def test_constant_medium_is_exact(src, s0):
    """s constant: tau = s |x - x0| solves eq. eikeq, so tau1 = s at every node."""
    n = 64
    t1, rounds, change = E.eikonal_sweep(np.full((n, n), s0), src, 1.0 / n, 60, 0.0)
    assert change == 0.0 and rounds < 60
    assert np.abs(t1 - s0).max() <= 1e-12 * s0


@pytest.mark.parametrize("src", [(0.5, 0.5), (0.0, 0.0), (0.984375, 0.125)])
def test_four_sweep_orders_reach_every_quadrant_in_one_round(src):
    """Straight rays from the source: each of the four sweep orders covers one
    quadrant, so one round reaches the solution and the second one only confirms it."""
    n = 64
    t1, rounds, change = E.eikonal_sweep(np.full((n, n), 0.5), src, 1.0 / n, 60, 1e-12)
    assert rounds == 2 and change <= 1e-12


def _linear_exact(n, src, c0, g):
    # c = c0 + g y: tau = arccosh(1 + g^2 |x - x0|^2 / (2 c(x0) c(x))) / g
    X, Y = _grid(n)
    cs, c = c0 + g * src[1], c0 + g * Y
    return np.arccosh(1.0 + g * g * ((X - src[0]) ** 2 + (Y - src[1]) ** 2) / (2.0 * cs * c)) / g


def test_linear_gradient_converges_first_order():
    """Velocity linear in depth has a closed-form travel time; the first-order scheme
    must approach it at rate h (errors halve as n doubles)."""
    c0, g, src = 1.0, 1.5, (0.4, 0.3)
    errs = []
    for n in (64, 128, 256):
        X, Y = _grid(n)
        t1, rounds, change = E.eikonal_sweep(1.0 / (c0 + g * Y), src, 1.0 / n, 200, 1e-13)
        assert change <= 1e-13
        tau = E.factored_phase(t1, src, 1.0 / n)
        err = np.abs(tau - _linear_exact(n, src, c0, g))
        errs.append(err.max())
        if n == 64:
            # the fixed nodes around the source take the straight-ray mean slowness,
            # second-order accurate there
            near = np.hypot(X - src[0], Y - src[1]) <= np.sqrt(2.0) / n
            assert near.sum() >= 4 and err[near].max() < 4e-5
    assert errs[-1] < 2.5e-4
    assert errs[0] / errs[1] > 1.7 and errs[1] / errs[2] > 1.7, errs


def test_mirror_symmetry():
    """A medium symmetric about x = 1/2 with the source on that line gives a travel
    time symmetric about it (node j <-> n - j)."""
    n = 64
    X, Y = _grid(n)
    c = 1.0 + 0.6 * np.exp(-((np.abs(X - 0.5) - 0.2) ** 2 + (Y - 0.6) ** 2) / 0.01) + 0.4 * Y
    t1, _, _ = E.eikonal_sweep(1.0 / c, (0.5, 0.25), 1.0 / n, 200, 0.0)
    assert np.abs(t1[:, 1:] - t1[:, :0:-1]).max() <= 1e-12


def test_converged_sweeps_are_a_fixed_point():
    """At convergence (tol 0) another round changes nothing, and the iterate after
    r + 1 forced rounds equals the converged one."""
    n = 48
    X, Y = _grid(n)
    c = 1.0 + 0.5 * np.sin(3 * X) * np.cos(2 * Y) + Y
    src = (0.3, 0.6)
    t1, rounds, change = E.eikonal_sweep(1.0 / c, src, 1.0 / n, 300, 0.0)
    assert change == 0.0
    t2, r2, ch2 = E.eikonal_sweep(1.0 / c, src, 1.0 / n, rounds + 1, -1.0)
    assert r2 == rounds + 1 and ch2 == 0.0
    assert np.array_equal(t1, t2)


def test_product_rule_matches_autograd_for_quadratic_tau1():
    """For a quadratic tau1 the finite differences of the rule are exact inside, so the
    product-rule derivatives equal the derivatives of tau0 tau1 taken by automatic
    differentiation; next to the source the rule falls back to the differences of
    tau0 tau1 itself."""
    n, h, src = 32, 1.0 / 32, (0.37, 0.40625)

    def tau1f(x, y):
        return 0.7 + 0.3 * x - 0.2 * y + 0.1 * x * y + 0.05 * y * y

    x = torch.arange(n, dtype=torch.float64) * h
    Y, X = torch.meshgrid(x, x, indexing="ij")
    t1 = tau1f(X, Y)
    px, py, lap = E.factored_derivatives(t1, src, h)
    Xa, Ya = X.clone().requires_grad_(True), Y.clone().requires_grad_(True)
    phi = torch.sqrt((Xa - src[0]) ** 2 + (Ya - src[1]) ** 2) * tau1f(Xa, Ya)
    gx, gy = torch.autograd.grad(phi.sum(), (Xa, Ya), create_graph=True)
    gxx = torch.autograd.grad(gx.sum(), Xa, retain_graph=True)[0]
    gyy = torch.autograd.grad(gy.sum(), Ya)[0]
    r = torch.sqrt((X - src[0]) ** 2 + (Y - src[1]) ** 2)
    inner = torch.zeros_like(r, dtype=torch.bool)
    inner[1:n - 1, 1:n - 1] = True
    far = inner & (r >= h)
    near = (r < h)
    assert far.sum() > 500 and near.sum() >= 1
    for a, b in ((px, gx), (py, gy), (lap, gxx + gyy)):
        assert torch.allclose(a[far], b.detach()[far], rtol=1e-9, atol=1e-9)
    fx, fy, fl = phase_derivatives(r * t1, h)
    for a, b in ((px, fx), (py, fy), (lap, fl)):
        assert torch.equal(a[near], b[near])
    # the open edge (j = n - 1) uses the one-sided rule on tau1, so it is first order only
    assert px[5, n - 1] != 0.0


def test_sources_outside_the_grid_are_rejected():
    with pytest.raises(ValueError):
        E.eikonal_sweep(np.ones((16, 16)), (1.2, 0.5), 1.0 / 16)
