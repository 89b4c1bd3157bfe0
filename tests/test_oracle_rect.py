"""Pins of the oracle on rectangular grids (n_x != n_y; the non-square domains of
Section 4.3.2).

Grid reading: n_x columns and n_y rows of stored nodes, powers of two, spacing
h = 1/max(n_x, n_y) on both axes (the longer side has unit length), each axis halved
per level.  The checks use what the mathematics fixes independently of the oracle's
code: the tensor-product sine modes of the Dirichlet Laplacian on a rectangle, a
dense operator assembled from Kronecker products, hand-computed sponge values, a
dense eigen-decomposition for the Chebyshev default, and the exact symmetry of the
whole method under transposition of the domain (swapping x and y swaps n_x and n_y,
the two phase derivatives, and the west/east with the south/north upwind roles).
"""
import math

import numpy as np
import pytest
import torch

import helm_inputs as hi
from oracle import eikonal as E
from oracle.adr import apply_M, phase_derivatives
from oracle.cycle import Problem, cycle
from oracle.grid import apply_A, cdot, damping_rho, prolong_bilinear, restrict_fw
from oracle.smooth import alpha_median_rule, lambda_gershgorin
from oracle.solve import fgmres

C128 = torch.complex128
SHAPES = [(16, 32), (32, 16), (8, 32)]  # (n_y, n_x)


def _mode(ny, nx, a, b):
    """sin(pi a x / X) sin(pi b y / Y) at the nodes, X = n_x h, Y = n_y h."""
    j, i = np.arange(nx), np.arange(ny)
    return torch.as_tensor(np.outer(np.sin(np.pi * b * i / ny), np.sin(np.pi * a * j / nx)).astype(np.complex128))


def _rand_grid(rng, ny, nx):
    v = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    v[0, :] = 0
    v[:, 0] = 0
    return torch.as_tensor(v)


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_helmholtz_symbol_on_rectangular_sine_modes(ny, nx):
    """A v = lambda v with lambda = (4/h^2)(sin^2(pi a/(2 n_x)) + sin^2(pi b/(2 n_y))) - kappa
    for the separable Dirichlet modes of the rectangle (Section 2 stencil)."""
    h = 1.0 / max(nx, ny)
    kap = 91.0 + 3.0j
    K = torch.full((ny, nx), kap, dtype=C128)
    for a, b in [(1, 1), (nx - 1, 1), (1, ny - 1), (nx // 2, ny // 2 - 1), (nx - 1, ny - 1)]:
        v = _mode(ny, nx, a, b)
        lam = 4 / h**2 * (math.sin(math.pi * a / (2 * nx)) ** 2 + math.sin(math.pi * b / (2 * ny)) ** 2) - kap
        assert torch.allclose(apply_A(v, K, h), lam * v, rtol=0, atol=1e-10 * abs(lam))


def _tridiag(m, h):
    return (2.0 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)) / (h * h)


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_operator_equals_dense_kronecker_assembly(ny, nx):
    """-Delta_h - kappa on the (n_y - 1) x (n_x - 1) unknowns equals
    kron(I_y, T_x) + kron(T_y, I_x) - diag(kappa), T the 1-D second difference."""
    rng = np.random.default_rng(3)
    h = 1.0 / max(nx, ny)
    kap = torch.as_tensor(rng.uniform(10, 300, (ny, nx)) + 1j * rng.uniform(0, 50, (ny, nx)))
    u = _rand_grid(rng, ny, nx)
    Lx, Ly = _tridiag(nx - 1, h), _tridiag(ny - 1, h)
    A = np.kron(np.eye(ny - 1), Lx) + np.kron(Ly, np.eye(nx - 1)) - np.diag(kap.numpy()[1:, 1:].ravel())
    ref = (A @ u.numpy()[1:, 1:].ravel()).reshape(ny - 1, nx - 1)
    out = apply_A(u, kap, h).numpy()
    assert np.allclose(out[1:, 1:], ref, rtol=1e-13, atol=1e-9)
    assert not out[0, :].any() and not out[:, 0].any()


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_full_weighting_symbol_and_transpose_on_rectangles(ny, nx):
    """R mode(a, b) = cos^2(pi a/(2 n_x)) cos^2(pi b/(2 n_y)) coarse mode; P = 4 R^T;
    P of a coarse delta is the bilinear hat."""
    for a, b in [(1, 1), (nx // 2 - 1, 1), (1, ny // 2 - 1), (3, 2)]:
        rc = restrict_fw(_mode(ny, nx, a, b))
        fac = math.cos(math.pi * a / (2 * nx)) ** 2 * math.cos(math.pi * b / (2 * ny)) ** 2
        assert rc.shape == (ny // 2, nx // 2)
        assert torch.allclose(rc, fac * _mode(ny // 2, nx // 2, a, b), atol=1e-13)
    rng = np.random.default_rng(5)
    x, y = _rand_grid(rng, ny, nx), _rand_grid(rng, ny // 2, nx // 2)
    lhs, rhs = cdot(restrict_fw(x), y), cdot(x, prolong_bilinear(y)) / 4
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)
    I, J = ny // 4, nx // 4 - 1
    e = torch.zeros((ny // 2, nx // 2), dtype=C128)
    e[I, J] = 1.0
    f = prolong_bilinear(e).real.numpy()
    hx = np.clip(1 - np.abs(np.arange(nx) / 2.0 - J), 0, None)
    hy = np.clip(1 - np.abs(np.arange(ny) / 2.0 - I), 0, None)
    assert np.array_equal(f, np.outer(hy, hx))


def test_sponge_ramp_values_on_a_rectangle():
    """W = 4 fine cells: rho = max over the axes of max(0, 1 - min(t, N - t)/4), N = 32
    columns and 16 rows; values computed by hand."""
    rho = damping_rho(32, 1, 4, ny=16).numpy()
    assert rho.shape == (16, 32)
    assert rho[8, 16] == 0.0           # centre
    assert rho[0, 16] == 1.0 and rho[8, 0] == 1.0
    assert rho[15, 16] == 0.75         # one row from the implicit row 16
    assert rho[8, 31] == 0.75          # one column from the implicit column 32
    assert rho[13, 16] == 0.25 and rho[12, 16] == 0.0
    assert rho[8, 28] == 0.0 and rho[8, 29] == 0.25
    assert rho[2, 30] == 0.5           # max(1 - 2/4, 1 - 2/4)
    assert rho[1, 29] == 0.75          # max(1 - 1/4, 1 - 3/4)
    assert np.array_equal(damping_rho(32, 2, 4, ny=16).numpy(), rho[::2, ::2])


def test_chebyshev_default_matches_dense_spectrum_on_a_rectangle():
    """alpha = lambda_bound / median of the eigenvalues of A^*A for constant n^2 without
    damping, here from a dense eigen-decomposition of the rectangular operator."""
    ny, nx, k = 8, 32, 40.0
    h = 1.0 / max(nx, ny)
    A = np.kron(np.eye(ny - 1), _tridiag(nx - 1, h)) + np.kron(_tridiag(ny - 1, h), np.eye(nx - 1)) \
        - k * k * np.eye((nx - 1) * (ny - 1))
    ev = np.linalg.eigvalsh(A.T @ A)
    lam = 1e9
    got = alpha_median_rule(k, 1.0, nx, lam, ny, h)
    assert got == pytest.approx(lam / np.median(ev), rel=1e-9)


def _problem(ny, nx, seed, transpose=False, **kw):
    case = hi.make_problem(nx, 0.5 * max(nx, ny), 3, seed, medium="grf", phase="fmm", damping_cells=6, ny=ny)
    vel, phi, g = case.velocity, case.phi, case.g
    if transpose:
        vel, phi, g = vel.T.copy(), phi.T.copy(), g.T.copy()
    P = Problem(vel, case.k, 3, damping_cells=6, phi=phi, **kw)
    return P, torch.as_tensor(g)


@pytest.mark.parametrize("ny,nx", [(32, 64), (64, 32)])
def test_cycle_commutes_with_transposition(ny, nx):
    """C(u, g) on the transposed domain is the transpose of C(u, g): every part of the
    cycle (sponge per axis, both transfer operators, both smoothers, the upwind ADR
    operator with phi_x and phi_y exchanged, GMRES) must treat the axes alike.  Using
    the size of one axis for the other breaks the symmetry."""
    P, g = _problem(ny, nx, 4)
    Pt, gt = _problem(ny, nx, 4, transpose=True)
    assert Pt.nx == ny and Pt.ny == nx
    assert np.allclose(P.weights.numpy(), Pt.weights.numpy(), rtol=1e-14, atol=0)
    rng = np.random.default_rng(8)
    u = _rand_grid(rng, ny, nx)
    out = cycle(P, g, u)
    out_t = cycle(Pt, gt, u.T.contiguous())
    assert torch.allclose(out_t, out.T, rtol=0, atol=1e-10 * float(out.abs().max()))
    # the upwind ADR operator alone, on level 2
    a = _rand_grid(rng, ny // 2, nx // 2)
    Ma, Mat = apply_M(a, P.adr[2]), apply_M(a.T.contiguous(), Pt.adr[2])
    assert torch.allclose(Mat, Ma.T, rtol=0, atol=1e-11 * float(Ma.abs().max()))


def test_rectangle_is_not_its_square_embedding():
    """The rectangle's cycle differs from the cycle on the square of its longer side
    with the same data in the common rows (the boundary at row n_y is real)."""
    P, g = _problem(32, 64, 4)
    rng = np.random.default_rng(2)
    u = _rand_grid(rng, 32, 64)
    out = cycle(P, g, u)
    assert out.shape == (32, 64)
    assert float(out[-1].abs().max()) > 0.0
    assert P.h[1] == 1.0 / 64 and P.rho[1].shape == (32, 64)


@pytest.mark.parametrize("ny,nx", [(64, 128), (128, 64)])
def test_solve_on_a_rectangle_converges_and_is_transposition_invariant(ny, nx):
    """FGMRES(20) with the Wave-ADR cycle reaches 1e-6 on a rectangle, and the
    transposed domain takes the same number of iterations with the transposed
    solution."""
    P, g = _problem(ny, nx, 6)
    Pt, gt = _problem(ny, nx, 6, transpose=True)
    x, it, rel, ok = fgmres(P, g, tol=1e-6, maxit=200)
    xt, itt, _, _ = fgmres(Pt, gt, tol=1e-6, maxit=200)
    assert ok and rel < 1e-6 and it < 200
    assert it == itt
    assert torch.allclose(xt, x.T, rtol=0, atol=1e-8 * float(x.abs().max()))


@pytest.mark.parametrize("ny,nx", [(16, 64), (64, 16)])
def test_phase_derivatives_per_axis(ny, nx):
    """phi = x^2 + 3 y: phi_x = 2x and Lap = 2 in the interior (central differences are
    exact on quadratics), phi_y = 3; the open edge of each axis takes its own size."""
    h = 1.0 / max(nx, ny)
    Y, X = np.meshgrid(np.arange(ny) * h, np.arange(nx) * h, indexing="ij")
    px, py, lap = phase_derivatives(torch.as_tensor(X * X + 3 * Y), h)
    assert np.allclose(px.numpy()[1:, 1:nx - 1], 2 * X[1:, 1:nx - 1], atol=1e-12)
    assert np.allclose(px.numpy()[1:, nx - 1], 2 * X[1:, nx - 1] - h, atol=1e-12)  # (x^2 - (x-h)^2)/h
    assert np.allclose(py.numpy()[1:, 1:], 3.0, atol=1e-10)
    assert np.allclose(lap.numpy()[1:, 1:nx - 1], 2.0, atol=1e-7)


@pytest.mark.parametrize("ny,nx", [(32, 128), (128, 32)])
def test_eikonal_constant_medium_exact_on_rectangles(ny, nx):
    """Constant slowness s: tau1 = s at every node (tau0 is exact), on both orientations."""
    h = 1.0 / max(nx, ny)
    src = (0.3 * nx * h, 0.6 * ny * h)
    t1, rounds, ch = E.eikonal_sweep(np.full((ny, nx), 0.5), src, h, 100, 0.0)
    assert t1.shape == (ny, nx) and ch == 0.0 and rounds < 100
    assert np.abs(t1 - 0.5).max() <= 1e-12 * 0.5


def test_eikonal_transposition():
    """Sweeping the transposed slowness from the mirrored source gives the transposed
    tau1 (the converged discrete solution does not depend on the sweep order)."""
    ny, nx = 32, 64
    h = 1.0 / 64
    s = 1.0 / hi.grf_velocity(np.random.default_rng(1), nx, ny=ny)
    src = (0.41, 0.2)
    t1, _, _ = E.eikonal_sweep(s, src, h, 1000, 1e-14)
    t1t, _, _ = E.eikonal_sweep(s.T.copy(), (src[1], src[0]), h, 1000, 1e-14)
    assert np.allclose(t1t, t1.T, rtol=1e-12, atol=0)
