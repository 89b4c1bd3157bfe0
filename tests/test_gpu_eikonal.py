"""GPU parity of the on-device travel-time phase (Section 3.2.1, factored eikonal
equation) against the plain C oracle, through the C ABI (helm_eikonal).

The sweeps are compared bit for bit (the oracle rounds every operation of the same
steps in IEEE double precision, and the tile wavefront of the device reproduces the
order of the sequential passes), after one and two rounds and at convergence, on
grids of one tile (n = 16, 32, 64: tile side n) and of several tiles (n = 256, 512:
64 x 64 tiles, up to 8 per side).  Grid sides are powers of two, so tiles always
divide the grid.  The ADR operators built from the installed phase (product-rule
derivatives, one source) are checked against the oracle like every other operator.
"""
import numpy as np
import pytest
import torch

import helm_inputs as hi
from gpu_util import TOL, check_report, operator_report
from oracle import eikonal as E
from oracle.cycle import Problem

pytestmark = pytest.mark.gpu


def _slowness(vel):
    # the library's s = sqrt(n^2) with n^2 = 1 / c^2
    return np.sqrt(1.0 / (vel * vel))


def _medium(n, medium, seed):
    rng = np.random.default_rng(seed)
    if medium == "grf":
        return hi.grf_velocity(rng, n)
    if medium == "layered":
        return hi.layered_velocity(rng, n, smooth=0.01)
    return np.ones((n, n))


CASES = [(16, "grf", 1, (0.3125, 0.4)), (32, "grf", 2, (0.61, 0.27)), (64, "layered", 3, (0.5, 0.5)),
         (256, "grf", 4, (0.137, 0.801)), (512, "layered", 5, (0.75, 0.3))]


@pytest.mark.parametrize("n,medium,seed,src", CASES)
def test_sweeps_bit_exact(n, medium, seed, src):
    from paper_2404_02493_amd import Helmholtz

    vel = _medium(n, medium, seed)
    levels = max(3, min(5, int(np.log2(n)) - 2))
    H = Helmholtz(vel, 0.5 * n, levels=levels, damping_cells=4)
    s = _slowness(vel)
    t1 = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
    phi = torch.empty_like(t1)
    print(f"eikonal n={n} {medium} seed={seed} src={src}", flush=True)
    for rounds in (1, 2):
        r, ch = H.eikonal(src, max_rounds=rounds, tol=-1.0, tau1_out=t1)
        ref, rr, rch = E.eikonal_sweep(s, src, 1.0 / n, rounds, -1.0)
        got = t1.cpu().numpy()
        assert r == rr == rounds
        assert ch == rch, (ch, rch)
        assert np.array_equal(got, ref), f"{rounds} rounds: max diff {np.abs(got - ref).max():.3e}"
    r, ch = H.eikonal(src, max_rounds=1000, tol=1e-12, tau1_out=t1, phi_out=phi)
    ref, rr, rch = E.eikonal_sweep(s, src, 1.0 / n, 1000, 1e-12)
    assert (r, ch) == (rr, rch) and ch <= 1e-12
    assert np.array_equal(t1.cpu().numpy(), ref)
    assert np.array_equal(phi.cpu().numpy(), E.factored_phase(ref, src, 1.0 / n))
    H.close()


def test_several_sources_first_arrival():
    """Several sources: tau is the smallest travel time over the sources."""
    from paper_2404_02493_amd import Helmholtz

    n = 128
    vel = _medium(n, "grf", 7)
    srcs = [(0.2, 0.3), (0.7, 0.65), (0.45, 0.9)]
    H = Helmholtz(vel, 64.0, levels=4, damping_cells=4)
    phi = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
    H.eikonal(srcs, max_rounds=1000, tol=1e-12, phi_out=phi)
    s = _slowness(vel)
    ref = np.full((n, n), np.inf)
    for src in srcs:
        t, _, _ = E.eikonal_sweep(s, src, 1.0 / n, 1000, 1e-12)
        ref = np.minimum(ref, E.factored_phase(t, src, 1.0 / n))
    assert np.array_equal(phi.cpu().numpy(), ref)
    H.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_factored_phase_operators_match_oracle(prec):
    """Every operator of the cycle (ADR operators on each ADR level, GMRES, ADR
    V-cycle and step, wave cycles) with the phase installed by helm_eikonal: ADR
    coefficients from the product rule of Section 3.2.1 on every ADR level."""
    from paper_2404_02493_amd import Helmholtz

    case = hi.make_problem(64, 40.0, 4, seed=11, medium="grf", phase="fmm", damping_cells=8)
    src = (float(case.sources[0][0]), float(case.sources[0][1]))
    P = Problem(case.velocity, case.k, case.levels, damping_cells=case.damping_cells, phi=case.phi)
    H = Helmholtz(case.velocity, case.k, levels=case.levels, precision=prec, damping_cells=case.damping_cells)
    t1 = torch.empty((case.n, case.n), dtype=torch.float64, device="cuda:0")
    H.eikonal(src, max_rounds=1000, tol=1e-12, tau1_out=t1)
    ref, _, _ = E.eikonal_sweep(_slowness(case.velocity), src, 1.0 / case.n, 1000, 1e-12)
    assert np.array_equal(t1.cpu().numpy(), ref)
    P.set_phase_factored(ref, src)
    H.set_weights(P.weights.numpy())
    report = operator_report(case, P, H, prec, np.random.default_rng(5))
    H.close()
    check_report(report, TOL[prec])


def test_factored_phase_has_no_adjoint():
    from paper_2404_02493_amd import Helmholtz
    from paper_2404_02493_amd._abi import HelmError

    case = hi.make_problem(64, 40.0, 4, seed=11, medium="grf", phase="fmm", damping_cells=8)
    H = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c64", damping_cells=case.damping_cells)
    H.eikonal(case.sources[0], max_rounds=100, tol=1e-12)
    g = torch.as_tensor(case.g).to(torch.complex64).to("cuda:0")
    with pytest.raises(HelmError, match="HELM_ESTATE"):
        H.cycle_backward(2, g, torch.zeros_like(g), torch.zeros_like(g))
    with pytest.raises(HelmError, match="HELM_EINVAL"):
        H.eikonal((1.5, 0.5))
    H.close()
