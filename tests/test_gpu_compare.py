"""GPU parity of the comparison preconditioners built on the same kernels
(Section 4.3.1): the CSL V-cycle (a cycle for the complex-shifted operator, shift 0.5,
no ADR correction) and Wave-Ray (eight plane-wave ray corrections instead of the
phase of the eikonal), against the FP64 oracle operator by operator, cycle by cycle and
solve by solve."""
import numpy as np
import pytest
import torch

import helm_inputs as hi
from gpu_util import TOL, assert_close, check_report, make_pair, operator_report, rand_grid, rounded, to_dev
from oracle.cycle import cycle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_case():
    return hi.make_problem(64, 40.0, 4, seed=11, medium="grf", phase="fmm", damping_cells=8)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_csl_operator_parity(small_case, prec):
    P, H = make_pair(small_case, prec, cycle_shift=0.5, adr_steps=0)
    report = operator_report(small_case, P, H, prec, np.random.default_rng(2))
    H.close()
    check_report(report, TOL[prec])


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_wave_ray_cycle_parity(small_case, prec):
    """Cycles with eight ray corrections (one per ray) from a random iterate and from
    zero, on level 1 and from level 2."""
    P, H = make_pair(small_case, prec)
    P.set_rays(8)
    H.set_rays(8)
    rng = np.random.default_rng(4)
    cd = H.cdtype
    u, g = rounded(rand_grid(rng, 64), cd), rounded(rand_grid(rng, 64), cd)
    out = H.debug_op(10, 1, to_dev(u, cd), to_dev(g, cd))
    r1 = assert_close(out, cycle(P, g, u), TOL[prec], "W1")
    out = H.debug_op(10, 1, None, to_dev(g, cd))
    r0 = assert_close(out, cycle(P, g, torch.zeros_like(g)), TOL[prec], "W1z")
    # the graph-replayed cycle (helm_cycle) agrees too
    ud = to_dev(u, cd)
    H.cycle(to_dev(g, cd), ud)
    rc = assert_close(ud, cycle(P, g, u), TOL[prec], "cycle")
    H.close()
    print(prec, r1, r0, rc, flush=True)


@pytest.mark.parametrize("name,kw,rays", [("csl", dict(cycle_shift=0.5, adr_steps=0), 0), ("wave_ray", {}, 8)])
def test_comparison_solve_matches_oracle(name, kw, rays):
    """FGMRES(20) to 1e-6 on the 128^2 constant medium: the oracle's iteration count
    (+-1) and solution."""
    from oracle.solve import fgmres

    c = hi.make_case("const128")
    P, H = make_pair(c, "c128", **kw)
    if rays:
        P.set_rays(rays)
        H.set_rays(rays)
    g = torch.as_tensor(c.g)
    x_or, its_or, rr_or, ok = fgmres(P, g, tol=1e-6, maxit=400)
    assert ok
    u, its, rr, _ = H.solve(g.to("cuda:0"), tol=1e-6, maxit=400, mode=0)
    H.close()
    print(name, "iterations gpu", its, "oracle", its_or, "relres", rr, rr_or, flush=True)
    assert rr < 1e-6 and abs(its - its_or) <= 1
    assert_close(u, x_or, 1e-6, "solution")


def test_rays_then_phase_again(small_case):
    """helm_set_phase after helm_set_rays returns to the single phase (and its fused
    ADR steps): the cycle equals that of a context that never had rays."""
    P, H = make_pair(small_case, "c128")
    H.set_rays(8)
    H.set_phase(small_case.phi)
    rng = np.random.default_rng(8)
    u, g = rand_grid(rng, 64), rand_grid(rng, 64)
    ud = to_dev(u, torch.complex128)
    H.cycle(to_dev(g, torch.complex128), ud)
    H.close()
    assert_close(ud, cycle(P, g, u), TOL["c128"], "cycle")
