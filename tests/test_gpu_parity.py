"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Inputs come from helm_inputs (seeded); weights are the oracle's defaults, passed
to the library.  Tolerances: relative 1e-12 for FP64 cycles, 1e-5 for FP32
cycles, on one operator or one cycle from an identical input, both as a relative
2-norm and element by element (max |gpu - ref| <= 10 tol max |ref|).
"""
import numpy as np
import pytest
import torch

import helm_inputs as hi
from gpu_util import (TOL, assert_close, check_report, make_pair, measure, operator_report, rand_grid, rounded,
                      to_dev, within)
from oracle.adr import adr_step, adr_vcycle, apply_M, gmres
from oracle.cycle import Problem, cycle, wave_adr_cycle
from oracle.grid import apply_A, prolong_bilinear, restrict_fw
from oracle.smooth import chebyshev, jacobi

pytestmark = pytest.mark.gpu

_rand = rand_grid
rel = lambda a, b: measure(a, b)[0]


@pytest.fixture(scope="module")
def small_case():
    return hi.make_problem(64, 40.0, 4, seed=11, medium="grf", phase="fmm", damping_cells=8)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_default_weights_match_oracle(small_case, prec):
    from paper_2404_02493_amd import Helmholtz

    c = small_case
    P = Problem(c.velocity, c.k, c.levels, damping_cells=c.damping_cells)
    H = Helmholtz(c.velocity, c.k, levels=c.levels, precision=prec, damping_cells=c.damping_cells)
    assert np.allclose(H.weights, P.weights.numpy(), rtol=1e-12)
    assert np.allclose(H.lambdas, [P.lam[l] for l in range(1, c.levels + 1)], rtol=1e-13)
    H.close()


MARCH = {"sstep_rows": {"2": 48, "3": 24, "4": 24}}


@pytest.mark.parametrize("form", ["sstep", "arnoldi", "tail"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_operator_parity(small_case, prec, form):
    """Every internal operator on identical inputs, for each form of the ADR
    smoother: s-step GMRES on separate kernels ("sstep"), Arnoldi GMRES on
    separate kernels ("arnoldi"), and the default: s-step GMRES with the coarsest
    ADR level's GMRES in one workgroup ("tail")."""
    arnoldi, tail_n = {"sstep": (0, 0), "arnoldi": (1, 0), "tail": (0, 64)}[form]
    P, H = make_pair(small_case, prec, gmres_arnoldi=arnoldi, tail_n=tail_n)
    report = operator_report(small_case, P, H, prec, np.random.default_rng(0))
    H.close()
    check_report(report, TOL[prec])


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_operator_parity_shifted(small_case, prec):
    """Every operator of the shifted equation (Section 4.3.2, relative shift 0.01 in
    kappa and in the ADR reaction term)."""
    P, H = make_pair(small_case, prec, shift=0.01)
    report = operator_report(small_case, P, H, prec, np.random.default_rng(1))
    H.close()
    check_report(report, TOL[prec])


def test_shifted_solve_matches_oracle():
    """FGMRES(20) on the shifted equation to the paper's tolerance 1e-7 (Table
    tab:shift protocol) on the 128^2 constant medium: the oracle's iteration count
    (+-1) and solution."""
    from oracle.solve import fgmres

    c = hi.make_case("const128")
    P, H = make_pair(c, "c128", shift=0.01)
    g = torch.as_tensor(c.g)
    x_or, its_or, rr_or, ok = fgmres(P, g, tol=1e-7, maxit=300)
    assert ok
    u, its, rr, _ = H.solve(g.to("cuda:0"), tol=1e-7, maxit=300, mode=0)
    H.close()
    print("shifted const128 iterations gpu", its, "oracle", its_or, "relres", rr, rr_or, flush=True)
    assert rr < 1e-7 and abs(its - its_or) <= 1
    assert_close(u, x_or, 1e-6, "solution")


@pytest.mark.parametrize("n", [256, 512])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_operator_parity_marching(n, prec):
    """The same operators with the s-step GMRES passes forced to the marching form on
    every ADR level (segments of 48 steps on level 2 as in the tuned 4096^2 solve, 24
    below), the coarsest ADR level included: the Gram pass, the pre-smoother pass that
    restricts the residual, the plain combine pass and the fused level-2 passes that
    re-modulate and demodulate (the cycles W2, W1 and W1z run all eight ADR steps)."""
    c = hi.make_problem(n, 0.625 * n, hi.default_levels(n), seed=40 + n, medium="grf", phase="fmm")
    P, H = make_pair(c, prec, tail_n=0, tuning=MARCH)
    assert H.get_tuning()["sstep_rows"] == {"2": 48, "3": 24, "4": 24}
    report = operator_report(c, P, H, prec, np.random.default_rng(n))
    H.close()
    check_report(report, TOL[prec])


@pytest.mark.parametrize("name", ["const128", "grf512"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_cycle_parity_along_oracle_iterates(name, prec):
    """One cycle from identical iterates u_k of the oracle's stationary iteration."""
    c = hi.make_case(name)
    P, H = make_pair(c, prec)
    g = rounded(torch.as_tensor(c.g), H.cdtype)
    u = torch.zeros_like(g)
    errs = []
    for k in range(3):
        ref = cycle(P, g, u)
        ud = to_dev(u, H.cdtype)
        H.cycle(to_dev(g, H.cdtype), ud)
        errs.append(measure(ud, ref))
        u = rounded(ref, H.cdtype)
    H.close()
    print(name, prec, [f"{e[0]:.2e}/{e[1]:.2e}" for e in errs])
    assert all(within(e, TOL[prec]) for e in errs), errs


# untuned default (tiles below 2048^2), marching with short segments, 32 x 32 tiles
FORMS = {"default": None, "march": {"sstep_rows": {"2": 24, "3": 16, "4": 16}},
         "tile32": {"sstep_rows": {"2": 2, "3": 2, "4": 2}}}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("m,mc", [(1, 1), (2, 4), (4, 2)])
def test_cycle_parity_gmres_depths(m, mc, form):
    """One FP64 cycle with other GMRES depths on the ADR levels (smoother m, coarsest
    mc), every ADR level in the untuned default form (overlapped 16 x 16 tiles on these
    small levels), forced to the marching form, or forced to 32 x 32 tiles, and the
    coarsest ADR level in the s-step form: covers the fused residual restriction and
    prolongation passes for every depth."""
    c = hi.make_problem(128, 80.0, 5, seed=21, medium="grf", phase="fmm", damping_cells=16)
    P, H = make_pair(c, "c128", tail_n=0, gmres_m=m, gmres_coarse_m=mc, tuning=FORMS[form])
    rng = np.random.default_rng(5)
    g = torch.as_tensor(c.g).to(torch.complex128)
    u = _rand(rng, c.n)
    ref = cycle(P, g, u)
    ud = to_dev(u, H.cdtype)
    H.cycle(to_dev(g, H.cdtype), ud)
    H.close()
    r, e = assert_close(ud, ref, TOL["c128"], f"m={m} mc={mc} {form}")
    print(m, mc, form, f"{r:.2e}/{e:.2e}")


@pytest.mark.parametrize("n,levels,tail_n", [(16, 3, 0), (32, 4, 0), (32, 4, 64), (64, 5, 0)])
def test_cycle_parity_tiny_grids(n, levels, tail_n):
    """One FP64 cycle on tiny grids, where the ADR levels are a few nodes per side and
    their s-step passes run in the default tile form (tail_n = 0) or the coarsest in one
    workgroup."""
    c = hi.make_problem(n, 0.6 * n, levels, seed=31, medium="grf", phase="fmm", damping_cells=4)
    P, H = make_pair(c, "c128", tail_n=tail_n)
    rng = np.random.default_rng(9)
    g = torch.as_tensor(c.g).to(torch.complex128)
    u = _rand(rng, c.n)
    ref = cycle(P, g, u)
    ud = to_dev(u, H.cdtype)
    H.cycle(to_dev(g, H.cdtype), ud)
    H.close()
    r, e = assert_close(ud, ref, TOL["c128"], f"n={n}")
    print(n, levels, tail_n, f"{r:.2e}/{e:.2e}")


def test_solve_fp64_matches_oracle():
    from oracle.solve import fgmres

    c = hi.make_case("const128")
    P, H = make_pair(c, "c128")
    g = torch.as_tensor(c.g)
    x_or, its_or, rr_or, ok = fgmres(P, g, tol=1e-6, maxit=300)
    assert ok
    u, its, rr, hist = H.solve(g.to("cuda:0"), tol=1e-6, maxit=300, mode=0)
    H.close()
    print("iterations gpu", its, "oracle", its_or, "relres", rr, rr_or)
    assert rr < 1e-6
    assert abs(its - its_or) <= 1
    assert rel(u, x_or) < 1e-6


@pytest.mark.parametrize("mode", [0, 1])
def test_solve_fp32_cycles(mode):
    """FP32 cycles inside FP64 FGMRES (mode 0) or FP64 iterative refinement (mode 1):
    the true FP64 residual reaches 1e-6; the error against the FP64 oracle solution
    is reported and bounded."""
    from oracle.solve import fgmres

    c = hi.make_case("const128")
    P, H = make_pair(c, "c64")
    g = torch.as_tensor(c.g)
    x_or, its_or, rr_or, ok = fgmres(P, g, tol=1e-8, maxit=400)
    u, its, rr, hist = H.solve(g.to("cuda:0"), tol=1e-6, maxit=400, mode=mode)
    H.close()
    err = rel(u, x_or)
    print("mode", mode, "iterations", its, "relres", rr, "error vs oracle", err)
    assert rr < 1e-6
    assert err < 1e-4


def test_cycle_before_phase_is_state_error():
    from paper_2404_02493_amd import Helmholtz, HelmError

    c = hi.make_problem(32, 10.0, 3, seed=1, damping_cells=4)
    H = Helmholtz(c.velocity, c.k, levels=3, damping_cells=4)
    g = torch.as_tensor(c.g).to("cuda:0")
    u = torch.zeros_like(g)
    with pytest.raises(HelmError) as e:
        H.cycle(g, u)
    assert e.value.status == 6
    H.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_graph_replays_match_eager(small_case, prec):
    """Cycles replayed from a captured HIP graph equal eager launches bit for bit,
    over several replays with eager work and synchronisations in between."""
    c = small_case
    P, Hg = make_pair(c, prec)
    _, He = make_pair(c, prec, use_graphs=0) if False else (None, None)
    from paper_2404_02493_amd import Helmholtz

    He = Helmholtz(c.velocity, c.k, levels=c.levels, precision=prec, damping_cells=c.damping_cells, use_graphs=0)
    He.set_phase(c.phi)
    He.set_weights(P.weights.numpy())
    rng = np.random.default_rng(7)
    g = to_dev(_rand(rng, c.n), Hg.cdtype)
    ug = torch.zeros_like(g)
    ue = torch.zeros_like(g)
    for rep in range(4):
        Hg.cycle(g, ug)
        He.cycle(g, ue)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), rep
        # eager work on the graph context between replays
        x = to_dev(_rand(rng, c.n), Hg.cdtype)
        Hg.debug_op(1, 1, x)
        _ = (x * 2).sum().item()
        torch.cuda.synchronize()
    Hg.close()
    He.close()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-13), ("c64", 1e-5)])
@pytest.mark.parametrize("literal", [0, 1])
def test_wave_tail_matches_per_level_kernels(prec, tol, literal):
    """The one-workgroup kernel for the small wave levels gives the cycle of the
    per-level kernels (wave_tail_n = 0), including the literal level-3 smoother,
    to the per-cycle tolerance of the precision (FP32: 1e-5 relative)."""
    from paper_2404_02493_amd import Helmholtz

    c = hi.make_problem(256, 160.0, 5, seed=8, medium="grf", phase="fmm", damping_cells=16)
    rng = np.random.default_rng(3)
    u0 = _rand(rng, 256)
    outs = []
    for wt in (0, 128):
        H = Helmholtz(c.velocity, c.k, levels=c.levels, precision=prec, damping_cells=16, wave_tail_n=wt,
                      level3_literal=literal)
        H.set_phase(c.phi)
        g = to_dev(torch.as_tensor(c.g), H.cdtype)
        u = to_dev(u0, H.cdtype)
        H.cycle(g, u)
        outs.append(u.cpu())
        H.close()
    assert rel(outs[1], outs[0]) < tol
