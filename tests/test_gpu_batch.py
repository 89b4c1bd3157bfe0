"""GPU: batched solves of independent problems of mixed sizes (helm_batch_*).

Each problem of a batch runs exactly the single-problem solve on its own context,
so the batch results must equal single solves bit for bit, whatever the lane
interleaving.  Inputs: the mixed-size batch generator (grid sizes drawn from
{256, 512, 1024}, k = 0.625 n, one to four sources, multi-source phase), here a
small sample of it plus smaller sizes for speed.
"""
import numpy as np
import pytest
import torch

import helm_inputs as hi

pytestmark = pytest.mark.gpu


def _problems(cases):
    return [dict(velocity=c.velocity, k=c.k, levels=c.levels, damping_cells=c.damping_cells, phi=c.phi)
            for c in cases]


@pytest.fixture(scope="module")
def small_batch():
    rng = np.random.default_rng(5)
    cases = []
    for p in range(6):
        n = int(rng.choice([128, 256]))
        cases.append(hi.make_problem(n, 0.625 * n, hi.default_levels(n), seed=500 + p, medium="grf", nsrc=(1, 4),
                                     phase="fmm", name=f"b{p}"))
    return cases


@pytest.mark.parametrize("prec,mode", [("c64", 1), ("c128", 0)])
def test_batch_equals_single_solves(small_batch, prec, mode):
    from paper_2404_02493_amd import Helmholtz, HelmholtzBatch

    B = HelmholtzBatch(_problems(small_batch), precision=prec, lanes=3)
    gs = [torch.as_tensor(c.g).to("cuda:0") for c in small_batch]
    us, its, rr, st = B.solve(gs, tol=1e-6, maxit=400, mode=mode)
    torch.cuda.synchronize()
    cls = B.classes()
    print("iters", its.tolist(), "relres", rr.tolist(), "classes", cls.tolist(), flush=True)
    # FP32 refinement: the problems of each size share a lockstep class; FP64 runs alone
    assert np.all(cls >= 0) if mode == 1 else np.all(cls == -1)
    assert np.all(st == 0) and np.all(rr < 1e-6)
    for p, c in enumerate(small_batch):
        H = Helmholtz(c.velocity, c.k, levels=c.levels, precision=prec, damping_cells=c.damping_cells)
        H.set_phase(c.phi)
        u, it, r, _ = H.solve(gs[p], tol=1e-6, maxit=400, mode=mode)
        assert it == its[p] and r == rr[p]
        assert torch.equal(u, us[p]), p
        H.close()
    if prec == "c128":
        # one problem of the batch against the FP64 oracle's FGMRES(20)
        from oracle.cycle import Problem
        from oracle.solve import fgmres

        p = min(range(len(small_batch)), key=lambda q: small_batch[q].n)
        c = small_batch[p]
        P = Problem(c.velocity, c.k, c.levels, damping_cells=c.damping_cells, phi=c.phi)
        x_or, its_or, rr_or, ok = fgmres(P, torch.as_tensor(c.g), tol=1e-6, maxit=400)
        err = (torch.linalg.norm(us[p].cpu() - x_or) / torch.linalg.norm(x_or)).item()
        print("batch problem", p, "n", c.n, "iterations", its[p], "oracle", its_or, "error", err, flush=True)
        assert ok and abs(int(its[p]) - its_or) <= 1 and err < 1e-6
    B.close()


def test_batch_statuses_and_problem_view(small_batch):
    from paper_2404_02493_amd import HelmholtzBatch

    B = HelmholtzBatch(_problems(small_batch), precision="c64", lanes=4)
    gs = [torch.as_tensor(c.g).to("cuda:0") for c in small_batch]
    us, its, rr, st = B.solve(gs, tol=1e-6, maxit=2, mode=1)
    assert np.all(st == 4) and np.all(its <= 2) and np.all(rr > 1e-6)  # HELM_ENOCONV per problem
    # a problem's own context: one cycle through the batch-owned context
    P0 = B.problem(0)
    g = gs[0].to(torch.complex64)
    u = torch.zeros_like(g)
    P0.cycle(g, u)
    assert torch.isfinite(torch.view_as_real(u)).all() and torch.linalg.norm(u) > 0
    B.close()


def test_batch_sample_of_the_mixed_size_batch():
    """Eight problems of the 64-problem mixed batch (sizes 256..1024), FP32 cycles with
    FP64 refinement, four lanes: every problem converges to 1e-6, and two of them
    match their single solves bit for bit."""
    from paper_2404_02493_amd import Helmholtz, HelmholtzBatch

    rng = np.random.default_rng(0)
    sizes = [256, 512, 1024, 256, 512, 256, 1024, 512]
    cases = [hi.make_problem(n, 0.625 * n, hi.default_levels(n), seed=9000 + p, medium="grf", nsrc=(1, 4),
                             phase="fmm", name=f"s{p}") for p, n in enumerate(sizes)]
    B = HelmholtzBatch(_problems(cases), precision="c64", lanes=4)
    gs = [torch.as_tensor(c.g).to("cuda:0") for c in cases]
    us, its, rr, st = B.solve(gs, tol=1e-6, maxit=2000, mode=1)
    torch.cuda.synchronize()
    print("iters", its.tolist(), flush=True)
    assert np.all(st == 0) and np.all(rr < 1e-6)
    for p in (2, 5):
        c = cases[p]
        H = Helmholtz(c.velocity, c.k, levels=c.levels, precision="c64", damping_cells=c.damping_cells)
        H.set_phase(c.phi)
        u, it, r, _ = H.solve(gs[p], tol=1e-6, maxit=2000, mode=1)
        assert it == its[p] and torch.equal(u, us[p])
        H.close()
    B.close()
    del rng


def test_lockstep_class_matches_single_solves_and_oracle():
    """Four problems of one size form a lockstep class (one launch per kernel for all of
    them): each result equals its single solve bit for bit, also with one lane, and one
    of them is checked against the FP64 oracle's solution."""
    from oracle.cycle import Problem
    from oracle.solve import fgmres
    from paper_2404_02493_amd import Helmholtz, HelmholtzBatch

    cases = [hi.make_problem(128, 80.0, 4, seed=700 + p, medium="grf", nsrc=(1, 3), phase="fmm", name=f"l{p}")
             for p in range(4)]
    assert len({c.damping_cells for c in cases}) == 1
    gs = [torch.as_tensor(c.g).to("cuda:0") for c in cases]
    results = []
    for lanes in (2, 1):
        B = HelmholtzBatch(_problems(cases), precision="c64", lanes=lanes)
        us, its, rr, st = B.solve(gs, tol=1e-6, maxit=600, mode=1)
        torch.cuda.synchronize()
        assert np.all(st == 0) and np.all(rr < 1e-6), (st, rr)
        cls = B.classes()
        assert np.all(cls == cls[0]) and cls[0] >= 0, cls  # one lockstep class
        results.append((us, its, rr))
        B.close()
    us, its, rr = results[0]
    print("lockstep iterations", its.tolist(), flush=True)
    assert np.array_equal(its, results[1][1])
    for p, c in enumerate(cases):
        assert torch.equal(us[p], results[1][0][p])
        H = Helmholtz(c.velocity, c.k, levels=c.levels, precision="c64", damping_cells=c.damping_cells)
        H.set_phase(c.phi)
        u, it, r, _ = H.solve(gs[p], tol=1e-6, maxit=600, mode=1)
        H.close()
        assert it == its[p] and r == rr[p], (p, it, its[p], r, rr[p])
        assert torch.equal(u, us[p]), p
    c = cases[1]
    P = Problem(c.velocity, c.k, c.levels, damping_cells=c.damping_cells, phi=c.phi)
    x_or, _, _, ok = fgmres(P, torch.as_tensor(c.g), tol=1e-9, maxit=400)
    err = (torch.linalg.norm(us[1].cpu() - x_or) / torch.linalg.norm(x_or)).item()
    print("lockstep problem 1 error against the oracle", err, flush=True)
    assert ok and err < 1e-4
