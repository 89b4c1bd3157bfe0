"""GPU: the launch-shape autotuner (helm_tune / helm_set_tuning).

The tuner only changes how FP64 partial sums are split over blocks, so a tuned
context must keep the oracle parity of an untuned one (relative 1e-12 for FP64
cycles, 1e-5 for FP32 cycles), and a cached tuning must apply exactly."""
import json

import numpy as np
import pytest
import torch

import helm_inputs as hi
from oracle.cycle import Problem, cycle

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_tuned_cycle_keeps_parity(prec, tol, tmp_path):
    from paper_2404_02493_amd import Helmholtz

    c = hi.make_problem(256, 160.0, 5, seed=4, medium="grf", phase="fmm", damping_cells=16)
    P = Problem(c.velocity, c.k, c.levels, damping_cells=16, phi=c.phi)
    H = Helmholtz(c.velocity, c.k, levels=c.levels, precision=prec, damping_cells=16)
    H.set_phase(c.phi)
    H.set_weights(P.weights.numpy())
    cache = str(tmp_path / "tune.json")
    res = H.tune(cache=cache)
    print(json.dumps(res), flush=True)
    assert res["fgmres_blocks"] in (256, 512, 1024, 2048)
    for l, rows in res["sstep_rows"].items():
        assert 2 <= int(l) <= c.levels and rows in (1, 2, 16, 24, 32, 40, 48, 64, 80, 96, 128)
    assert H.get_tuning()["sstep_rows"] == res["sstep_rows"]
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal((256, 256)) + 1j * rng.standard_normal((256, 256))
    u0[0, :] = 0
    u0[:, 0] = 0
    g = torch.as_tensor(c.g)
    ref = cycle(P, g.to(torch.complex128), torch.as_tensor(u0))
    dt = H.cdtype
    gd = g.to(dt).to("cuda:0")
    ud = torch.as_tensor(u0).to(dt).to("cuda:0")
    if prec == "c64":  # the oracle sees the rounded inputs
        ref = cycle(P, g.to(dt).to(torch.complex128), torch.as_tensor(u0).to(dt).to(torch.complex128))
    H.cycle(gd, ud)
    err = (torch.linalg.norm(ud.cpu().to(torch.complex128) - ref) / torch.linalg.norm(ref)).item()
    assert err < tol, err
    # a second context takes the cached choice without measuring
    H2 = Helmholtz(c.velocity, c.k, levels=c.levels, precision=prec, damping_cells=16)
    res2 = H2.tune(cache=cache)
    assert res2 == res
    assert H2.get_tuning()["fgmres_blocks"] == res["fgmres_blocks"]
    H.close()
    H2.close()


def test_set_tuning_rejects_bad_input():
    from paper_2404_02493_amd import Helmholtz, HelmError

    c = hi.make_problem(128, 80.0, 4, seed=1, medium="const", phase="analytic", damping_cells=16)
    H = Helmholtz(c.velocity, c.k, levels=c.levels, damping_cells=16)
    before = H.get_tuning()
    for bad in ['{"sstep_rows": {"9": 16}}', '{"fgmres_blocks": 99999}', '{"sstep_rows": {"2": x}}',
                '{"sstep_rows": {"2": 8}}', '{"sstep_rows": {"2": 36}}']:
        with pytest.raises(HelmError):
            H.set_tuning(bad)
        assert H.get_tuning() == before
    H.set_tuning('{"sstep_rows": {"2": 32}, "fgmres_blocks": 512}')
    t = H.get_tuning()
    assert t["sstep_rows"] == {"2": 32} and t["fgmres_blocks"] == 512
    H.close()


@pytest.mark.parametrize("form", [1, 2])
@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_tile_form_keeps_parity(form, prec, tol):
    """The overlapped-tile form of the s-step passes (forced on every ADR level, the
    level-2 post-smoother's fused epilogues still marching; the coarsest ADR level in
    the s-step form too, so that its pass adds the prolongation itself) keeps the oracle
    parity."""
    from paper_2404_02493_amd import Helmholtz

    c = hi.make_problem(256, 160.0, 5, seed=6, medium="grf", phase="fmm", damping_cells=16)
    P = Problem(c.velocity, c.k, c.levels, damping_cells=16, phi=c.phi)
    H = Helmholtz(c.velocity, c.k, levels=c.levels, precision=prec, damping_cells=16, tail_n=0)
    H.set_phase(c.phi)
    H.set_weights(P.weights.numpy())
    H.set_tuning(json.dumps({"sstep_rows": {"2": form, "3": form, "4": form}}))
    assert H.get_tuning()["sstep_rows"] == {"2": form, "3": form, "4": form}
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal((256, 256)) + 1j * rng.standard_normal((256, 256))
    u0[0, :] = 0
    u0[:, 0] = 0
    dt = H.cdtype
    g = torch.as_tensor(c.g).to(dt)
    u0t = torch.as_tensor(u0).to(dt)
    ref = cycle(P, g.to(torch.complex128), u0t.to(torch.complex128))
    ud = u0t.to("cuda:0")
    H.cycle(g.to("cuda:0"), ud)
    err = (torch.linalg.norm(ud.cpu().to(torch.complex128) - ref) / torch.linalg.norm(ref)).item()
    print(form, prec, f"{err:.2e}", flush=True)
    assert err < tol, err
    # GMRES from a nonzero iterate on level 2 through the tile passes alone
    from oracle.adr import apply_M, gmres
    n2 = 128
    x0 = torch.as_tensor(rng.standard_normal((n2, n2)) + 1j * rng.standard_normal((n2, n2))).to(dt)
    b = torch.as_tensor(rng.standard_normal((n2, n2)) + 1j * rng.standard_normal((n2, n2))).to(dt)
    for t in (x0, b):
        t[0, :] = 0
        t[:, 0] = 0
    out = H.debug_op(7, 2, x0.to("cuda:0"), b.to("cuda:0"))
    refg = gmres(lambda v: apply_M(v, P.adr[2]), b.to(torch.complex128), x0.to(torch.complex128), P.gmres_m)
    errg = (torch.linalg.norm(out.cpu().to(torch.complex128) - refg) / torch.linalg.norm(refg)).item()
    assert errg < tol, errg
    H.close()
