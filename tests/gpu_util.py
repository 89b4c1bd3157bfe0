"""Helpers shared by the GPU parity tests (comparison measures, oracle/GPU pairs).

Every comparison is made twice: as a relative 2-norm over the whole grid and
element by element, max |gpu - ref| <= 10 tol max |ref|, so that an error confined
to a few nodes (the ring, the open edge, a tile seam) cannot hide in the norm.
"""
import numpy as np
import torch

TOL = {"c128": 1e-12, "c64": 1e-5}
ELEM_FACTOR = 10.0


def _c128(x):
    return x.detach().cpu().to(torch.complex128)


def rel(a, b):
    a, b = _c128(a), _c128(b)
    return (torch.linalg.norm(a - b) / torch.linalg.norm(b)).item()


def elem(a, b):
    """max |a - b| / max |b|."""
    a, b = _c128(a), _c128(b)
    return ((a - b).abs().max() / b.abs().max()).item()


def measure(a, b):
    """(relative 2-norm, element-wise) pair of a result against its reference."""
    return rel(a, b), elem(a, b)


def within(m, tol):
    r, e = m
    return r < tol and e < ELEM_FACTOR * tol


def assert_close(a, b, tol, what=""):
    r, e = measure(a, b)
    assert r < tol and e < ELEM_FACTOR * tol, f"{what}: rel {r:.3e}, elem {e:.3e} (tol {tol:g})"
    return r, e


def rand_grid(rng, n, dtype=torch.complex128):
    """Random complex grid of n x n (or of shape n = (rows, columns)), zero on the ring;
    values representable in ``dtype``."""
    shape = (n, n) if isinstance(n, int) else tuple(n)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    v[0, :] = 0
    v[:, 0] = 0
    return torch.as_tensor(v).to(dtype).to(torch.complex128)


def to_dev(x, dtype):
    return x.to(dtype).to("cuda:0").contiguous()


def rounded(x, dtype):
    """Input as the GPU sees it, upcast back for the oracle."""
    return x.to(dtype).to(torch.complex128)


def make_pair(case, prec, gmres_arnoldi=0, tail_n=64, tuning=None, **kw):
    """(oracle Problem, GPU Helmholtz) on the same case, with the oracle's default
    weights passed to the library; ``tuning`` is a helm_set_tuning JSON dict."""
    import json

    from oracle.cycle import Problem
    from paper_2404_02493_amd import Helmholtz

    P = Problem(case.velocity, case.k, case.levels, damping_cells=case.damping_cells, phi=case.phi, **kw)
    H = Helmholtz(case.velocity, case.k, levels=case.levels, precision=prec, damping_cells=case.damping_cells,
                  gmres_arnoldi=gmres_arnoldi, tail_n=tail_n,
                  **{k: (v if isinstance(v, float) else int(v)) for k, v in kw.items()})
    H.set_phase(case.phi)
    H.set_weights(P.weights.numpy())
    if tuning is not None:
        H.set_tuning(json.dumps(tuning))
    return P, H


def operator_report(c, P, H, prec, rng):
    """Every internal operator of the library on identical random inputs against the
    oracle: {name: (relative 2-norm, element-wise)}."""
    from oracle.adr import adr_step, adr_vcycle, apply_M, gmres
    from oracle.cycle import cycle, wave_adr_cycle
    from oracle.grid import apply_A, prolong_bilinear, restrict_fw
    from oracle.smooth import chebyshev, jacobi

    _rand = rand_grid
    cd = H.cdtype
    L = c.levels
    report = {}

    def shape(l, half=False):  # (rows, columns) of level l (half: of level l + 1)
        s = l if not half else l + 1
        return (c.rows >> (s - 1), c.n >> (s - 1))

    for l in range(1, L + 1):
        nl = shape(l)
        dt = H.level_dtype(l)
        x = rounded(_rand(rng, nl), dt)
        out = H.debug_op(1, l, to_dev(x, dt), out_dtype=dt)
        report[f"A{l}"] = measure(out, apply_A(x, P.kappa[l], P.h[l]))
        if l < L:
            dtc = H.level_dtype(l + 1)
            out = H.debug_op(2, l, to_dev(x, dt), out_shape_level=l + 1, out_dtype=dtc)
            report[f"R{l}"] = measure(out, restrict_fw(x))
            e = rounded(_rand(rng, shape(l, True)), dtc)
            base = rounded(_rand(rng, nl), dt)
            outp = to_dev(base, dt)
            H.debug_op(3, l, to_dev(e, dtc), out=outp)
            report[f"P{l}"] = measure(outp, base + prolong_bilinear(e))
            g = rounded(_rand(rng, nl), dt)
            out = H.debug_op(11, l, to_dev(x, dt), to_dev(g, dt), out_shape_level=l + 1, out_dtype=dtc)
            report[f"RR{l}"] = measure(out, restrict_fw(g - apply_A(x, P.kappa[l], P.h[l])))
    # Jacobi (level 1)
    x, g = rounded(_rand(rng, shape(1)), cd), rounded(_rand(rng, shape(1)), cd)
    out = H.debug_op(4, 1, to_dev(x, cd), to_dev(g, cd))
    report["J1"] = measure(out, jacobi(x, g, P.kappa[1], P.h[1], P.weights[0]))
    # Chebyshev on level 2 (pre count) and the coarsest level
    for l, m in [(2, P.cheb_pre), (L, P.cheb_coarse)]:
        nl = shape(l)
        dt = H.level_dtype(l)
        x, g = rounded(_rand(rng, nl), dt), rounded(_rand(rng, nl), dt)
        out = H.debug_op(5, l, to_dev(x, dt), to_dev(g, dt), out_dtype=dt)
        report[f"C{l}"] = measure(out, chebyshev(x, g, P.kappa[l], P.h[l], P.weights[l - 1], m, P.lam[l]))
    # ADR operator on every ADR level
    for l in range(2, P.LA + 1):
        nl = shape(l)
        x = rounded(_rand(rng, nl), cd)
        out = H.debug_op(6, l, to_dev(x, cd))
        report[f"M{l}"] = measure(out, apply_M(x, P.adr[l]))
    # GMRES(3) from a nonzero x0 on level 2
    n2 = shape(2)
    x0, b = rounded(_rand(rng, n2), cd), rounded(_rand(rng, n2), cd)
    out = H.debug_op(7, 2, to_dev(x0, cd), to_dev(b, cd))
    report["G2"] = measure(out, gmres(lambda v: apply_M(v, P.adr[2]), b, x0, P.gmres_m))
    # ADR V-cycle from level 2
    out = H.debug_op(8, 2, None, to_dev(b, cd))
    report["V2"] = measure(out, adr_vcycle(P, 2, b, None))
    # one ADR step on level 2
    u2, g2 = rounded(_rand(rng, n2), cd), rounded(_rand(rng, n2), cd)
    out = H.debug_op(9, 2, to_dev(u2, cd), to_dev(g2, cd))
    report["S2"] = measure(out, adr_step(P, g2, u2))
    # coarse cycle from level 2 with zero iterate
    out = H.debug_op(10, 2, None, to_dev(g2, cd))
    report["W2"] = measure(out, wave_adr_cycle(P, 2, g2, torch.zeros_like(g2)))
    # fine cycle from a random iterate
    u, g = rounded(_rand(rng, shape(1)), cd), rounded(_rand(rng, shape(1)), cd)
    out = H.debug_op(10, 1, to_dev(u, cd), to_dev(g, cd))
    report["W1"] = measure(out, cycle(P, g, u))
    # fine cycle from a zero iterate (the preconditioner application inside FGMRES)
    out = H.debug_op(10, 1, None, to_dev(g, cd))
    report["W1z"] = measure(out, cycle(P, g, torch.zeros_like(g)))
    return report


def check_report(report, tol):
    bad = {k: v for k, v in report.items() if not within(v, tol)}
    print({k: f"{v[0]:.2e}/{v[1]:.2e}" for k, v in report.items()}, flush=True)
    assert not bad, bad


