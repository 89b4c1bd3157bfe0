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
    """Random complex grid, zero on the ring; values representable in ``dtype``."""
    v = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
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
