"""Factored eikonal phase and its product-rule derivatives (Section 3.2.1).

Test infrastructure only (see the package docstring).

The travel time is tau = tau0 * tau1 with tau0 = |x - x0| (eq. eikonal_cons) and
tau1 from the factored equation |tau0 grad tau1 + tau1 grad tau0|^2 = s^2, solved
by the plain C code of ``eikonal.c`` (fast sweeping).  The ADR coefficients then
take the derivatives of the phase from the product rule of Section 3.2.1,

    grad tau = tau0 grad tau1 + tau1 grad tau0,
    Lap tau  = tau1 Lap tau0 + 2 grad tau0 . grad tau1 + tau0 Lap tau1,

with grad tau0 = (x - x0)/r and Lap tau0 = 1/r (r = |x - x0|, two dimensions)
exact, and the finite-difference rule of the phase (second order inside, first
order at the open edge) applied to tau1.  Reading where the paper is silent: at a
level node closer to the source than one level spacing, tau0 is not smooth on the
stencil and the rule is applied to tau = tau0 tau1 itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import torch

from .adr import phase_derivatives
from .grid import _mask_ring

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eikonal.c")
_LIB = os.path.join(_HERE, "_eikonal.so")
_lib = None

F64 = torch.float64


def build(cc: str = "gcc") -> str:
    """Compile eikonal.c (no floating-point contraction) into oracle/_eikonal.so."""
    cmd = [cc, "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.c_void_p
        lib.oracle_eik_sweep.restype = ctypes.c_int
        lib.oracle_eik_sweep.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_double, dp, dp, dp]
        _lib = lib
    return _lib


def eikonal_sweep(slowness: np.ndarray, src, h: float, max_rounds: int = 100, tol: float = 0.0):
    """tau1 on the (rows, columns) nodes of ``slowness`` by fast sweeping; returns
    (tau1, rounds, last change)."""
    s = np.ascontiguousarray(slowness, dtype=np.float64)
    ny, n = s.shape
    t = np.empty((ny, n), dtype=np.float64)
    rounds = ctypes.c_int32(0)
    change = ctypes.c_double(0.0)
    rc = _load().oracle_eik_sweep(n, ny, h, s.ctypes.data, float(src[0]), float(src[1]), int(max_rounds), float(tol),
                                  t.ctypes.data, ctypes.addressof(rounds), ctypes.addressof(change))
    if rc != 0:
        raise ValueError(f"oracle_eik_sweep failed ({rc})")
    return t, int(rounds.value), float(change.value)


def tau0(n: int, h: float, src, ny: int | None = None) -> np.ndarray:
    """|x - x0| at the nodes (x = j h, y = i h) of n columns and ny rows (ny = n by default)."""
    ny = n if ny is None else ny
    X, Y = np.meshgrid(np.arange(n) * h, np.arange(ny) * h)
    return np.sqrt((X - src[0]) ** 2 + (Y - src[1]) ** 2)


def factored_phase(tau1: np.ndarray, src, h: float) -> np.ndarray:
    """tau = tau0 tau1."""
    return tau0(tau1.shape[1], h, src, tau1.shape[0]) * tau1


def factored_derivatives(tau1_l: torch.Tensor, src, h: float):
    """phi_x, phi_y and Lap phi at the unknowns of one level from tau1 on that level
    (injected) by the product rule, zero on the ring (same layout as
    ``phase_derivatives``)."""
    Y, X = torch.meshgrid(torch.arange(tau1_l.shape[0], dtype=F64) * h,
                          torch.arange(tau1_l.shape[1], dtype=F64) * h, indexing="ij")
    dx, dy = X - src[0], Y - src[1]
    r = torch.sqrt(dx * dx + dy * dy)
    near = r < h
    rs = torch.where(near, torch.ones_like(r), r)
    gx, gy, l0 = dx / rs, dy / rs, 1.0 / rs
    t1x, t1y, t1l = phase_derivatives(tau1_l, h)
    px = r * t1x + tau1_l * gx
    py = r * t1y + tau1_l * gy
    lap = tau1_l * l0 + 2.0 * (gx * t1x + gy * t1y) + r * t1l
    fx, fy, fl = phase_derivatives(r * tau1_l, h)
    px = torch.where(near, fx, px)
    py = torch.where(near, fy, py)
    lap = torch.where(near, fl, lap)
    return _mask_ring(px), _mask_ring(py), _mask_ring(lap)


def factored_adr_coefficients(tau1_l, src, n2_l, rho_l, k, strength, sigma, h, shift: float = 0.0):
    """Per-level ADR coefficients (eq. ADR) with the phase derivatives of
    ``factored_derivatives``; the same dictionary as ``adr.adr_coefficients``."""
    px, py, lap = factored_derivatives(tau1_l, src, h)
    delta = strength * rho_l * rho_l + shift
    c0 = (-1j * sigma * k) * lap + (k * k) * (px * px + py * py - n2_l) \
        - 1j * sigma * (k * k) * n2_l * delta
    return dict(px=px, py=py, c0=_mask_ring(c0), h=h, k=k, sigma=sigma)
