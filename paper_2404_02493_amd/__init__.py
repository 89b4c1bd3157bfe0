"""MI355X (gfx950) Wave-ADR Helmholtz solver: thin Python binding of libhelm.so.

Every grid operation runs in the HIP kernels of libhelm.so; this module only
marshals arguments (device pointers of torch tensors, the current HIP stream).
Importing it fails loudly when the library has not been built; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from ._abi import HELM_C64, HELM_C128, HelmDesc, HelmError, lib, lib_path, check

__all__ = ["Helmholtz", "HelmDesc", "HelmError", "HELM_C64", "HELM_C128", "lib", "lib_path", "default_desc"]


def _torch():
    import torch

    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def default_desc(n: int, k: float) -> HelmDesc:
    d = HelmDesc()
    lib().helm_desc_default(ctypes.byref(d), int(n), float(k))
    return d


class Helmholtz:
    """One discrete damped Helmholtz problem on the GPU with its Wave-ADR hierarchy.

    velocity: (n, n) wave speed c(x) > 0 (numpy or torch; copied to the device as float64).
    precision: "c128" (FP64 cycles) or "c64" (FP32 cycles; the coarsest level stays FP64).
    Remaining keyword arguments set the fields of ``helm_desc``.
    """

    def __init__(self, velocity, k: float, levels: int | None = None, precision: str = "c128",
                 device: str = "cuda:0", stream=None, **fields):
        torch = _torch()
        self.device = torch.device(device)
        vel = torch.as_tensor(np.asarray(velocity) if not isinstance(velocity, torch.Tensor) else velocity)
        vel = vel.to(device=self.device, dtype=torch.float64).contiguous()
        n = int(vel.shape[0])
        d = default_desc(n, k)
        if levels is not None:
            d.levels = int(levels)
        d.cycle_prec = HELM_C64 if precision == "c64" else HELM_C128
        for key, val in fields.items():
            if not hasattr(d, key):
                raise TypeError(f"unknown field {key}")
            setattr(d, key, val)
        self.desc = d
        self.n = n
        self.levels = int(d.levels)
        self.cdtype = torch.complex64 if d.cycle_prec == HELM_C64 else torch.complex128
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().helm_setup(ctypes.byref(d), _ptr(vel), ctypes.byref(self._ctx), _stream_ptr(stream)))
        self._vel = vel

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().helm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ parameters
    def set_phase(self, phi, stream=None):
        torch = _torch()
        t = torch.as_tensor(np.asarray(phi) if not isinstance(phi, torch.Tensor) else phi)
        is64 = t.dtype == torch.float64
        t = t.to(device=self.device, dtype=torch.float64 if is64 else torch.float32).contiguous()
        self._phi = t
        check(lib().helm_set_phase(self._ctx, _ptr(t), int(is64), _stream_ptr(stream)))

    @property
    def weights(self) -> np.ndarray:
        w = (ctypes.c_double * self.levels)()
        check(lib().helm_get_weights(self._ctx, w))
        return np.array(w[:], dtype=np.float64)

    def set_weights(self, w):
        arr = (ctypes.c_double * self.levels)(*[float(x) for x in w])
        check(lib().helm_set_weights(self._ctx, arr))

    @property
    def lambdas(self) -> np.ndarray:
        w = (ctypes.c_double * self.levels)()
        check(lib().helm_get_lambdas(self._ctx, w))
        return np.array(w[:], dtype=np.float64)

    # ------------------------------------------------------------------ operations
    def _grid(self, x, dtype=None):
        torch = _torch()
        dtype = dtype or self.cdtype
        t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x))
        t = t.to(device=self.device, dtype=dtype).contiguous()
        if tuple(t.shape) != (self.n, self.n):
            raise ValueError(f"expected a ({self.n}, {self.n}) grid, got {tuple(t.shape)}")
        return t

    def cycle(self, g, u, stream=None):
        """u <- C(u, g) in place (u must be a contiguous device tensor of the cycle dtype)."""
        check(lib().helm_cycle(self._ctx, _ptr(g), _ptr(u), _stream_ptr(stream)))
        return u

    def solve(self, g, u=None, tol: float = 1e-6, maxit: int = 1000, mode: int = 0, stream=None,
              raise_on_noconv: bool = False):
        """Returns (u, iterations, relres, history); g, u complex128 device tensors."""
        torch = _torch()
        g = self._grid(g, torch.complex128)
        u = torch.zeros_like(g) if u is None else self._grid(u, torch.complex128)
        its = ctypes.c_int32()
        rr = ctypes.c_double()
        hist = (ctypes.c_double * (maxit + 1))()
        st = lib().helm_solve(self._ctx, _ptr(g), _ptr(u), float(tol), int(maxit), int(mode), ctypes.byref(its),
                              ctypes.byref(rr), hist, _stream_ptr(stream))
        if st not in (0, 4) or (st == 4 and raise_on_noconv):
            check(st)
        n = its.value if mode == 0 else len([h for h in hist[: maxit + 1] if h > 0])
        return u, its.value, rr.value, np.array(hist[: max(n, 0)])

    def residual(self, g, u, stream=None):
        torch = _torch()
        g = self._grid(g, torch.complex128)
        u = self._grid(u, torch.complex128)
        r = torch.empty_like(g)
        rn = ctypes.c_double()
        gn = ctypes.c_double()
        check(lib().helm_residual(self._ctx, _ptr(g), _ptr(u), _ptr(r), ctypes.byref(rn), ctypes.byref(gn),
                                  _stream_ptr(stream)))
        return r, rn.value, gn.value

    def debug_op(self, op: int, level: int, x=None, x2=None, out=None, out_shape_level=None, out_dtype=None,
                 stream=None):
        """Runs one internal operator (see helm_debug_op in include/helm.h)."""
        torch = _torch()
        lvl = out_shape_level if out_shape_level is not None else level
        nl = self.n >> (lvl - 1)
        if out is None:
            out = torch.zeros((nl, nl), dtype=out_dtype or self.cdtype, device=self.device)
        check(lib().helm_debug_op(self._ctx, int(op), int(level), _ptr(x), _ptr(x2), _ptr(out), _stream_ptr(stream)))
        return out

    def profile_begin(self):
        check(lib().helm_profile_begin(self._ctx))

    def profile_end(self) -> dict:
        import json

        buf = ctypes.create_string_buffer(1 << 20)
        check(lib().helm_profile_end(self._ctx, buf, len(buf)))
        return json.loads(buf.value.decode())

    def level_dtype(self, level: int):
        torch = _torch()
        if level == self.levels:
            return torch.complex128
        return self.cdtype
