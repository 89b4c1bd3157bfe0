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

__all__ = ["Helmholtz", "HelmholtzBatch", "HelmDesc", "HelmError", "HELM_C64", "HELM_C128", "lib", "lib_path", "default_desc"]


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

    velocity: (ny, n) wave speed c(x) > 0 (numpy or torch; copied to the device as float64):
    n nodes per row (x) and ny rows (y), powers of two; ny != n is a non-square domain
    with h = 1/max(n, ny).  Every grid argument below has this shape on the fine level.
    precision: "c128" (FP64 cycles) or "c64" (FP32 cycles; the coarsest level stays FP64).
    Remaining keyword arguments set the fields of ``helm_desc``.
    """

    def __init__(self, velocity, k: float, levels: int | None = None, precision: str = "c128",
                 device: str = "cuda:0", stream=None, **fields):
        torch = _torch()
        self.device = torch.device(device)
        vel = torch.as_tensor(np.asarray(velocity) if not isinstance(velocity, torch.Tensor) else velocity)
        vel = vel.to(device=self.device, dtype=torch.float64).contiguous()
        ny, n = int(vel.shape[0]), int(vel.shape[1])
        d = default_desc(n, k)
        if ny != n:
            d.ny = ny
            lg = int(np.log2(min(n, ny)))
            d.levels = max(2, min(7, lg - 3))
        if levels is not None:
            d.levels = int(levels)
        d.cycle_prec = HELM_C64 if precision == "c64" else HELM_C128
        for key, val in fields.items():
            if not hasattr(d, key):
                raise TypeError(f"unknown field {key}")
            setattr(d, key, val)
        self.desc = d
        self.n = n
        self.ny = ny
        self.shape = (ny, n)
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

    def eikonal(self, sources, max_rounds: int = 1000, tol: float = 1e-10, tau1_out=None, phi_out=None,
                stream=None):
        """Travel-time phase of the point sources, computed on the device (factored
        eikonal equation, fast sweeping) and installed as the ADR phase; one source
        uses product-rule phase derivatives.  tau1_out / phi_out: optional float64
        device tensors of the grid's shape.  Returns (rounds, last-round largest decrease)."""
        torch = _torch()
        src = np.ascontiguousarray(np.atleast_2d(np.asarray(sources, dtype=np.float64)))
        for t in (tau1_out, phi_out):
            if t is not None and (t.dtype != torch.float64 or tuple(t.shape) != self.shape
                                  or not t.is_contiguous() or t.device != self.device):
                raise ValueError("tau1_out / phi_out must be contiguous float64 tensors of the grid's shape on the "
                                 "context's device")
        rounds = ctypes.c_int32(0)
        change = ctypes.c_double(0.0)
        check(lib().helm_eikonal(self._ctx, src.ctypes.data, int(src.shape[0]), int(max_rounds), float(tol),
                                 _ptr(tau1_out) if tau1_out is not None else None,
                                 _ptr(phi_out) if phi_out is not None else None,
                                 ctypes.byref(rounds), ctypes.byref(change), _stream_ptr(stream)))
        return int(rounds.value), float(change.value)

    def set_rays(self, count: int = 8, stream=None):
        """Wave-Ray phases: the ADR corrections cycle through count plane waves."""
        check(lib().helm_set_rays(self._ctx, int(count), _stream_ptr(stream)))

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
        if tuple(t.shape) != self.shape:
            raise ValueError(f"expected a {self.shape} grid, got {tuple(t.shape)}")
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

    def residual(self, g, u, r=None, noalloc: bool = False, stream=None):
        """(r = g - A u, ||r||, ||g||) in FP64; noalloc=True takes the entry point whose
        reduction scratch is the library's static device array (no allocation)."""
        torch = _torch()
        g = self._grid(g, torch.complex128)
        u = self._grid(u, torch.complex128)
        r = torch.empty_like(g) if r is None else r
        rn = ctypes.c_double()
        gn = ctypes.c_double()
        fn = lib().helm_residual_noalloc if noalloc else lib().helm_residual
        check(fn(self._ctx, _ptr(g), _ptr(u), _ptr(r), ctypes.byref(rn), ctypes.byref(gn), _stream_ptr(stream)))
        return r, rn.value, gn.value

    # ------------------------------------------------------------------ unrolled cycles and their adjoint
    def loss(self, g, u, grad: bool = False, stream=None):
        """L = ||g - A u||^2 (FP64) for cycle-dtype device grids g, u; with grad=True also
        dL/du in torch's complex convention.  Returns (L, grad_u or None)."""
        torch = _torch()
        gu = torch.empty_like(u) if grad else None
        val = ctypes.c_double()
        check(lib().helm_loss(self._ctx, _ptr(g), _ptr(u), ctypes.byref(val), _ptr(gu), _stream_ptr(stream)))
        return val.value, gu

    def cycle_backward(self, K: int, g, grad_uK, u0=None, ckpt=None, stream=None):
        """Cotangents of the phase and of the weights for u_K = C^K(u_0, g), given the
        cotangent of u_K.  Returns (grad_phi device tensor of the grid's shape, grad_w
        (levels,) float64 device tensor)."""
        torch = _torch()
        pdt = torch.float32 if self.cdtype == torch.complex64 else torch.float64
        gphi = torch.empty(self.shape, dtype=pdt, device=self.device)
        gw = torch.empty((self.levels,), dtype=torch.float64, device=self.device)
        check(lib().helm_cycle_backward(self._ctx, int(K), _ptr(g), _ptr(u0), _ptr(grad_uK), _ptr(gphi), _ptr(gw),
                                        _ptr(ckpt), _stream_ptr(stream)))
        return gphi, gw

    def cycle_record(self, K: int, g, u_out, u0=None, ckpt=None, stream=None):
        """u_out <- u_K = C^K(u_0, g) with every cycle recorded on its own tape for
        cycle_reverse (helm_cycle_record).  Raises HelmError (HELM_ENOMEM) when the K tapes
        do not fit; cycle_backward still applies then."""
        check(lib().helm_cycle_record(self._ctx, int(K), _ptr(g), _ptr(u0), _ptr(u_out), _ptr(ckpt),
                                      _stream_ptr(stream)))
        return u_out

    def cycle_reverse(self, K: int, g, grad_uK, stream=None):
        """The cotangents of cycle_backward from the tapes of the last cycle_record (same K
        and g, phase and weights unchanged since).  Returns (grad_phi, grad_w)."""
        torch = _torch()
        pdt = torch.float32 if self.cdtype == torch.complex64 else torch.float64
        gphi = torch.empty(self.shape, dtype=pdt, device=self.device)
        gw = torch.empty((self.levels,), dtype=torch.float64, device=self.device)
        check(lib().helm_cycle_reverse(self._ctx, int(K), _ptr(g), _ptr(grad_uK), _ptr(gphi), _ptr(gw),
                                       _stream_ptr(stream)))
        return gphi, gw

    def unrolled(self, phi, w, g, K: int):
        """u_K after K cycles from u_0 = 0 as a differentiable function of the phase phi
        (tensor of the grid's shape) and the weights w (levels float64 tensor); g is a cycle-dtype
        device grid.  The forward pass records the cycles (helm_cycle_record) and the
        backward pass reverses them (helm_cycle_reverse); when the tapes do not fit, the
        forward runs plain cycles and the backward is helm_cycle_backward.  The phase and
        the weights must stay as the forward pass set them until its backward pass."""
        return _Unrolled.apply(phi, w, g, self, int(K))

    def residual_loss(self, g, u):
        """Differentiable L = ||g - A u||^2 (float64 device scalar) of a cycle-dtype grid u."""
        return _Loss.apply(u, g, self)

    def debug_op(self, op: int, level: int, x=None, x2=None, out=None, out_shape_level=None, out_dtype=None,
                 stream=None):
        """Runs one internal operator (see helm_debug_op in include/helm.h)."""
        torch = _torch()
        lvl = out_shape_level if out_shape_level is not None else level
        if out is None:
            out = torch.zeros((self.ny >> (lvl - 1), self.n >> (lvl - 1)), dtype=out_dtype or self.cdtype,
                              device=self.device)
        check(lib().helm_debug_op(self._ctx, int(op), int(level), _ptr(x), _ptr(x2), _ptr(out), _stream_ptr(stream)))
        return out

    # ------------------------------------------------------------------ autotuning
    def tuning_key(self) -> str:
        torch = _torch()
        d = self.desc
        name = torch.cuda.get_device_name(self.device)
        size = f"n={self.n}" if self.ny == self.n else f"n={self.n}x{self.ny}"
        return (f"{name}|{size}|L={self.levels}|{'c64' if self.cdtype == torch.complex64 else 'c128'}"
                f"|m={d.gmres_m}/{d.gmres_coarse_m}|adr={d.adr_levels}|tail={d.tail_n}|arnoldi={d.gmres_arnoldi}"
                f"|restart={d.restart}|v4")

    def tune(self, cache: str | None = None, stream=None) -> dict:
        """Chooses launch shapes by measurement (helm_tune) and applies them.  With a
        cache path (JSON file), a stored choice for the same device / size / precision /
        solver shape is applied instead of measuring, and new measurements are stored."""
        import json

        key = self.tuning_key() if cache else None
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_tuning(table[key])
                return table[key]
        buf = ctypes.create_string_buffer(1 << 16)
        check(lib().helm_tune(self._ctx, buf, len(buf), _stream_ptr(stream)))
        res = json.loads(buf.value.decode())
        if cache:
            table[key] = res
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return res

    def set_tuning(self, tuning):
        import json

        text = tuning if isinstance(tuning, str) else json.dumps(tuning)
        check(lib().helm_set_tuning(self._ctx, text.encode()))

    def get_tuning(self) -> dict:
        import json

        buf = ctypes.create_string_buffer(1 << 12)
        check(lib().helm_get_tuning(self._ctx, buf, len(buf)))
        return json.loads(buf.value.decode())

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


class _Borrowed(Helmholtz):
    """A problem context owned by a batch (not destroyed by this object)."""

    def __init__(self, ctx, n, levels, cdtype, device, ny=None):
        self._ctx = ctx
        self.n, self.levels, self.cdtype, self.device = n, levels, cdtype, device
        self.ny = n if ny is None else ny
        self.shape = (self.ny, self.n)

    def close(self):
        self._ctx = ctypes.c_void_p()


class HelmholtzBatch:
    """Independent problems of mixed sizes solved together (helm_batch_* in include/helm.h).

    problems: list of dicts with keys velocity ((ny, n), ny = n for the square), k, and optionally levels, phi,
    damping_cells and any other helm_desc field.  lanes: problems in flight at once."""

    def __init__(self, problems, precision: str = "c64", lanes: int = 4, device: str = "cuda:0", stream=None):
        torch = _torch()
        self.device = torch.device(device)
        self.cdtype = torch.complex64 if precision == "c64" else torch.complex128
        descs = (HelmDesc * len(problems))()
        vels, phis, keep = [], [], []
        self.sizes = []
        for p, prob in enumerate(problems):
            vel = torch.as_tensor(np.asarray(prob["velocity"], dtype=np.float64)).to(self.device).contiguous()
            ny, n = int(vel.shape[0]), int(vel.shape[1])
            d = default_desc(n, float(prob["k"]))
            if ny != n:
                d.ny = ny
                d.levels = max(2, min(7, int(np.log2(min(n, ny))) - 3))
            d.cycle_prec = HELM_C64 if precision == "c64" else HELM_C128
            for key, val in prob.items():
                if key in ("velocity", "k", "phi"):
                    continue
                if not hasattr(d, key):
                    raise TypeError(f"unknown field {key}")
                setattr(d, key, val)
            descs[p] = d
            phi = prob.get("phi")
            pt = None
            if phi is not None:
                pt = torch.as_tensor(np.asarray(phi, dtype=np.float64)).to(self.device).contiguous()
            keep += [vel, pt]
            vels.append(vel.data_ptr())
            phis.append(pt.data_ptr() if pt is not None else None)
            self.sizes.append((n, int(d.levels), ny))
        VA = ctypes.c_void_p * len(problems)
        self._b = ctypes.c_void_p()
        check(lib().helm_batch_setup(len(problems), descs, VA(*vels), VA(*phis), 1, int(lanes),
                                     ctypes.byref(self._b), _stream_ptr(stream)))
        self.nprob = len(problems)

    def problem(self, p: int) -> Helmholtz:
        """The single-problem view of problem p (for set_weights, cycle, ...)."""
        ctx = ctypes.c_void_p()
        check(lib().helm_batch_get(self._b, int(p), ctypes.byref(ctx)))
        n, L, ny = self.sizes[p]
        return _Borrowed(ctx, n, L, self.cdtype, self.device, ny)

    def solve(self, gs, us=None, tol: float = 1e-6, maxit: int = 1000, mode: int = 1, stream=None):
        """Solves every problem; gs, us: lists of complex128 device grids.  Returns
        (us, iters, relres, status) with numpy arrays of per-problem results."""
        torch = _torch()
        gs = [g.to(device=self.device, dtype=torch.complex128).contiguous() for g in gs]
        us = [torch.zeros_like(g) for g in gs] if us is None else us
        VA = ctypes.c_void_p * self.nprob
        its = (ctypes.c_int32 * self.nprob)()
        rr = (ctypes.c_double * self.nprob)()
        st = (ctypes.c_int32 * self.nprob)()
        code = lib().helm_batch_solve(self._b, VA(*[g.data_ptr() for g in gs]), VA(*[u.data_ptr() for u in us]),
                                      float(tol), int(maxit), int(mode), its, rr, st, _stream_ptr(stream))
        if code not in (0, 4):
            check(code)
        return us, np.array(its[:]), np.array(rr[:]), np.array(st[:])

    def classes(self) -> np.ndarray:
        """Lockstep class of every problem at the last solve (-1: it ran alone)."""
        out = (ctypes.c_int32 * self.nprob)()
        check(lib().helm_batch_classes(self._b, out))
        return np.array(out[:])

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            lib().helm_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    torch = _torch()

    class Unrolled(torch.autograd.Function):
        @staticmethod
        def forward(ctx, phi, w, g, helm, K):
            helm.set_phase(phi.detach())
            helm.set_weights([float(x) for x in w.detach().cpu().tolist()])
            u = torch.empty_like(g)
            try:
                helm.cycle_record(K, g, u)
                ctx.recorded = True
            except HelmError as e:
                if e.status != 2:  # HELM_ENOMEM: the tapes do not fit
                    raise
                u.zero_()
                for _ in range(K):
                    helm.cycle(g, u)
                ctx.recorded = False
            ctx.helm, ctx.K = helm, K
            ctx.phi_meta = (phi.dtype, phi.device)
            ctx.w_meta = (w.dtype, w.device)
            ctx.save_for_backward(g)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            (g,) = ctx.saved_tensors
            helm = ctx.helm
            gu = grad_u.contiguous().to(g.dtype)
            if ctx.recorded:
                gphi, gw = helm.cycle_reverse(ctx.K, g, gu)
            else:
                gphi, gw = helm.cycle_backward(ctx.K, g, gu)
            return (gphi.to(dtype=ctx.phi_meta[0], device=ctx.phi_meta[1]),
                    gw.to(dtype=ctx.w_meta[0], device=ctx.w_meta[1]), None, None, None)

    class Loss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u, g, helm):
            val, gu = helm.loss(g, u.contiguous(), grad=True)
            ctx.save_for_backward(gu)
            return torch.tensor(val, dtype=torch.float64, device=u.device)

        @staticmethod
        def backward(ctx, grad_out):
            (gu,) = ctx.saved_tensors
            return gu * grad_out.to(gu.real.dtype), None, None

    return Unrolled, Loss


class _Lazy:
    def __init__(self, idx):
        self.idx = idx
        self.cls = None

    def apply(self, *args):
        if self.cls is None:
            self.cls = _autograd_function()[self.idx]
        return self.cls.apply(*args)


_Unrolled = _Lazy(0)
_Loss = _Lazy(1)
