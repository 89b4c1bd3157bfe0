"""Seeded synthetic inputs for the Helmholtz problems (velocity, source, phase).

This module is shared by the CPU oracle and by the GPU path; it holds none of
the solver's arithmetic.  Every generator takes an explicit seed and draws from
``numpy.random.Generator(PCG64(seed))``.

Grid convention (both sides): n = 2^a columns (x) and ny = 2^b rows (y) of nodes
(ny = n for the square domains), h = 1/max(n, ny), node (i, j) sits at
(x, y) = (j h, i h); arrays are (ny, n), row-major, x fastest.  Row 0 and column 0
are the zero Dirichlet ring; the ring at index ny (rows) and n (columns) is implicit.

The paper's workloads use CIFAR-10, OpenFWI and STL-10 derived media, which
are not available; the media below are synthetic stand-ins of the same kind
(smooth random fields, layered models with inclusions), see ``make_case``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Case",
    "make_case",
    "make_problem",
    "gaussian_sources",
    "grf_velocity",
    "layered_velocity",
    "fmm_phase",
    "analytic_phase",
    "default_levels",
    "CONFIGS",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_FMM_LIB = os.path.join(_HERE, "_fmm.so")


@dataclass
class Case:
    """One Helmholtz problem instance (all arrays are numpy, host memory)."""

    name: str
    n: int
    k: float
    levels: int
    damping_cells: int
    velocity: np.ndarray  # (ny, n) float64, c(x) > 0
    g: np.ndarray  # (ny, n) complex128, zero on the boundary ring
    phi: np.ndarray  # (ny, n) float64 or float32
    sources: np.ndarray  # (ns, 2) source positions (x, y)
    meta: dict = field(default_factory=dict)
    ny: int = 0  # rows of nodes; 0: ny = n (square domain)

    @property
    def rows(self) -> int:
        return self.ny if self.ny else self.n

    @property
    def shape(self):
        return (self.rows, self.n)


def default_levels(n: int) -> int:
    """L = min(7, log2 n - 3)."""
    return int(min(7, int(np.log2(n)) - 3))


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_sources(n: int, xy: np.ndarray, sigma_cells: float = 2.0, ny: int | None = None) -> np.ndarray:
    """Sum of unit-mass Gaussians exp(-|x-x0|^2/(2 s^2)) / (2 pi s^2), s = sigma_cells*h,
    sampled at interior nodes; zero on the boundary ring."""
    ny = n if ny is None else ny
    h = 1.0 / max(n, ny)
    s = sigma_cells * h
    x = np.arange(n) * h
    y = np.arange(ny) * h
    g = np.zeros((ny, n), dtype=np.float64)
    for x0, y0 in np.atleast_2d(xy):
        gx = np.exp(-((x - x0) ** 2) / (2 * s * s))
        gy = np.exp(-((y - y0) ** 2) / (2 * s * s))
        g += np.outer(gy, gx) / (2 * np.pi * s * s)
    g[0, :] = 0.0
    g[:, 0] = 0.0
    return g.astype(np.complex128)


def _source_positions(rng: np.random.Generator, n: int, count: int, margin_cells: int,
                      ny: int | None = None) -> np.ndarray:
    ny = n if ny is None else ny
    h = 1.0 / max(n, ny)
    if ny == n:
        lo, hi = margin_cells * h, 1.0 - margin_cells * h
        return rng.uniform(lo, hi, size=(count, 2))
    lo = np.array([margin_cells * h, margin_cells * h])
    hi = np.array([n * h - margin_cells * h, ny * h - margin_cells * h])
    return rng.uniform(lo, hi, size=(count, 2))


def grf_velocity(rng: np.random.Generator, n: int, corr_len: float = 0.1,
                 cmin: float = 1.5, cmax: float = 4.5, ny: int | None = None) -> np.ndarray:
    """Gaussian random field with squared-exponential covariance exp(-r^2/(2 l^2)):
    white noise on a 2ny x 2n periodic grid, Gaussian filter of std l/sqrt(2),
    crop ny x n, affine min-max map to [cmin, cmax]."""
    ny = n if ny is None else ny
    h = 1.0 / max(n, ny)
    xi = rng.standard_normal((2 * ny, 2 * n))
    fy = np.fft.fftfreq(2 * ny, d=h)
    fx = np.fft.fftfreq(2 * n, d=h)
    s = corr_len / np.sqrt(2.0)
    filt = np.exp(-2.0 * (np.pi ** 2) * (s ** 2) * (fy[:, None] ** 2 + fx[None, :] ** 2))
    field_ = np.real(np.fft.ifft2(np.fft.fft2(xi) * filt))[:ny, :n]
    lo, hi = field_.min(), field_.max()
    return cmin + (cmax - cmin) * (field_ - lo) / (hi - lo)


def layered_velocity(rng: np.random.Generator, n: int, nlayers: int = 8, nellipses: int = 20,
                     cmin: float = 1.5, cmax: float = 4.5, contrast: float = 0.3,
                     smooth: float = 0.0, ny: int | None = None) -> np.ndarray:
    """Horizontal layers (sorted uniform interface depths, per-layer speed
    U[cmin, cmax]) plus elliptical inclusions multiplying the speed by
    (1 +/- contrast), applied in order; then, if smooth > 0, a Gaussian filter of
    standard deviation ``smooth`` (physical units, nearest-value boundaries).
    Depths and inclusion centres scale with the extents (n h, ny h) of the domain."""
    ny = n if ny is None else ny
    h = 1.0 / max(n, ny)
    ext_x, ext_y = n * h, ny * h
    depths = np.sort(rng.uniform(0.0, 1.0, size=nlayers - 1)) * ext_y
    speeds = rng.uniform(cmin, cmax, size=nlayers)
    y = np.arange(ny) * h
    layer = np.searchsorted(depths, y, side="right")
    c = np.repeat(speeds[layer][:, None], n, axis=1)
    X, Y = np.meshgrid(np.arange(n) * h, y)
    for _ in range(nellipses):
        cx, cy = rng.uniform(0.05, 0.95, size=2) * np.array([ext_x, ext_y])
        a, b = rng.uniform(0.02, 0.08, size=2)
        th = rng.uniform(0.0, np.pi)
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        dx, dy = X - cx, Y - cy
        u = dx * np.cos(th) + dy * np.sin(th)
        v = -dx * np.sin(th) + dy * np.cos(th)
        inside = (u / a) ** 2 + (v / b) ** 2 <= 1.0
        c = np.where(inside, c * (1.0 + sign * contrast), c)
    if smooth > 0.0:
        from scipy.ndimage import gaussian_filter

        c = gaussian_filter(c, smooth / h, mode="nearest")
    return c


def analytic_phase(n: int, xy: np.ndarray, slowness: float = 1.0, ny: int | None = None) -> np.ndarray:
    """phi = s * min over sources |x - x0| (exact eikonal solution for constant s)."""
    ny = n if ny is None else ny
    h = 1.0 / max(n, ny)
    X, Y = np.meshgrid(np.arange(n) * h, np.arange(ny) * h)
    d = np.full((ny, n), np.inf)
    for x0, y0 in np.atleast_2d(xy):
        d = np.minimum(d, np.hypot(X - x0, Y - y0))
    return slowness * d


def _load_fmm():
    if not os.path.exists(_FMM_LIB):
        raise RuntimeError(
            f"{_FMM_LIB} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(_FMM_LIB)
    lib.fmm_eikonal.restype = ctypes.c_int
    lib.fmm_eikonal.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    return lib


def fmm_phase(velocity: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """First-arrival travel time from the sources (first-order fast marching)."""
    ny, n = velocity.shape
    s = np.ascontiguousarray(1.0 / velocity, dtype=np.float64)
    src = np.ascontiguousarray(np.atleast_2d(xy), dtype=np.float64)
    T = np.empty((ny, n), dtype=np.float64)
    rc = _load_fmm().fmm_eikonal(n, ny, 1.0 / max(n, ny), s.ctypes.data, src.shape[0], src.ctypes.data,
                                 T.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"fmm_eikonal failed with code {rc}")
    return T


def build_fmm(cc: str = "gcc") -> str:
    """Compile the fast-marching helper into helm_inputs/_fmm.so."""
    import subprocess

    src = os.path.join(_HERE, "fmm.c")
    cmd = [cc, "-O2", "-shared", "-fPIC", "-o", _FMM_LIB, src, "-lm"]
    subprocess.run(cmd, check=True)
    return _FMM_LIB


# Workload recipes (sizes, media, sources).  k is the angular frequency.
CONFIGS = {
    # constant medium, 128 x 128, k = 80, analytic phase, 4 levels
    "const128": dict(n=128, k=80.0, levels=4, medium="const", nsrc=(1, 1), phase="analytic"),
    # smooth random medium, 512 x 512, k = 320, fast-marching phase
    "grf512": dict(n=512, k=320.0, levels=6, medium="grf", nsrc=(1, 1), phase="fmm"),
    # differentiation workload, 1024 x 1024, k = 640, float32 phase
    "grf1024": dict(n=1024, k=640.0, levels=7, medium="grf", nsrc=(1, 1), phase="fmm32"),
    # layered + inclusions smoothed over about one wavelength, 4096 x 4096, k = 2100
    "layered4096": dict(n=4096, k=2100.0, levels=7, medium="layered", nsrc=(1, 1), phase="fmm", smooth=0.01),
    # the same model without smoothing (sharp interfaces)
    "layered4096_sharp": dict(n=4096, k=2100.0, levels=7, medium="layered", nsrc=(1, 1), phase="fmm"),
    # non-square domain of aspect 4 (4096 columns, 1024 rows; the paper's non-square
    # seismic models are 3-4.5 times wider than deep), the same spacing and frequency
    "layered4096x1024": dict(n=4096, ny=1024, k=2100.0, levels=7, medium="layered", nsrc=(1, 1), phase="fmm",
                             smooth=0.01),
}


def sponge_cells(n: int, k: float, cmax: float, minimum: int = 16) -> int:
    """Sponge width in fine cells: one wavelength 2 pi c_max / k at the largest wave
    speed of the medium (the usual thickness of the damping layer), at least 16;
    n = 1/h, the node count of the longer side."""
    return int(max(minimum, int(np.ceil(2.0 * np.pi * cmax * n / k))))


def make_problem(n: int, k: float, levels: int, seed: int, medium: str = "const",
                 nsrc=(1, 1), phase: str = "analytic", damping_cells=None,
                 name: str = "custom", smooth: float = 0.0, ny: int | None = None) -> Case:
    """Build one seeded problem on n columns and ny rows of nodes (ny None: square).
    medium in {const, grf, layered}; phase in {analytic, fmm, fmm32};
    nsrc = (min, max) number of sources; damping_cells None = one wavelength at the
    top speed, at least 16."""
    rows = n if ny is None else ny
    rng = _rng(seed)
    count = int(rng.integers(nsrc[0], nsrc[1] + 1))
    if medium == "const":
        vel = np.ones((rows, n))
    elif medium == "grf":
        vel = grf_velocity(rng, n, ny=rows)
    elif medium == "layered":
        vel = layered_velocity(rng, n, smooth=smooth, ny=rows)
    else:
        raise ValueError(medium)
    if damping_cells is None:
        damping_cells = sponge_cells(max(n, rows), k, float(vel.max()))
    # sources at least 4 cells inside the sponge-free region
    xy = _source_positions(rng, n, count, damping_cells + 4, ny=rows)
    g = gaussian_sources(n, xy, ny=rows)
    if phase == "analytic":
        if medium != "const":
            raise ValueError("analytic phase needs a constant medium")
        phi = analytic_phase(n, xy, 1.0 / vel[0, 0], ny=rows)
    elif phase in ("fmm", "fmm32"):
        phi = fmm_phase(vel, xy)
        if phase == "fmm32":
            phi = phi.astype(np.float32)
    else:
        raise ValueError(phase)
    return Case(name=name, n=n, k=float(k), levels=int(levels), damping_cells=damping_cells,
                velocity=np.ascontiguousarray(vel, dtype=np.float64), g=g, phi=phi, sources=xy,
                meta=dict(seed=seed, medium=medium, phase=phase, smooth=smooth), ny=0 if rows == n else rows)


def make_case(name: str, seed: int = 0) -> Case:
    cfg = dict(CONFIGS[name])
    return make_problem(cfg.pop("n"), cfg.pop("k"), cfg.pop("levels"), seed, name=name, **cfg)


def make_batch(seed: int = 0, count: int = 64, sizes=(256, 512, 1024)):
    """Mixed batch: n ~ U{sizes}, k = 0.625 n, L = min(7, log2 n - 3), own random
    field per problem, 1-4 sources with a multi-source fast-marching phase."""
    rng = _rng(seed)
    out = []
    for p in range(count):
        n = int(rng.choice(sizes))
        out.append(make_problem(n, 0.625 * n, default_levels(n), seed * 1000 + p, medium="grf",
                                nsrc=(1, 4), phase="fmm", name=f"batch{p}"))
    return out
