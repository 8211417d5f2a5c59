"""Seeded synthetic workloads for the space-fractional reaction-diffusion step.

This module only describes problems and draws their initial fields. It holds
none of the method's arithmetic (no operators, transforms, coefficients or
reaction terms), so both the FP64 oracle and the GPU library can take their
inputs from it without sharing any computation.

Grid convention (the paper writes N for the number of intervals per axis,
Section 3.1): a workload gives the number of *unknowns* per axis, n.

* periodic:  N = n,     h = length / n,       x_j = lo + j h,       j = 0..n-1
* Dirichlet: N = n + 1, h = length / (n + 1), x_j = lo + (j + 1) h, j = 0..n-1
* Neumann:   N = n - 1, h = length / (n - 1), x_j = lo + j h,       j = 0..n-1

Arrays are shaped ``[S, (nz,) ny, nx]`` in C order, so x is the fastest axis.
Random draws use ``numpy.random.default_rng(seed)`` in FP64; the u draw comes
before the v draw.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

BCS = ("periodic", "dirichlet", "neumann")
REACTIONS = ("linear", "fhn", "gray_scott", "schnakenberg", "gierer_meinhardt")
SCHEMES = ("p13", "exp")


@dataclass(frozen=True)
class Workload:
    name: str
    bc: str
    shape: tuple            # numpy order, slowest axis first; x is last
    domain: tuple           # (lo, hi), the same on every axis
    alpha: tuple            # fractional order per species
    kappa: tuple            # diffusion coefficient per species
    reaction: str
    params: tuple
    dt: float
    nsteps: int
    seed: int
    init: str               # name of the initial-field recipe
    ckpt_every: int = 0
    scheme: str = "p13"
    dtype: str = "f64"
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def ndim(self) -> int:
        return len(self.shape)

    @property
    def nspecies(self) -> int:
        return len(self.alpha)

    @property
    def npoints(self) -> int:
        return int(np.prod(self.shape))

    def intervals(self, n: int) -> int:
        return {"periodic": n, "dirichlet": n + 1, "neumann": n - 1}[self.bc]

    @property
    def h(self) -> tuple:
        """Mesh width per axis in numpy order (slowest first)."""
        lo, hi = self.domain
        return tuple((hi - lo) / self.intervals(n) for n in self.shape)

    @property
    def h_xyz(self) -> tuple:
        """Mesh width per axis with x first (the library's axis order)."""
        return tuple(reversed(self.h))

    @property
    def n_xyz(self) -> tuple:
        return tuple(reversed(self.shape))

    def coords(self, axis: int) -> np.ndarray:
        """Node coordinates along numpy axis ``axis``."""
        lo, _ = self.domain
        n = self.shape[axis]
        h = self.h[axis]
        j = np.arange(n, dtype=np.float64)
        if self.bc == "dirichlet":
            j = j + 1.0
        return lo + j * h

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _box5(a: np.ndarray) -> np.ndarray:
    """Mean of a point and its 4 axis neighbours in 2D, mirrored at the ends."""
    p = np.pad(a, 1, mode="reflect")
    return (p[1:-1, 1:-1] + p[:-2, 1:-1] + p[2:, 1:-1] + p[1:-1, :-2] + p[1:-1, 2:]) / 5.0


def initial_fields(wl: Workload) -> np.ndarray:
    """FP64 initial fields ``[S, *shape]`` for a workload, drawn from its seed."""
    rng = np.random.default_rng(wl.seed)
    shp = wl.shape
    if wl.init == "fhn_noise":
        u = 0.5 + 0.05 * rng.standard_normal(shp)
        v = 0.1 * rng.uniform(0.0, 1.0, shp)
        u = _box5(u)
        return np.stack([u, v])
    if wl.init == "gs_square":
        grids = np.meshgrid(*[wl.coords(a) for a in range(wl.ndim)], indexing="ij")
        inside = np.ones(shp, dtype=bool)
        for g in grids:
            inside &= np.abs(g) <= 0.1 + 1e-12
        u = np.where(inside, 0.5, 1.0)
        v = np.where(inside, 0.25, 0.0)
        u = u + 0.01 * rng.uniform(-1.0, 1.0, shp)
        v = v + 0.01 * rng.uniform(-1.0, 1.0, shp)
        return np.stack([u, v])
    if wl.init == "schnak_noise":
        u = 0.9 + 0.01 * rng.standard_normal(shp)
        v = 0.9 + 0.01 * rng.standard_normal(shp)
        return np.stack([u, v])
    if wl.init == "gm_noise":
        u = 1.1 + 0.01 * rng.standard_normal(shp)
        v = 1.21 + 0.01 * rng.standard_normal(shp)
        if wl.ndim == 2:
            u, v = _box5(u), _box5(v)
        return np.stack([u, v])
    # Deterministic initial data of the paper's applications (Section 5.2);
    # no random draws.
    if wl.init == "paper_fhn":
        # u = 1 on 0 < x <= 0.125, 0 < y < 0.125; v = 0.1 on 0.125 <= y < 2.5
        y, x = np.meshgrid(wl.coords(0), wl.coords(1), indexing="ij")
        u = np.where((x > 0) & (x <= 0.125) & (y > 0) & (y < 0.125), 1.0, 0.0)
        v = np.where((y >= 0.125) & (y < 2.5), 0.1, 0.0)
        return np.stack([u, v])
    if wl.init == "paper_gm":
        # u = (1 + 0.001 sum_{j=1..20} cos(pi j y / 2)) sech^2(r / (2 eps)) / 2,
        # v = cosh(1 - r) / (3 cosh 1), r = |(x, y)|
        eps = float(wl.extra["eps"])
        y, x = np.meshgrid(wl.coords(0), wl.coords(1), indexing="ij")
        r = np.sqrt(x * x + y * y)
        ripple = sum(np.cos(0.5 * np.pi * j * y) for j in range(1, 21))
        u = 0.5 * (1.0 + 0.001 * ripple) / np.cosh(r / (2.0 * eps)) ** 2
        v = np.cosh(1.0 - r) / (3.0 * np.cosh(1.0))
        return np.stack([u, v])
    if wl.init == "paper_gs":
        # (u, v) = (1/2, 1/4) in the disk (x-1/2)^2 + (y-1/2)^2 <= 0.0016, else (1, 0)
        y, x = np.meshgrid(wl.coords(0), wl.coords(1), indexing="ij")
        inside = (x - 0.5) ** 2 + (y - 0.5) ** 2 <= 0.0016
        return np.stack([np.where(inside, 0.5, 1.0), np.where(inside, 0.25, 0.0)])
    if wl.init == "paper_schnak":
        # u = 1 - exp(-10 (X^2 + Y^2 + Z^2)), v = exp(-10 (X^2 + 2 Y^2 + Z^2)),
        # X = x - l/2 etc. on (0, l)^3
        lo, hi = wl.domain
        c = 0.5 * (lo + hi)
        z, y, x = np.meshgrid(wl.coords(0) - c, wl.coords(1) - c, wl.coords(2) - c,
                              indexing="ij")
        u = 1.0 - np.exp(-10.0 * (x * x + y * y + z * z))
        v = np.exp(-10.0 * (x * x + 2.0 * y * y + z * z))
        return np.stack([u, v])
    if wl.init == "normal":
        base = np.asarray(wl.extra.get("mean", [0.5] * wl.nspecies))
        sd = float(wl.extra.get("sd", 0.1))
        out = []
        for s in range(wl.nspecies):
            out.append(base[s] + sd * rng.standard_normal(shp))
        return np.stack(out)
    raise ValueError(f"unknown init recipe {wl.init!r}")


# The five workloads of the benchmark description. Each is one species pair
# (S = 2). Sizes are unknowns per axis.
C1_FHN = Workload(
    name="fhn2d_neumann_64", bc="neumann", shape=(64, 64), domain=(0.0, 2.5),
    alpha=(1.5, 1.5), kappa=(1e-4, 0.0), reaction="fhn",
    params=(0.1, 0.01, 0.5, 1.0, 0.0), dt=0.1, nsteps=100, seed=0,
    init="fhn_noise", dtype="f64")

C2_GS = Workload(
    name="grayscott2d_periodic_512", bc="periodic", shape=(512, 512), domain=(-1.0, 1.0),
    alpha=(1.7, 1.7), kappa=(2e-5, 1e-5), reaction="gray_scott",
    params=(0.04, 0.06), dt=1.0, nsteps=2000, seed=1, init="gs_square", dtype="f32")

C3_SCHNAK_DIR = Workload(
    name="schnakenberg3d_dirichlet_128", bc="dirichlet", shape=(128, 128, 128),
    domain=(0.0, 1.0), alpha=(1.8, 1.8), kappa=(0.05, 1.0), reaction="schnakenberg",
    params=(1.0, 0.1305, 0.7695), dt=0.01, nsteps=500, seed=2, init="schnak_noise",
    dtype="f32")

C4_GM_ADJ = Workload(
    name="gierermeinhardt2d_neumann_256_adjoint", bc="neumann", shape=(256, 256),
    domain=(0.0, 2.0), alpha=(1.6, 1.6), kappa=(1e-3, 0.05), reaction="gierer_meinhardt",
    params=(0.1, 1.0, 1.0, 1.0, 1.0), dt=0.05, nsteps=200, seed=3, init="gm_noise",
    ckpt_every=20, dtype="f32",
    extra={"target": {"alpha": (1.65, 1.65), "kappa": (1.1e-3, 0.05),
                      "params": (0.11, 1.0, 1.0, 1.0, 1.0)}})

C5_SCHNAK_NEU = Workload(
    name="schnakenberg3d_neumann_256", bc="neumann", shape=(256, 256, 256),
    domain=(0.0, 1.0), alpha=(1.5, 1.5), kappa=(0.05, 1.0), reaction="schnakenberg",
    params=(1.0, 0.1305, 0.7695), dt=0.005, nsteps=1000, seed=4, init="schnak_noise",
    ckpt_every=32, dtype="f32",
    extra={"alphas": (1.2, 1.5, 1.9),
           "target": {"alpha_shift": 0.05, "kappa_v_scale": 1.1}})

ALL = (C1_FHN, C2_GS, C3_SCHNAK_DIR, C4_GM_ADJ, C5_SCHNAK_NEU)

# The parameter sets, grids, steps and initial data of the paper's own
# applications (Section 5.2). N is the paper's number of intervals; the
# unknowns per axis follow the boundary condition (periodic: n = N). Where the
# paper lists several orders or constants, the first listed is the preset and
# the rest are in extra["sweep"].
PAPER_FHN = Workload(
    name="paper_fhn2d_periodic_256", bc="periodic", shape=(256, 256), domain=(0.0, 2.5),
    alpha=(2.0, 2.0), kappa=(1e-4, 0.0), reaction="fhn", params=(0.1, 0.01, 0.5, 1.0, 0.0),
    dt=1.0, nsteps=2000, seed=0, init="paper_fhn", dtype="f64",
    extra={"sweep": {"alpha": (2.0, 1.7, 1.5), "bc": ("periodic", "neumann")}})

# f_u = u^2/v - u, f_v = u^2/(eps mu) - v/mu as the Gierer-Meinhardt family with
# (rho, mu_u, sigma_u, sigma_v, mu_v) = (0, 1, 1, 1/(eps mu), 1/mu);
# kappa_u = eps^2, kappa_v = K/mu; orders (alpha, beta) per species.
_GM_EPS, _GM_MU, _GM_K = 0.04, 0.1, 0.0162
PAPER_GM = Workload(
    name="paper_gm2d_neumann_64", bc="neumann", shape=(65, 65), domain=(-1.0, 1.0),
    alpha=(2.0, 1.9), kappa=(_GM_EPS ** 2, _GM_K / _GM_MU), reaction="gierer_meinhardt",
    params=(0.0, 1.0, 1.0, 1.0 / (_GM_EPS * _GM_MU), 1.0 / _GM_MU), dt=0.1, nsteps=10000,
    seed=0, init="paper_gm", dtype="f64",
    extra={"eps": _GM_EPS, "sweep": {"beta": (2.0, 1.9, 1.8), "K": (0.0162, 0.0128)}})

PAPER_GS = Workload(
    name="paper_gs2d_periodic_265", bc="periodic", shape=(265, 265), domain=(0.0, 1.0),
    alpha=(2.0, 2.0), kappa=(2e-5, 1e-5), reaction="gray_scott", params=(0.03, 0.055),
    dt=1.0, nsteps=8000, seed=0, init="paper_gs", dtype="f64",
    extra={"sweep": {"alpha": (2.0, 1.7, 1.5), "K": (0.055, 0.061, 0.063)}})

PAPER_SCHNAK = Workload(
    name="paper_schnakenberg3d_periodic_32", bc="periodic", shape=(32, 32, 32),
    domain=(0.0, 10.0), alpha=(2.0, 2.0), kappa=(1.0, 10.0), reaction="schnakenberg",
    params=(1.0, 0.1, 0.9), dt=1.0, nsteps=200, seed=0, init="paper_schnak", dtype="f64",
    extra={"sweep": {"alpha": (2.0, 1.5), "l": (10.0, 20.0, 40.0)}})

PAPER = (PAPER_FHN, PAPER_GM, PAPER_GS, PAPER_SCHNAK)


def small(wl: Workload, shape: tuple, nsteps: int | None = None, **kw) -> Workload:
    """The same problem on a smaller grid (tests)."""
    return wl.replace(shape=tuple(shape), nsteps=wl.nsteps if nsteps is None else nsteps, **kw)
