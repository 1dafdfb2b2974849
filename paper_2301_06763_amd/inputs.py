"""Seeded synthetic density fields on nested meshes.

This module only builds inputs: it samples analytic density profiles at
cell centres and draws seeded random parameters.  It holds none of the
potential method's arithmetic, so both the CPU oracle's tests and the GPU
path can take their inputs from it.

Geometry (Sect. 2, Fig. 1 of the paper): L concentric levels of N^3 cells,
coarsest box side B (default 1.0), level l (0-based) has cell size
h_l = B / (N 2^l); cell centres at (i - N/2 + 1/2) h_l.

Workloads (all G = 1, B = 1, seeds fixed):

* ``plummer32``: N=32, L=3, one Plummer sphere (M=1, a=0.05) at the origin.
* ``random12``: N=12, L=1, uniform [0,1) random density (seed 12), the
  single-level brute-force check.
* ``ellipsoid64``: N=64, L=5, homogeneous ellipsoid, semi-axes
  (0.08, 0.05, 0.03), rho=1, times (1 + 0.01 xi), xi ~ N(0,1) per cell and
  level (seed 2 + l).
* ``binary128``: N=128, L=8, Plummer spheres of mass 1 and 0.5, scale 2 h_8,
  centres (+-3 h_8, 0, 0) (a tight, dipole-dominated pair on coarse levels).
* ``clumps256``: N=256, L=6, 64 Plummer clumps (seed 4): masses log-uniform
  in [1e-3, 1], scale radii log-uniform in [2 h_6, 2 h_1], centre distances
  log-uniform in [h_6, 0.25] with isotropic directions.
* ``serving`` requests: N in {32, 64, 128}, L in {2..8}, 1-4 components,
  each a Plummer sphere or a homogeneous ellipsoid (seed 5 + request id).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


@dataclass
class Workload:
    name: str
    N: int
    L: int
    h0: float
    G: float = 1.0
    rho: torch.Tensor | None = None          # [L, N, N, N] float64, [z][y][x]
    components: list = field(default_factory=list)  # analytic description

    @property
    def spacings(self):
        return [self.h0 / 2 ** l for l in range(self.L)]


def centres_1d(N: int, h: float, device=None) -> torch.Tensor:
    return (torch.arange(N, dtype=torch.float64, device=device) - (N / 2 - 0.5)) * h


def _grid(N, h, centre, device):
    c = centres_1d(N, h, device)
    dx = (c - centre[0])
    dy = (c - centre[1])
    dz = (c - centre[2])
    return dx, dy, dz


def _r2(N, h, centre, device):
    dx, dy, dz = _grid(N, h, centre, device)
    return (dz * dz)[:, None, None] + (dy * dy)[None, :, None] + (dx * dx)[None, None, :]


def plummer_level(N, h, M, a, centre=(0.0, 0.0, 0.0), device=None) -> torch.Tensor:
    """Plummer density 3M/(4 pi a^3) (1 + r^2/a^2)^(-5/2) at cell centres."""
    q = 1.0 + _r2(N, h, centre, device) / (a * a)
    return (3.0 * M / (4.0 * math.pi * a ** 3)) / (q * q * torch.sqrt(q))


def ellipsoid_level(N, h, axes, rho=1.0, centre=(0.0, 0.0, 0.0), device=None) -> torch.Tensor:
    """Homogeneous ellipsoid (semi-axes along x, y, z) sampled at cell centres."""
    dx, dy, dz = _grid(N, h, centre, device)
    q = ((dz / axes[2]) ** 2)[:, None, None] + ((dy / axes[1]) ** 2)[None, :, None] \
        + ((dx / axes[0]) ** 2)[None, None, :]
    return torch.where(q <= 1.0, torch.full_like(q, rho), torch.zeros_like(q))


def polytrope2_level(N, h, rho0, R, centre=(0.0, 0.0, 0.0), device=None) -> torch.Tensor:
    """rho0 (1 - r^2/R^2)^2 inside R (zero outside) at cell centres."""
    u = 1.0 - _r2(N, h, centre, device) / (R * R)
    return torch.where(u > 0, rho0 * u * u, torch.zeros_like(u))


def _levels(N, L, h0, fn, device):
    return torch.stack([fn(l, h0 / 2 ** l) for l in range(L)])


def plummer32(device=None) -> Workload:
    N, L, B = 32, 3, 1.0
    h0 = B / N
    rho = _levels(N, L, h0, lambda l, h: plummer_level(N, h, 1.0, 0.05, device=device), device)
    return Workload("plummer32", N, L, h0, rho=rho,
                    components=[("plummer", dict(M=1.0, a=0.05, centre=(0.0, 0.0, 0.0)))])


def random12(device=None) -> Workload:
    N = 12
    rng = np.random.default_rng(12)
    rho = torch.from_numpy(rng.random((1, N, N, N))).to(device)
    return Workload("random12", N, 1, 1.0 / N, rho=rho)


def ellipsoid64(device=None, noise=0.01) -> Workload:
    N, L, B = 64, 5, 1.0
    h0 = B / N
    axes = (0.08, 0.05, 0.03)

    def lev(l, h):
        base = ellipsoid_level(N, h, axes, 1.0, device=device)
        xi = np.random.default_rng(2 + l).standard_normal((N, N, N))
        return base * (1.0 + noise * torch.from_numpy(xi).to(base.device))

    return Workload("ellipsoid64", N, L, h0, rho=_levels(N, L, h0, lev, device),
                    components=[("ellipsoid", dict(a=axes, rho=1.0, centre=(0.0, 0.0, 0.0)))])


def binary128(device=None) -> Workload:
    N, L, B = 128, 8, 1.0
    h0 = B / N
    hL = h0 / 2 ** (L - 1)
    comps = [("plummer", dict(M=1.0, a=2 * hL, centre=(-3 * hL, 0.0, 0.0))),
             ("plummer", dict(M=0.5, a=2 * hL, centre=(3 * hL, 0.0, 0.0)))]

    def lev(l, h):
        return sum(plummer_level(N, h, c["M"], c["a"], c["centre"], device) for _, c in comps)

    return Workload("binary128", N, L, h0, rho=_levels(N, L, h0, lev, device), components=comps)


def clumps256(device=None, N=256, L=6, nclumps=64, seed=4) -> Workload:
    B = 1.0
    h0 = B / N
    hL = h0 / 2 ** (L - 1)
    rng = np.random.default_rng(seed)
    comps = []
    for _ in range(nclumps):
        M = math.exp(rng.uniform(math.log(1e-3), math.log(1.0)))
        a = math.exp(rng.uniform(math.log(2 * hL), math.log(2 * h0)))
        d = math.exp(rng.uniform(math.log(hL), math.log(0.25)))
        v = rng.standard_normal(3)
        v = v / np.linalg.norm(v)
        comps.append(("plummer", dict(M=M, a=a, centre=tuple(float(t) for t in d * v))))

    def lev(l, h):
        acc = torch.zeros((N, N, N), dtype=torch.float64, device=device)
        for _, c in comps:
            acc += plummer_level(N, h, c["M"], c["a"], c["centre"], device)
        return acc

    return Workload("clumps256", N, L, h0, rho=_levels(N, L, h0, lev, device), components=comps)


def serving_request(rid: int, device=None, Ns=(32, 64, 128), Lrange=(2, 8)) -> Workload:
    """One request of the serving stream (seed 5 + rid)."""
    rng = np.random.default_rng(5 + rid)
    N = int(rng.choice(Ns))
    L = int(rng.integers(Lrange[0], Lrange[1] + 1))
    B = 1.0
    h0 = B / N
    hL = h0 / 2 ** (L - 1)
    BL = N * hL
    comps = []
    for _ in range(int(rng.integers(1, 5))):
        centre = tuple(float(t) for t in rng.uniform(-BL / 4, BL / 4, size=3))
        if rng.random() < 0.5:
            M = math.exp(rng.uniform(math.log(0.1), math.log(1.0)))
            a = math.exp(rng.uniform(math.log(2 * hL), math.log(0.1)))
            comps.append(("plummer", dict(M=M, a=a, centre=centre)))
        else:
            a1 = math.exp(rng.uniform(math.log(4 * hL), math.log(0.1)))
            a2 = a1 * rng.uniform(0.5, 1.0)
            a3 = a2 * rng.uniform(0.5, 1.0)
            comps.append(("ellipsoid", dict(a=(a1, a2, a3), rho=1.0, centre=centre)))

    def lev(l, h):
        acc = torch.zeros((N, N, N), dtype=torch.float64, device=device)
        for kind, c in comps:
            if kind == "plummer":
                acc += plummer_level(N, h, c["M"], c["a"], c["centre"], device)
            else:
                acc += ellipsoid_level(N, h, c["a"], c["rho"], c["centre"], device)
        return acc

    return Workload(f"serving{rid}", N, L, h0, rho=_levels(N, L, h0, lev, device), components=comps)


def random_levels(N, L, seed, device=None, h0=None) -> Workload:
    """Uniform [0,1) random densities on every level (seed, seed+1, ...)."""
    h0 = 1.0 / N if h0 is None else h0
    rho = torch.stack([torch.from_numpy(np.random.default_rng(seed + l).random((N, N, N)))
                       for l in range(L)]).to(device)
    return Workload(f"random{N}x{L}", N, L, h0, rho=rho)


WORKLOADS = {
    "plummer32": plummer32,
    "random12": random12,
    "ellipsoid64": ellipsoid64,
    "binary128": binary128,
    "clumps256": clumps256,
}
