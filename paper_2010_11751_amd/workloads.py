"""Seeded synthetic inputs shared by the GPU path's tests and benchmark and by
the oracle's tests.

This module holds none of the method's arithmetic: it produces sizes,
relaxation frequencies, velocity fields and random arrays, which both sides
then consume through their own code.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ENSEMBLE_SEED = 2010_11751


def omega_from_nu(nu: float) -> float:
    """Relaxation frequency for a kinematic viscosity in lattice units
    (nu = (1/omega - 1/2) c_s^2 with c_s^2 = 1/3, Sec. 2.6)."""
    return 1.0 / (3.0 * nu + 0.5)


@dataclass(frozen=True)
class Cavity:
    """Lid-driven cubic cavity of n^3 cells, wall layer included; the lid is
    the top z layer moving along +x; nu = u_lid * n / Re."""
    n: int
    re: float
    u_lid: float

    @property
    def nu(self) -> float:
        return self.u_lid * self.n / self.re

    @property
    def omega(self) -> float:
        return omega_from_nu(self.nu)

    @property
    def cells(self) -> int:
        return self.n ** 3

    @property
    def fluid_cells(self) -> int:
        return (self.n - 2) ** 3


# Workloads: the small correctness cavity, the 256^3 measurement cavity, the
# 512^3 D3Q27 cavity and the 256^3 Taylor-Green box.
CAVITY_SMALL = Cavity(32, 100.0, 0.02)
CAVITY_256 = Cavity(256, 1000.0, 0.05)
CAVITY_512 = Cavity(512, 5000.0, 0.05)
TGV_N, TGV_U0, TGV_NU, TGV_STEPS = 256, 0.04, 0.01, 2000


def taylor_green_velocity(nx: int, ny: int, nz: int, u0: float, dims: int = 3) -> np.ndarray:
    """Node-centred Taylor-Green field u[3][Ntot] at cell (x, y, z) with linear
    index (x*ny + y)*nz + z and wave numbers k_a = 2 pi / n_a.
    dims=3: u0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0);
    dims=2: the z-invariant field u0 (sin kx cos ky, -cos kx sin ky, 0)."""
    x = np.arange(nx, dtype=np.float64)[:, None, None] * (2.0 * math.pi / nx)
    y = np.arange(ny, dtype=np.float64)[None, :, None] * (2.0 * math.pi / ny)
    z = np.arange(nz, dtype=np.float64)[None, None, :] * (2.0 * math.pi / nz)
    cz = np.cos(z) if dims == 3 else np.ones_like(z)
    shape = (nx, ny, nz)
    ux = np.broadcast_to(u0 * np.sin(x) * np.cos(y) * cz, shape)
    uy = np.broadcast_to(-u0 * np.cos(x) * np.sin(y) * cz, shape)
    uz = np.zeros(shape)
    return np.stack([a.ravel() for a in (ux, uy, uz)])


def random_populations(seed: int, q: int, ncells: int, lo: float = 0.01, hi: float = 0.1) -> np.ndarray:
    """Positive random populations f[ncells][q], uniform in [lo, hi)."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(ncells, q))


def random_velocity(seed: int, n: int, amp: float = 0.05) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-amp, amp, size=(n, 3))


def random_density(seed: int, n: int, lo: float = 0.9, hi: float = 1.1) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def shuffled_order(seed: int, n: int) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n).astype(np.int64)


@dataclass(frozen=True)
class EnsembleMember:
    n: int
    re: float
    u_lid: float

    @property
    def nu(self) -> float:
        return self.u_lid * self.n / self.re

    @property
    def omega(self) -> float:
        return omega_from_nu(self.nu)


def ensemble(count: int = 512, seed: int = ENSEMBLE_SEED, lmin: int = 16, lmax: int = 64,
             re_min: float = 100.0, re_max: float = 1000.0, u_lid: float = 0.03):
    """Independent cubic cavities: edge ~ U{lmin..lmax} (wall layer included),
    Re ~ U[re_min, re_max], fixed lid speed."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lmin, lmax + 1, size=count)
    res = rng.uniform(re_min, re_max, size=count)
    return [EnsembleMember(int(n), float(r), u_lid) for n, r in zip(sizes, res)]
