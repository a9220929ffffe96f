"""Python access to the plain FP64 CPU oracle (``oracle/lbm_oracle.c``).

TEST INFRASTRUCTURE: only ``tests/``, the smoke check of ``__graft_entry__``
and the CPU-baseline leg of ``bench.py`` use this package. It shares no code
with the GPU path (``paper_2010_11751_amd``) and never imports it.

Arrays are numpy FP64, populations in the layout named by the configuration
(SoA ``pop[k][Ntot]`` or AoS ``pop[Ntot][Q]``), flags uint8 with FLUID=0,
WALL=1, LID=2, linear cell index ``i = (x*ny + y)*nz + z`` (Sec. 2.5).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

FLUID, WALL, LID, PRESSURE = 0, 1, 2, 3
CAVITY, PERIODIC, CHANNEL = 0, 1, 2
BGK, TRT, REG, RR = 0, 1, 2, 3
NW4, RM, HM, CM, CHM, K = 4, 5, 6, 7, 8, 9
SOA, AOS = 0, 1
MODELS = {"bgk": BGK, "trt": TRT, "reg": REG, "rr": RR,
          "nw4": NW4, "rm": RM, "hm": HM, "cm": CM, "chm": CHM, "k": K}
MOMENT_SPACE = ("nw4", "rm", "hm", "cm", "chm", "k")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-fopenmp", "-shared", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("geometry", ctypes.c_int32), ("model", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("omega", ctypes.c_double), ("trt_lambda", ctypes.c_double),
                ("omega_bulk", ctypes.c_double), ("omega3", ctypes.c_double),
                ("omega4", ctypes.c_double), ("u_lid", ctypes.c_double * 3),
                ("force", ctypes.c_double * 3)]


@dataclass
class Config:
    q: int = 19
    nx: int = 8
    ny: int = 8
    nz: int = 8
    geometry: int = CAVITY
    model: int = BGK
    layout: int = SOA
    omega: float = 1.0
    trt_lambda: float = 0.25
    omega_bulk: float | None = None
    omega3: float = 1.0
    omega4: float = 1.0
    u_lid: tuple = (0.0, 0.0, 0.0)
    force: tuple = (0.0, 0.0, 0.0)

    @property
    def ntot(self) -> int:
        return self.nx * self.ny * self.nz

    def c_struct(self) -> _Cfg:
        if self.model == K and self.q != 19:
            raise ValueError("the cumulant model is defined on D3Q19 only")
        ob = self.omega if self.omega_bulk is None else self.omega_bulk
        return _Cfg(self.q, self.nx, self.ny, self.nz, self.geometry, self.model, self.layout, 0,
                    self.omega, self.trt_lambda, ob, self.omega3, self.omega4,
                    (ctypes.c_double * 3)(*self.u_lid),
                    (ctypes.c_double * 3)(*self.force))


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        cfgp = ctypes.POINTER(_Cfg)
        L.oracle_lattice.argtypes = [ctypes.c_int, P, P, P]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_neighbour_index.argtypes = [cfgp, ctypes.c_int64, ctypes.c_int]
        L.oracle_neighbour_index.restype = ctypes.c_int64
        L.oracle_flags.argtypes = [cfgp, P]
        L.oracle_flags.restype = None
        L.oracle_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P]
        L.oracle_equilibrium.restype = None
        L.oracle_collide.argtypes = [cfgp, P, P]
        L.oracle_init_state.argtypes = [cfgp, P, P, P, P]
        L.oracle_init_state_ex.argtypes = [cfgp, P, P, P, P, P, P]
        L.oracle_reference_step.argtypes = [cfgp, P, P, P]
        L.oracle_reference_step_ex.argtypes = [cfgp, P, P, P, P]
        L.oracle_pull_step_ex.argtypes = [cfgp, P, P, P, P, P]
        L.oracle_aa_natural_ex.argtypes = [cfgp, P, P, P, P]
        L.oracle_reference_cells.argtypes = [cfgp, P, P, P, ctypes.c_int64, P]
        L.oracle_2pop_step.argtypes = [cfgp, P, P, P, P]
        L.oracle_pull_step.argtypes = [cfgp, P, P, P, P]
        L.oracle_swap_step.argtypes = [cfgp, P, P, P]
        L.oracle_aa_step.argtypes = [cfgp, P, P, ctypes.c_int, P]
        L.oracle_aa_natural.argtypes = [cfgp, P, P, P]
        L.oracle_macroscopic.argtypes = [cfgp, P, P, P, P]
        L.oracle_invariants.argtypes = [cfgp, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle call failed with {rc}")


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (for timing)."""
    lib().oracle_set_threads(int(n))


def lattice(q: int):
    """(c[q][3] int, t[q], opp[q]) in the oracle's velocity order."""
    c = np.zeros((q, 3), np.int32)
    t = np.zeros(q)
    opp = np.zeros(q, np.int32)
    _check(lib().oracle_lattice(q, _p(c), _p(t), _p(opp)))
    return c, t, opp


def flags(cfg: Config) -> np.ndarray:
    fl = np.zeros(cfg.ntot, np.uint8)
    lib().oracle_flags(ctypes.byref(cfg.c_struct()), _p(fl))
    return fl


def neighbour_index(cfg: Config, i: int, k: int) -> int:
    return int(lib().oracle_neighbour_index(ctypes.byref(cfg.c_struct()), i, k))


def equilibrium(q: int, rho: float, u, model: int = BGK) -> np.ndarray:
    E = np.zeros(q)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    lib().oracle_equilibrium(q, model, float(rho), _p(uu), _p(E))
    return E


def collide(cfg: Config, f) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(cfg.q)
    _check(lib().oracle_collide(ctypes.byref(cfg.c_struct()), _p(f), _p(out)))
    return out


def init_state(cfg: Config, fl: np.ndarray, rho=None, u=None, wall_u=None, wall_rho=None) -> np.ndarray:
    """Wall terms in wall cells (from the lid velocity, or from per-cell
    wall_u[3][Ntot] and wall_rho[Ntot] when given), E(rho, u) in fluid cells;
    u is u[3][Ntot]."""
    pop = np.zeros(cfg.ntot * cfg.q)

    def arr(a):
        return None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()
    r, v, wu, wr = arr(rho), arr(u), arr(wall_u), arr(wall_rho)
    _check(lib().oracle_init_state_ex(ctypes.byref(cfg.c_struct()), _p(fl), _p(r), _p(v), _p(wu), _p(wr),
                                      _p(pop)))
    return pop


def _q(qlink, cfg):
    if qlink is None:
        return None
    q = np.ascontiguousarray(qlink, dtype=np.float64).ravel()
    if q.size != cfg.q * cfg.ntot or not np.all((q > 0.0) & (q <= 1.0)):
        raise ValueError("qlink: q[k][Ntot] wall distances in (0, 1]")
    return q


def reference_step(cfg: Config, fl, f, qlink=None) -> np.ndarray:
    """One reference step; qlink[k][Ntot] (optional) gives each fluid cell's
    wall distance along -c_k for the curved-wall rule (1/2: half-way)."""
    new = np.empty_like(f)
    _check(lib().oracle_reference_step_ex(ctypes.byref(cfg.c_struct()), _p(fl), _p(f), _p(_q(qlink, cfg)), _p(new)))
    return new


def reference_cells(cfg: Config, fl, f, cells) -> np.ndarray:
    """Reference-step populations of the listed cells only: out[j][k]."""
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.zeros((cells.size, cfg.q))
    _check(lib().oracle_reference_cells(ctypes.byref(cfg.c_struct()), _p(fl), _p(f), _p(cells),
                                        cells.size, _p(out)))
    return out


def twopop_step(cfg: Config, fl, pop, out, order=None) -> None:
    _check(lib().oracle_2pop_step(ctypes.byref(cfg.c_struct()), _p(fl), _p(pop), _p(out), _p(order)))


def pull_step(cfg: Config, fl, pop, out, order=None, qlink=None) -> None:
    _check(lib().oracle_pull_step_ex(ctypes.byref(cfg.c_struct()), _p(fl), _p(pop), _p(_q(qlink, cfg)), _p(out),
                                     _p(order)))


def swap_step(cfg: Config, fl, pop, order=None) -> None:
    _check(lib().oracle_swap_step(ctypes.byref(cfg.c_struct()), _p(fl), _p(pop), _p(order)))


def aa_step(cfg: Config, fl, pop, odd: bool, order=None) -> None:
    _check(lib().oracle_aa_step(ctypes.byref(cfg.c_struct()), _p(fl), _p(pop), int(bool(odd)), _p(order)))


def aa_natural(cfg: Config, fl, pop, qlink=None) -> np.ndarray:
    f = np.empty_like(pop)
    _check(lib().oracle_aa_natural_ex(ctypes.byref(cfg.c_struct()), _p(fl), _p(pop), _p(_q(qlink, cfg)), _p(f)))
    return f


def macroscopic(cfg: Config, fl, f):
    rho = np.zeros(cfg.ntot)
    u = np.zeros(3 * cfg.ntot)
    _check(lib().oracle_macroscopic(ctypes.byref(cfg.c_struct()), _p(fl), _p(f), _p(rho), _p(u)))
    return rho, u.reshape(3, cfg.ntot)


def invariants(cfg: Config, fl, f):
    m = ctypes.c_double()
    e = ctypes.c_double()
    _check(lib().oracle_invariants(ctypes.byref(cfg.c_struct()), _p(fl), _p(f),
                                   ctypes.byref(m), ctypes.byref(e)))
    return m.value, e.value


def to_soa(cfg: Config, pop) -> np.ndarray:
    """Populations of any layout as the natural f[k][Ntot] array."""
    if cfg.layout == SOA:
        return pop.reshape(cfg.q, cfg.ntot).copy()
    return pop.reshape(cfg.ntot, cfg.q).T.copy()


class Simulation:
    """Runs the oracle with one of the three schemes of Table 1, or the
    two-population scheme in pull form ("2pop_pull": an AA even step first,
    then pull steps between two arrays), and reads back the natural
    pre-collision populations f[k][Ntot] at whole steps."""

    def __init__(self, cfg: Config, scheme: str = "2pop", rho=None, u=None, order=None, cell_types=None,
                 wall_u=None, wall_rho=None, qlink=None):
        """cell_types (uint8 FLUID / WALL / LID / PRESSURE per cell) replaces
        the geometry's flags; wall_u[3][Ntot] and wall_rho[Ntot] give each wall
        cell its own velocity and density; qlink[k][Ntot] the curved-wall
        distances (reference step and 2Pop pull only)."""
        if qlink is not None and scheme not in ("ref", "2pop_pull"):
            raise ValueError("curved walls: reference step and 2Pop pull only")
        self.cfg, self.scheme, self.order, self.qlink = cfg, scheme, order, qlink
        self.flags = flags(cfg) if cell_types is None else np.ascontiguousarray(cell_types, dtype=np.uint8).copy()
        self.pop = init_state(cfg, self.flags, rho, u, wall_u, wall_rho)
        self.out = self.pop.copy() if scheme in ("2pop", "2pop_pull") else None
        self.t = 0

    def step(self, n: int = 1) -> None:
        for _ in range(n):
            if self.scheme == "ref":
                self.pop = reference_step(self.cfg, self.flags, self.pop, self.qlink)
            elif self.scheme == "2pop":
                twopop_step(self.cfg, self.flags, self.pop, self.out, self.order)
                self.pop, self.out = self.out, self.pop
            elif self.scheme == "swap":
                swap_step(self.cfg, self.flags, self.pop, self.order)
            elif self.scheme == "aa":
                aa_step(self.cfg, self.flags, self.pop, self.t % 2 == 1, self.order)
            elif self.scheme == "2pop_pull":
                if self.t == 0:
                    aa_step(self.cfg, self.flags, self.pop, False, self.order)
                else:
                    pull_step(self.cfg, self.flags, self.pop, self.out, self.order, self.qlink)
                    self.pop, self.out = self.out, self.pop
            else:
                raise ValueError(self.scheme)
            self.t += 1

    def natural(self) -> np.ndarray:
        """Pre-collision populations in the configured layout."""
        if (self.scheme == "aa" and self.t % 2 == 1) or (self.scheme == "2pop_pull" and self.t > 0):
            return aa_natural(self.cfg, self.flags, self.pop, self.qlink)
        return self.pop.copy()

    def populations(self) -> np.ndarray:
        """f[k][Ntot] (natural SoA)."""
        return to_soa(self.cfg, self.natural())

    def macroscopic(self):
        return macroscopic(self.cfg, self.flags, self.natural())

    def invariants(self):
        return invariants(self.cfg, self.flags, self.natural())
