"""GPU parity of caller-defined geometry (lbm_set_geometry): random obstacle
cells and a solid block inside cavity, periodic and channel boxes, every wall
cell with its own wall velocity and density in the momentum-exchange term
(Eqs. momentum-exchange, storage2). FP64 max |df| <= 1e-12 against the
oracle after 22 steps; flags bit-exact; invalid geometries rejected."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2010_11751_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
GEOM = {"cavity": O.CAVITY, "periodic": O.PERIODIC, "channel": O.CHANNEL}


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def max_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def geometry(cfg, seed, fraction=0.12):
    """The box's own walls, random obstacle cells, one solid block (flat
    faces next to the fluid), random wall velocities and densities."""
    fl = O.flags(cfg).reshape(cfg.nx, cfg.ny, cfg.nz).copy()
    rng = np.random.default_rng(seed)
    fl[(rng.random(fl.shape) < fraction) & (fl == O.FLUID)] = O.WALL
    fl[3:6, 2:5, 3:6] = O.WALL
    types = fl.ravel()
    wu = W.random_velocity(seed + 1, cfg.ntot, amp=0.03).T.copy()
    wu[:, types == O.FLUID] = 0.0
    wr = W.random_density(seed + 2, cfg.ntot)
    return types, wu, wr


def cases():
    out = []
    for q in (19, 27):
        for geo in ("cavity", "periodic", "channel"):
            for scheme in ("2pop", "swap", "aa", "2pop_pull"):
                out.append((q, geo, scheme, "soa"))
        out.append((q, "cavity", "aa", "aos"))
    return out


@pytest.mark.parametrize("q,geo,scheme,layout", cases())
def test_custom_geometry_matches_oracle(lbm, q, geo, scheme, layout):
    nx, ny, nz = 13, 11, 12
    print(f"case: geometry q={q} {geo} {scheme} {layout}", flush=True)
    cfg = O.Config(q=q, nx=nx, ny=ny, nz=nz, geometry=GEOM[geo], model=O.TRT, omega=1.75,
                   u_lid=(0.04, 0.0, 0.0))
    types, wu, wr = geometry(cfg, 21 + q)
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision="trt", omega=1.75, u_lid=0.04, layout=layout,
                      geometry=geo)
    sim.set_geometry(torch.from_numpy(types), torch.from_numpy(wu), torch.from_numpy(wr))
    assert np.array_equal(sim.flags().cpu().numpy(), types)
    assert sim.info().fluid_cells == int((types == O.FLUID).sum())
    ref = O.Simulation(cfg, "ref", cell_types=types, wall_u=wu, wall_rho=wr)
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= 1e-15
    for n in (21, 1):
        sim.step(n)
        ref.step(n)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, n


@pytest.mark.parametrize("scheme", ("2pop", "aa", "2pop_pull"))
def test_custom_geometry_graph_replay_and_reinit(lbm, scheme):
    """Small lattice: steps replay from a captured graph; a later
    lbm_init_equilibrium keeps the per-cell wall terms."""
    nx, ny, nz = 12, 10, 11
    cfg = O.Config(q=19, nx=nx, ny=ny, nz=nz, geometry=O.PERIODIC, model=O.BGK, omega=1.8)
    types, wu, wr = geometry(cfg, 31)
    sim = lbm.Lattice(19, nx, ny, nz, scheme=scheme, collision="bgk", omega=1.8, geometry="periodic")
    sim.set_geometry(torch.from_numpy(types), torch.from_numpy(wu), torch.from_numpy(wr))
    sim.step(130)
    u0 = W.random_velocity(33, cfg.ntot, amp=0.03).T.copy()
    u0[:, types != O.FLUID] = 0.0
    sim.init_equilibrium(None, torch.from_numpy(u0))
    ref = O.Simulation(cfg, "ref", u=u0, cell_types=types, wall_u=wu, wall_rho=wr)
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= 1e-15
    sim.step(129)
    ref.step(129)
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL


def test_invalid_geometries_are_rejected(lbm):
    n = 8
    sim = lbm.Lattice(19, n, scheme="aa", collision="bgk", omega=1.5, u_lid=0.03)
    before = sim.populations().cpu()
    base = O.flags(O.Config(q=19, nx=n, ny=n, nz=n))
    bad_face = base.copy()
    bad_face[0] = O.FLUID                      # fluid on the x = 0 face of a cavity
    bad_type = base.copy()
    bad_type[100] = 7
    fast = np.zeros((3, n ** 3))
    fast[0, base != O.FLUID] = 0.5             # |u_w| >= 0.4
    for types, wu in ((bad_face, None), (bad_type, None), (base, fast)):
        with pytest.raises(lbm.LBMError) as e:
            sim.set_geometry(torch.from_numpy(types), None if wu is None else torch.from_numpy(wu))
        assert "geometry" in str(e.value)
    assert torch.equal(sim.populations().cpu(), before)
    assert sim.info().fluid_cells == (n - 2) ** 3


def relative_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def test_custom_geometry_shifted_storage(lbm):
    """FP32- and FP16-shifted storage on an obstacle geometry: velocity
    relative L2 against FP64 after 300 steps."""
    n = 24
    cfg = O.Config(q=19, nx=n, ny=n, nz=n, model=O.TRT, omega=1.8, u_lid=(0.05, 0.0, 0.0))
    types, wu, wr = geometry(cfg, 41, fraction=0.05)
    us = {}
    for dtype in ("f64", "f32", "f16"):
        sim = lbm.Lattice(19, n, scheme="aa", collision="trt", omega=1.8, u_lid=0.05, dtype=dtype)
        sim.set_geometry(torch.from_numpy(types), torch.from_numpy(wu), torch.from_numpy(wr))
        sim.step(300)
        us[dtype] = sim.macroscopic()[1].cpu().numpy()
    e32, e16 = relative_l2(us["f32"], us["f64"]), relative_l2(us["f16"], us["f64"])
    print(f"obstacles: velocity rel L2 f32 {e32:.3e} f16 {e16:.3e}", flush=True)
    assert e32 <= 1e-5
    assert e16 <= 1e-3
