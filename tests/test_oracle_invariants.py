"""Pins of two oracle outputs that the GPU tests use as checkers:

- the global invariants (mass sum_fluid sum_k f_k and kinetic energy
  1/2 sum_fluid rho |u|^2), against the density and velocity fields the
  state was built from: an equilibrium E(rho, u) carries exactly the density
  rho and momentum rho u (Sec. 2.6, closed-form moments of E), so the
  invariants of a freshly built state are fixed by its input fields;
- the per-cell reference step (the sampled checker of the full-size GPU
  tests), against the whole-lattice reference step of Sec. 2.1, cell by cell
  and bit for bit.
"""
import numpy as np
import pytest

from paper_2010_11751_amd import workloads as W


def fluid_count(orc, cfg):
    return int((orc.flags(cfg) == orc.FLUID).sum())


@pytest.mark.parametrize("q", (19, 27))
@pytest.mark.parametrize("model", ("bgk", "rr", "nw4"))
@pytest.mark.parametrize("geom", ("periodic", "cavity"))
def test_invariants_of_a_uniform_flow(orc, q, model, geom):
    """Uniform (rho0, u0) with rho0 != 1: mass = rho0 N and
    KE = 1/2 rho0 |u0|^2 N over the N fluid cells. A dropped 1/2, or
    rho |u|^2 written as |rho u|^2, misses by a factor 2 or rho0."""
    gid = {"periodic": orc.PERIODIC, "cavity": orc.CAVITY}[geom]
    cfg = orc.Config(q=q, nx=6, ny=5, nz=7, geometry=gid, model=orc.MODELS[model], omega=1.3,
                     u_lid=(0.03, 0.0, 0.0))
    rho0, u0 = 1.3, np.array([0.04, -0.03, 0.02])
    rho = np.full(cfg.ntot, rho0)
    u = np.repeat(u0[:, None], cfg.ntot, axis=1)
    sim = orc.Simulation(cfg, "ref", rho=rho, u=u)
    m, ke = sim.invariants()
    n = fluid_count(orc, cfg)
    assert abs(m - rho0 * n) < 1e-13 * rho0 * n
    want = 0.5 * rho0 * float(u0 @ u0) * n
    assert abs(ke - want) < 1e-12 * want


@pytest.mark.parametrize("q", (19, 27))
def test_invariants_of_a_nonuniform_field(orc, q):
    """Taylor-Green velocity with a random density field on a periodic box:
    mass = sum rho_i and KE = 1/2 sum rho_i |u_i|^2, cell by cell from the
    input fields."""
    nx, ny, nz = 8, 6, 5
    cfg = orc.Config(q=q, nx=nx, ny=ny, nz=nz, geometry=orc.PERIODIC, model=orc.BGK, omega=1.1)
    u = W.taylor_green_velocity(nx, ny, nz, 0.05)
    u[2] = 0.01 * np.sin(np.arange(cfg.ntot))            # a third component too
    rho = W.random_density(71, cfg.ntot, 0.8, 1.25)
    sim = orc.Simulation(cfg, "ref", rho=rho, u=u)
    m, ke = sim.invariants()
    assert abs(m - rho.sum()) < 1e-13 * rho.sum()
    want = 0.5 * float((rho * (u * u).sum(axis=0)).sum())
    assert abs(ke - want) < 1e-12 * want


def test_invariants_skip_wall_cells(orc):
    """Wall cells hold momentum-exchange terms, not populations: a cavity
    whose lid moves fast still has the mass and energy of its fluid alone."""
    cfg = orc.Config(q=19, nx=5, ny=6, nz=7, model=orc.BGK, omega=1.0, u_lid=(0.3, 0.0, 0.0))
    sim = orc.Simulation(cfg, "ref")
    m, ke = sim.invariants()
    assert m == pytest.approx(fluid_count(orc, cfg), rel=1e-14)
    assert abs(ke) < 1e-28


GEOMS = [(19, "cavity", m) for m in ("bgk", "trt", "reg", "rr", "cm", "k")] + \
        [(19, "periodic", m) for m in ("bgk", "rr")] + \
        [(19, "channel", "trt")] + \
        [(27, "cavity", m) for m in ("bgk", "rr", "hm")] + \
        [(27, "periodic", "rr")]


@pytest.mark.parametrize("q,geom,model", GEOMS)
def test_reference_cells_equal_the_reference_step(orc, q, geom, model):
    """Every cell of a small lattice, evaluated one by one, equals the
    whole-lattice reference step bit for bit, from a random non-equilibrium
    state and after a few steps."""
    gid = {"cavity": orc.CAVITY, "periodic": orc.PERIODIC, "channel": orc.CHANNEL}[geom]
    cfg = orc.Config(q=q, nx=6, ny=5, nz=7, geometry=gid, model=orc.MODELS[model], omega=1.75,
                     omega_bulk=1.3 if model in ("reg", "rr", "cm") else None, omega3=1.2, omega4=0.9,
                     u_lid=(0.06, 0.01, 0.0))
    sim = orc.Simulation(cfg, "ref", u=W.random_velocity(73, cfg.ntot, amp=0.04).T)
    f = sim.populations()
    fl = sim.flags
    rnd = W.random_populations(74, q, cfg.ntot).T
    f[:, fl == orc.FLUID] = rnd[:, fl == orc.FLUID]
    sim.pop[:] = f.ravel()
    cells = np.arange(cfg.ntot)
    for _ in range(3):
        want = orc.reference_step(cfg, fl, sim.pop)
        got = orc.reference_cells(cfg, fl, sim.pop, cells)
        assert np.array_equal(got, want.reshape(q, cfg.ntot).T)
        sim.pop = want


@pytest.mark.parametrize("q", (19, 27))
def test_reference_cells_with_caller_walls(orc, q):
    """Caller geometry: random obstacles whose walls move with their own
    velocities and densities; a shuffled subset of cells (with repeats)."""
    cfg = orc.Config(q=q, nx=9, ny=8, nz=7, model=orc.TRT, omega=1.6, u_lid=(0.04, 0.0, 0.0))
    fl = orc.flags(cfg).reshape(cfg.nx, cfg.ny, cfg.nz).copy()
    rng = np.random.default_rng(75)
    fl[(rng.random(fl.shape) < 0.15) & (fl == orc.FLUID)] = orc.WALL
    fl = fl.ravel()
    wu = W.random_velocity(76, cfg.ntot, amp=0.03).T.copy()
    wu[:, fl == orc.FLUID] = 0.0
    wr = W.random_density(77, cfg.ntot)
    sim = orc.Simulation(cfg, "ref", cell_types=fl, wall_u=wu, wall_rho=wr)
    sim.step(4)
    cells = np.concatenate([W.shuffled_order(78, cfg.ntot)[:150], [0, 5, 5, cfg.ntot - 1]])
    want = orc.reference_step(cfg, fl, sim.pop).reshape(q, cfg.ntot).T
    got = orc.reference_cells(cfg, fl, sim.pop, cells)
    assert np.array_equal(got, want[cells])
