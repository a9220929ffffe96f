"""Pins of the oracle's caller-defined geometry: any cell may be a wall, and
each wall cell stores the momentum-exchange term of its own wall velocity u_w
and wall density rho_w, -6 t_k rho_w c_k . u_w (Eqs. momentum-exchange,
storage2). The built-in cavity is one such geometry."""
import numpy as np
import pytest

from paper_2010_11751_amd import workloads as W

SCHEMES = ("ref", "2pop", "swap", "aa", "2pop_pull")


@pytest.mark.parametrize("scheme", SCHEMES)
def test_cell_types_reproduce_the_builtin_cavity(orc, scheme):
    """The cavity's own flags as caller cell types, with the lid velocity as
    per-cell wall velocity of the lid layer: bit-identical evolution."""
    cfg = orc.Config(q=19, nx=8, ny=9, nz=10, model=orc.TRT, omega=1.6, u_lid=(0.05, 0.01, 0.0))
    fl = orc.flags(cfg)
    wu = np.zeros((3, cfg.ntot))
    for a in range(3):
        wu[a, fl == orc.LID] = cfg.u_lid[a]
    a = orc.Simulation(cfg, scheme)
    b = orc.Simulation(cfg, scheme, cell_types=fl, wall_u=wu)
    a.step(13)
    b.step(13)
    assert np.array_equal(a.populations(), b.populations())


@pytest.mark.parametrize("omega", [0.8, 1.0, 1.6])
def test_two_moving_walls_with_wall_density(orc, omega):
    """Channel between two walls moving along x at u_b and u_t, the top one
    with wall density rho_w: in the fluid (rho = 1) the steady profile is
    linear and reaches u_b and rho_w u_t at the half-way wall positions
    z = 1/2 and z = nz - 3/2 (the term carries rho_w u_w)."""
    nz, ub, ut, rw = 12, -0.02, 0.05, 1.2
    cfg = orc.Config(q=19, nx=1, ny=1, nz=nz, geometry=orc.CHANNEL, model=orc.BGK, omega=omega)
    types = np.zeros(nz, np.uint8)
    types[0] = types[-1] = orc.WALL
    wu = np.zeros((3, nz))
    wu[0, 0], wu[0, -1] = ub, ut
    wr = np.ones(nz)
    wr[-1] = rw
    sim = orc.Simulation(cfg, "aa", cell_types=types, wall_u=wu, wall_rho=wr)
    sim.step(20000)
    rho, u = sim.macroscopic()
    z = np.arange(1, nz - 1)
    want = ub + (rw * ut - ub) * (z - 0.5) / (nz - 2)
    assert np.abs(u[0, 1:nz - 1] - want).max() < 1e-9 * ut
    assert np.abs(rho[1:nz - 1] - 1).max() < 1e-10


def obstacle_types(orc, cfg, seed, fraction=0.1):
    """The geometry's own walls plus random interior obstacle cells and one
    solid block (flat faces next to the fluid)."""
    fl = orc.flags(cfg).reshape(cfg.nx, cfg.ny, cfg.nz).copy()
    rng = np.random.default_rng(seed)
    inner = rng.random(fl.shape) < fraction
    fl[inner & (fl == orc.FLUID)] = orc.WALL
    fl[2:5, 3:6, 2:4] = orc.WALL
    return fl.ravel()


@pytest.mark.parametrize("scheme", ("2pop", "swap", "aa", "2pop_pull"))
@pytest.mark.parametrize("q", (19, 27))
def test_obstacles_schemes_match_reference(orc, scheme, q):
    """Cavity with random obstacles whose walls move with random velocities
    and densities: every scheme equals the reference step bit for bit."""
    cfg = orc.Config(q=q, nx=11, ny=10, nz=9, model=orc.BGK, omega=1.7, u_lid=(0.04, 0.0, 0.0))
    types = obstacle_types(orc, cfg, 3)
    wu = W.random_velocity(5, cfg.ntot, amp=0.03).T.copy()
    wu[:, types == orc.FLUID] = 0.0
    wr = W.random_density(6, cfg.ntot)
    ref = orc.Simulation(cfg, "ref", cell_types=types, wall_u=wu, wall_rho=wr)
    sim = orc.Simulation(cfg, scheme, cell_types=types, wall_u=wu, wall_rho=wr)
    for n in (7, 1):
        ref.step(n)
        sim.step(n)
        assert np.array_equal(sim.populations(), ref.populations())


@pytest.mark.parametrize("q", (19, 27))
def test_resting_obstacles_conserve_mass(orc, q):
    """Resting obstacle walls (and the lid, moving along its own plane) move
    no mass across any link: total mass is conserved to round-off."""
    cfg = orc.Config(q=q, nx=11, ny=10, nz=9, model=orc.TRT, omega=1.9, u_lid=(0.05, 0.0, 0.0))
    types = obstacle_types(orc, cfg, 4)
    sim = orc.Simulation(cfg, "aa", cell_types=types)
    m0, _ = sim.invariants()
    sim.step(40)
    m1, _ = sim.invariants()
    assert abs(m1 - m0) < 1e-12 * m0


def test_wall_moving_into_the_fluid_injects_mass(orc):
    """A wall cell with a normal velocity component pushes fluid: the mass
    change of one step is the sum of the momentum-exchange terms it hands to
    its fluid neighbours, -6 t_k rho_w c_k . u_w over the bounced links."""
    cfg = orc.Config(q=19, nx=7, ny=7, nz=7, model=orc.BGK, omega=1.0)
    types = orc.flags(cfg).copy()
    wu = np.zeros((3, cfg.ntot))
    i = (3 * 7 + 3) * 7 + 0                      # cell (3, 3, 0) of the bottom wall
    wu[2, i] = 0.01                              # moves up, into the fluid
    c, t, _ = orc.lattice(19)
    sim = orc.Simulation(cfg, "ref", cell_types=types, wall_u=wu)
    m0, _ = sim.invariants()
    sim.step(1)
    m1, _ = sim.invariants()
    # links from the fluid into cell i: fluid x = i - c_k with c_kz = -1 ... the
    # bounced population is k with x + c_k = i, term -6 t_k c_k . u_w
    want = sum(-6 * t[k] * c[k, 2] * 0.01 for k in range(19) if c[k, 2] == -1)
    assert abs((m1 - m0) - want) < 1e-13   # round-off of a sum of 125
