"""Pins of the oracle's boundary extensions of the link-wise bounce-back
(Sec. 1.1: it extends to curved walls while staying local; Sec. 2.1,
Eq. momentum-exchange, has the wall density rho_w).

Curved walls: the wall crosses the link from fluid cell x to wall cell
s = x - c_k at the fraction q of the link; q = 1/2 is the half-way wall.
Pressure walls: cells of type PRESSURE reflect with the opposite sign and
store twice the even part of the equilibrium at their density (the density,
not the velocity, is set at the half-way wall)."""
import math

import numpy as np
import pytest

from paper_2010_11751_amd import workloads as W


def nu_of(omega):
    return (1.0 / omega - 0.5) / 3.0


def channel_qlink(orc, cfg, qb, qt):
    """qlink of a channel (walls at z = 0 and z = nz-1): the links of the
    first and last fluid layers towards the walls get qb and qt."""
    c, _, _ = orc.lattice(cfg.q)
    ql = np.full((cfg.q, cfg.ntot), 0.5)
    z = np.arange(cfg.ntot) % cfg.nz
    for k in range(cfg.q):
        if c[k, 2] == 1:      # x - c_k lies one layer below
            ql[k, z == 1] = qb
        if c[k, 2] == -1:
            ql[k, z == cfg.nz - 2] = qt
    return ql


@pytest.mark.parametrize("scheme", ("ref", "2pop_pull"))
def test_half_way_distances_are_the_plain_bounce_back(orc, scheme):
    """q = 1/2 on every link gives the half-way rule bit for bit."""
    cfg = orc.Config(q=19, nx=7, ny=6, nz=8, model=orc.TRT, omega=1.7, u_lid=(0.05, 0.02, 0.0))
    u0 = W.random_velocity(101, cfg.ntot, amp=0.03).T
    a = orc.Simulation(cfg, scheme, u=u0)
    b = orc.Simulation(cfg, scheme, u=u0, qlink=np.full((19, cfg.ntot), 0.5))
    a.step(9)
    b.step(9)
    assert np.array_equal(a.populations(), b.populations())


@pytest.mark.parametrize("model", ("bgk", "trt"))
@pytest.mark.parametrize("omega", (0.8, 1.0, 1.6))
@pytest.mark.parametrize("qb,qt", [(0.2, 0.7), (0.35, 0.95), (0.8, 0.15), (1.0, 0.05)])
def test_couette_between_curved_walls_is_exact(orc, model, omega, qb, qt):
    """Plane Couette flow with the still wall at z = 1 - qb and the lid
    (moving at U) at z = nz - 2 + qt: the steady profile is the straight
    line through the two wall positions, u_x = U (z - z_b) / (z_t - z_b),
    for every q and relaxation rate."""
    nz, U = 10, 0.02
    cfg = orc.Config(q=19, nx=1, ny=1, nz=nz, geometry=orc.CHANNEL, model=orc.MODELS[model], omega=omega,
                     u_lid=(U, 0.0, 0.0))
    sim = orc.Simulation(cfg, "ref", qlink=channel_qlink(orc, cfg, qb, qt))
    sim.step(8000)
    _, u = sim.macroscopic()
    z = np.arange(1, nz - 1)
    zb, zt = 1 - qb, nz - 2 + qt
    want = U * (z - zb) / (zt - zb)
    assert np.abs(u[0, 1:nz - 1] - want).max() < 1e-11 * U
    assert np.abs(u[1:, 1:nz - 1]).max() < 1e-13


@pytest.mark.parametrize("q", (19, 27))
def test_curved_pull_scheme_equals_reference_step(orc, q):
    """Random wall distances on every link of a moving-lid cavity: the 2Pop
    pull scheme (the pull form the rule is written in) equals the reference
    step bit for bit, at every step count."""
    cfg = orc.Config(q=q, nx=7, ny=6, nz=8, model=orc.TRT, omega=1.75, u_lid=(0.05, 0.0, 0.01))
    ql = np.random.default_rng(103).uniform(0.05, 1.0, size=(q, cfg.ntot))
    a = orc.Simulation(cfg, "ref", qlink=ql)
    b = orc.Simulation(cfg, "2pop_pull", qlink=ql)
    for n in (1, 4, 3):
        a.step(n)
        b.step(n)
        assert np.array_equal(a.populations(), b.populations()), n


def test_curved_walls_need_a_pull_form_scheme(orc):
    cfg = orc.Config(q=19, nx=5, ny=5, nz=5)
    with pytest.raises(ValueError):
        orc.Simulation(cfg, "aa", qlink=np.full((19, cfg.ntot), 0.5))


def box_with_pressure_wall(orc, q, rho_w, omega, model="bgk"):
    """A closed box whose x = 0 face is a pressure wall of density rho_w,
    the other faces still walls."""
    nx, ny, nz = 6, 5, 7
    cfg = orc.Config(q=q, nx=nx, ny=ny, nz=nz, geometry=orc.CAVITY, model=orc.MODELS[model], omega=omega)
    fl = orc.flags(cfg).copy()
    fl[fl == orc.LID] = orc.WALL
    rw = np.ones(cfg.ntot)
    for y in range(1, ny - 1):
        for z in range(1, nz - 1):
            fl[(0 * ny + y) * nz + z] = orc.PRESSURE
            rw[(0 * ny + y) * nz + z] = rho_w
    return cfg, fl, rw


@pytest.mark.parametrize("q", (19, 27))
@pytest.mark.parametrize("omega", (0.7, 1.0, 1.7))
def test_box_relaxes_to_the_pressure_wall_density(orc, q, omega):
    """Starting at rest with rho = 1, the fluid of a box with one pressure
    wall at rho_w = 1.01 ends at rest with rho = rho_w everywhere: the only
    steady state the anti-bounce-back admits."""
    cfg, fl, rw = box_with_pressure_wall(orc, q, 1.01, omega)
    sim = orc.Simulation(cfg, "ref", cell_types=fl, wall_rho=rw)
    sim.step(3000)
    rho, u = sim.macroscopic()
    m = fl == orc.FLUID
    assert np.abs(rho[m] - 1.01).max() < 1e-13
    assert np.abs(u[:, m]).max() < 1e-13


def test_rest_at_the_wall_density_is_a_fixed_point(orc):
    cfg, fl, rw = box_with_pressure_wall(orc, 19, 0.97, 1.3)
    rho0 = np.where(fl == orc.FLUID, 0.97, 1.0)
    sim = orc.Simulation(cfg, "ref", cell_types=fl, wall_rho=rw, rho=rho0)
    f0 = sim.populations()
    sim.step(50)
    assert np.abs(sim.populations() - f0).max() < 1e-15


def pressure_channel(orc, nx, nz, d, omega, steps):
    """Channel between still walls at z = 0 and nz - 1 (half-way at z = 1/2
    and nz - 3/2), pressure walls of density 1 + d/2 at x = 0 and 1 - d/2
    at x = nx - 1; TRT with Lambda = 3/16 (no wall slip)."""
    cfg = orc.Config(q=19, nx=nx, ny=1, nz=nz, geometry=orc.PERIODIC, model=orc.TRT, omega=omega,
                     trt_lambda=3 / 16)
    types = np.zeros(cfg.ntot, np.uint8)
    rw = np.ones(cfg.ntot)
    x, z = np.arange(cfg.ntot) // nz, np.arange(cfg.ntot) % nz
    types[(x == 0) | (x == nx - 1)] = orc.PRESSURE
    rw[x == 0], rw[x == nx - 1] = 1 + d / 2, 1 - d / 2
    types[(z == 0) | (z == nz - 1)] = orc.WALL
    sim = orc.Simulation(cfg, "ref", cell_types=types, wall_rho=rw)
    sim.step(steps)
    rho, u = sim.macroscopic()
    return rho.reshape(nx, nz), u[0].reshape(nx, nz)


def test_pressure_driven_channel():
    """Mid-channel, the steady profile is the Navier-Stokes parabola of the
    local pressure gradient (p = rho/3). The gradient there equals the one
    the walls' densities impose over the half-way distance nx - 2, up to a
    loss at the ends that is independent of the length, so its relative size
    halves when the channel doubles."""
    import oracle as orc
    nz, d, omega = 10, 2e-4, 1.2
    z = np.arange(1, nz - 1)
    shape = (z - 0.5) * (nz - 1.5 - z)
    errs = []
    for nx in (40, 80):
        rho, ux = pressure_channel(orc, nx, nz, d, omega, 40000)
        xm = nx // 2
        r = rho[xm, 1:nz - 1].mean()
        g_local = -(rho[xm + 1, 1:nz - 1].mean() - rho[xm - 1, 1:nz - 1].mean()) / 2 / 3
        assert np.abs(ux[xm, 1:nz - 1] - g_local / (2 * nu_of(omega) * r) * shape).max() < 1e-6 * ux[xm].max()
        g_mean = d / 3 / (nx - 2)
        want = g_mean / (2 * nu_of(omega) * r) * shape
        errs.append(np.abs(ux[xm, 1:nz - 1] - want).max() / want.max())
    assert errs[0] < 0.05 and errs[1] < 0.03
    assert 1.8 < errs[0] / errs[1] < 2.2


@pytest.mark.parametrize("q", (19, 27))
def test_schemes_agree_with_pressure_walls(orc, q):
    """Every scheme applies the reflected sign at the same sites: 2Pop, swap,
    AA and 2Pop pull equal the reference step bit for bit, in both layouts."""
    cfg, fl, rw = box_with_pressure_wall(orc, q, 1.02, 1.6, "trt")
    fl = fl.copy()
    fl[(1 * 5 + 2) * 7 + 3] = orc.PRESSURE          # an inner pressure cell as well
    rw[(1 * 5 + 2) * 7 + 3] = 0.99
    wu = np.zeros((3, cfg.ntot))
    wu[1, fl == orc.PRESSURE] = 0.01                 # pressure walls with a tangential velocity term
    u0 = W.random_velocity(107, cfg.ntot, amp=0.03).T
    ref = orc.Simulation(cfg, "ref", cell_types=fl, wall_rho=rw, wall_u=wu, u=u0)
    ref.step(5)
    want = ref.populations()
    for layout in (orc.SOA, orc.AOS):
        c2 = orc.Config(q=q, nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, model=cfg.model, omega=cfg.omega, layout=layout)
        for scheme in ("2pop", "swap", "aa", "2pop_pull"):
            sim = orc.Simulation(c2, scheme, cell_types=fl, wall_rho=rw, wall_u=wu, u=u0)
            sim.step(5)
            assert np.array_equal(sim.populations(), want), (layout, scheme)
