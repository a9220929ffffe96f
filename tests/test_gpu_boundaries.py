"""GPU parity of the boundary extensions against the FP64 oracle: pressure
(density) walls in every scheme and layout, curved walls (per-link wall
distance q) under the 2Pop pull scheme. FP64 to max |df| <= 1e-12, shifted
FP32 storage to velocity relative L2 <= 1e-5."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2010_11751_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
SCHEMES = ("2pop", "swap", "aa", "2pop_pull")


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def max_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def pressure_box(nx, ny, nz):
    """Still walls on every face but x = 0 (pressure wall, rho_w = 1.02,
    tangential u_w = 0.01 in its quadratic term) and x = nx-1 (pressure wall,
    rho_w = 0.99), plus one pressure cell inside the box."""
    n = nx * ny * nz
    x, y, z = np.arange(n) // (ny * nz), (np.arange(n) // nz) % ny, np.arange(n) % nz
    face = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
    types = np.where(face, O.WALL, O.FLUID).astype(np.uint8)
    inner_x = (y > 0) & (y < ny - 1) & (z > 0) & (z < nz - 1)
    rw = np.ones(n)
    types[(x == 0) & inner_x] = O.PRESSURE
    rw[(x == 0) & inner_x] = 1.02
    types[(x == nx - 1) & inner_x] = O.PRESSURE
    rw[(x == nx - 1) & inner_x] = 0.99
    c = ((nx // 2) * ny + ny // 2) * nz + nz // 2
    types[c] = O.PRESSURE
    rw[c] = 1.005
    wu = np.zeros((3, n))
    wu[1, types == O.PRESSURE] = 0.01
    return types, wu, rw


@pytest.mark.parametrize("layout", ("soa", "aos", "blocked"))
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q,coll", [(19, "trt"), (19, "bgk"), (27, "rr")])
def test_pressure_walls_match_oracle(lbm, q, coll, scheme, layout):
    nx, ny, nz, omega = 11, 9, 13, 1.7
    types, wu, rw = pressure_box(nx, ny, nz)
    u0 = W.random_velocity(109, nx * ny * nz, amp=0.03).T.copy()
    print(f"case: pressure walls q={q} {coll} {scheme} {layout}", flush=True)
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision=coll, omega=omega, layout=layout)
    sim.set_geometry(torch.from_numpy(types), torch.from_numpy(wu), torch.from_numpy(rw))
    sim.init_equilibrium(None, torch.from_numpy(u0))
    cfg = O.Config(q=q, nx=nx, ny=ny, nz=nz, model=O.MODELS[coll], omega=omega)
    ref = O.Simulation(cfg, "ref", u=u0, cell_types=types, wall_u=wu, wall_rho=rw)
    assert np.array_equal(sim.flags().cpu().numpy(), types)
    for n in (7, 1, 70):   # odd, even, then graph replays of the fused kernels
        sim.step(n)
        ref.step(n)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, n


@pytest.mark.parametrize("scheme", SCHEMES)
def test_pressure_walls_fp32_shifted(lbm, scheme):
    nx, ny, nz, omega = 11, 9, 13, 1.7
    types, wu, rw = pressure_box(nx, ny, nz)
    sim = lbm.Lattice(19, nx, ny, nz, scheme=scheme, collision="trt", omega=omega, dtype="f32")
    sim.set_geometry(torch.from_numpy(types), torch.from_numpy(wu), torch.from_numpy(rw))
    ref = O.Simulation(O.Config(q=19, nx=nx, ny=ny, nz=nz, model=O.TRT, omega=omega), "ref",
                       cell_types=types, wall_u=wu, wall_rho=rw)
    sim.step(60)
    ref.step(60)
    _, u = sim.macroscopic()
    _, ur = ref.macroscopic()
    err = rel_l2(u.cpu().numpy(), ur)
    print(f"pressure f32 {scheme}: velocity rel L2 {err:.2e}", flush=True)
    assert err <= 1e-5


def random_qlink(q, n, seed):
    return np.random.default_rng(seed).uniform(0.05, 1.0, size=(q, n))


@pytest.mark.parametrize("layout", ("soa", "aos", "blocked"))
@pytest.mark.parametrize("q,coll", [(19, "bgk"), (19, "trt"), (19, "cm"), (27, "rr")])
def test_curved_walls_match_oracle(lbm, q, coll, layout):
    """Random wall distances on every link of a moving-lid cavity, 2Pop pull:
    eager steps, then graph replays of the fused kernels."""
    nx, ny, nz, omega = 12, 10, 14, 1.71
    ql = random_qlink(q, nx * ny * nz, 113)
    print(f"case: curved q={q} {coll} {layout}", flush=True)
    sim = lbm.Lattice(q, nx, ny, nz, scheme="2pop_pull", collision=coll, omega=omega, u_lid=0.05, layout=layout)
    sim.set_wall_distances(torch.from_numpy(ql))
    cfg = O.Config(q=q, nx=nx, ny=ny, nz=nz, model=O.MODELS[coll], omega=omega, u_lid=(0.05, 0.0, 0.0))
    ref = O.Simulation(cfg, "2pop_pull", qlink=ql)
    for n in (1, 6, 70):
        sim.step(n)
        ref.step(n)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, n
    m, _ = sim.invariants()
    rm, _ = ref.invariants()
    assert abs(m - rm) <= 1e-12 * rm


def test_curved_walls_fp32_shifted(lbm):
    nx, ny, nz, omega = 12, 10, 14, 1.71
    ql = random_qlink(19, nx * ny * nz, 127)
    sim = lbm.Lattice(19, nx, ny, nz, scheme="2pop_pull", collision="trt", omega=omega, u_lid=0.05, dtype="f32")
    sim.set_wall_distances(torch.from_numpy(ql))
    ref = O.Simulation(O.Config(q=19, nx=nx, ny=ny, nz=nz, model=O.TRT, omega=omega, u_lid=(0.05, 0.0, 0.0)),
                       "2pop_pull", qlink=ql)
    sim.step(61)
    ref.step(61)
    _, u = sim.macroscopic()
    _, ur = ref.macroscopic()
    err = rel_l2(u.cpu().numpy(), ur)
    print(f"curved f32: velocity rel L2 {err:.2e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("qb,qt", [(0.2, 0.7), (0.9, 0.15)])
def test_curved_couette_on_the_gpu(lbm, qb, qt):
    """Plane Couette flow between walls at z = 1 - qb and z = nz - 2 + qt:
    the exact straight line through the wall positions."""
    nz, U, omega = 10, 0.02, 1.0
    sim = lbm.Lattice(19, 1, 1, nz, scheme="2pop_pull", collision="bgk", omega=omega, geometry="channel",
                      lid_velocity=(U, 0.0, 0.0))
    c, _, _ = O.lattice(19)
    ql = np.full((19, nz), 0.5)
    for k in range(19):
        if c[k, 2] == 1:
            ql[k, 1] = qb
        if c[k, 2] == -1:
            ql[k, nz - 2] = qt
    sim.set_wall_distances(torch.from_numpy(ql))
    sim.step(8000)
    _, u = sim.macroscopic()
    z = np.arange(1, nz - 1)
    want = U * (z - (1 - qb)) / ((nz - 2 + qt) - (1 - qb))
    assert max_err(u.cpu().numpy()[0, 1:nz - 1], want) < 1e-11 * U


def test_wall_distance_errors(lbm):
    n = 8 ** 3
    sim = lbm.Lattice(19, 8, scheme="aa", collision="bgk", omega=1.5, u_lid=0.03)
    with pytest.raises(lbm.LBMError) as e:          # curved walls need the pull form
        sim.set_wall_distances(torch.from_numpy(random_qlink(19, n, 1)))
    assert e.value.code == lbm.EUNSUPPORTED
    bad = np.full((19, n), 0.5)
    bad[3, 100] = 1.5
    with pytest.raises(lbm.LBMError) as e:
        sim.set_wall_distances(torch.from_numpy(bad))
    assert e.value.code == lbm.EINVAL
    plain = lbm.Lattice(19, 8, scheme="aa", collision="bgk", omega=1.5, u_lid=0.03)
    sim.set_wall_distances(torch.from_numpy(np.full((19, n), 0.5)))   # all half-way: the plain rule
    sim.step(9)
    plain.step(9)
    assert torch.equal(sim.populations().cpu(), plain.populations().cpu())
