"""The position-driven 2Pop pull and AA odd kernels of the built-in cavity
(every wall, edge and corner decision taken from the cell's coordinates, no
flag byte and no edge-cell list) against the FP64 oracle, and bit for bit
against the flag-driven kernels in every storage type and layout.

LBM_PULL_KERNEL (LBM_AA_KERNEL for the AA odd step) picks the kernel when a
lattice is created: "box" forces the position-driven one on the built-in
cavity, "flag" the flag-driven one; unset, the library takes whichever
measured faster for the storage type and layout."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2010_11751_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def lattice(lbm, monkeypatch, kernel, *args, **kw):
    var = "LBM_AA_KERNEL" if kw.get("scheme") == "aa" else "LBM_PULL_KERNEL"
    monkeypatch.setenv(var, kernel)
    try:
        return lbm.Lattice(*args, **kw)
    finally:
        monkeypatch.delenv(var)


@pytest.mark.parametrize("layout", ("soa", "aos", "blocked"))
@pytest.mark.parametrize("q,coll", [(19, "bgk"), (19, "trt"), (19, "cm"), (27, "rr"), (27, "bgk")])
def test_box_pull_fp64_matches_oracle(lbm, monkeypatch, q, coll, layout):
    """Ragged cavities (rows shorter and longer than a wave) with a lid moving
    in all three directions: eager steps, then graph replays."""
    for nx, ny, nz in ((12, 10, 14), (5, 7, 70)):
        omega = 1.73
        lid = (0.04, -0.015, 0.01)
        print(f"case: box pull q={q} {coll} {layout} {nx}x{ny}x{nz}", flush=True)
        sim = lattice(lbm, monkeypatch, "box", q, nx, ny, nz, scheme="2pop_pull", collision=coll, omega=omega,
                      layout=layout, lid_velocity=lid)
        ref = O.Simulation(O.Config(q=q, nx=nx, ny=ny, nz=nz, model=O.MODELS[coll], omega=omega, u_lid=lid),
                           "ref")
        for n in (1, 6, 70):
            sim.step(n)
            ref.step(n)
            assert np.abs(sim.populations().cpu().numpy() - ref.populations()).max() <= TOL, n
        m, _ = sim.invariants()
        rm, _ = ref.invariants()
        assert abs(m - rm) <= 1e-12 * rm


@pytest.mark.parametrize("dtype", ("f64", "f32", "f16"))
@pytest.mark.parametrize("layout", ("soa", "blocked"))
@pytest.mark.parametrize("q,coll", [(19, "trt"), (27, "rr")])
def test_box_pull_equals_flag_pull(lbm, monkeypatch, q, coll, layout, dtype):
    """Same bits as the flag-driven kernel, shifted storage included (the
    wall terms come from the same table rounded to the storage type)."""
    nx, ny, nz = 13, 11, 66
    kw = dict(scheme="2pop_pull", collision=coll, omega=1.91, layout=layout, dtype=dtype,
              lid_velocity=(0.05, 0.01, 0.0))
    got = {}
    for kernel in ("box", "flag"):
        sim = lattice(lbm, monkeypatch, kernel, q, nx, ny, nz, **kw)
        sim.step(37)
        got[kernel] = sim.populations().cpu()
        sim.step(64)
        got[kernel + "_later"] = sim.populations().cpu()
    assert torch.equal(got["box"], got["flag"])
    assert torch.equal(got["box_later"], got["flag_later"])


def test_box_pull_default_choice_at_256(lbm, monkeypatch):
    """The benchmark's FP32 blocked cavity: the default kernel (position-driven
    for this storage and layout) equals the flag-driven one after a few steps."""
    cav = W.CAVITY_256
    got = []
    for kernel in ("", "flag"):
        print(f"case: 256^3 f32 blocked pull, kernel '{kernel or 'default'}'", flush=True)
        sim = lattice(lbm, monkeypatch, kernel, 19, cav.n, scheme="2pop_pull", collision="bgk", omega=cav.omega,
                      u_lid=cav.u_lid, dtype="f32", layout="blocked")
        sim.step(5)
        got.append(sim.populations().cpu())
        del sim
        torch.cuda.empty_cache()
    assert torch.equal(got[0], got[1])


def test_caller_walls_leave_the_box_kernel(lbm, monkeypatch):
    """After lbm_set_geometry the wall terms are per cell, so the flag-driven
    kernel takes over: a moving obstacle changes the flow as in the oracle."""
    nx, ny, nz, omega = 10, 9, 12, 1.6
    sim = lattice(lbm, monkeypatch, "box", 19, nx, ny, nz, scheme="2pop_pull", collision="bgk", omega=omega,
                  u_lid=0.03)
    cfg = O.Config(q=19, nx=nx, ny=ny, nz=nz, omega=omega, u_lid=(0.03, 0.0, 0.0))
    types = O.flags(cfg).copy()
    wu = np.zeros((3, cfg.ntot))
    wu[0, types == O.LID] = 0.03
    c = ((nx // 2) * ny + ny // 2) * nz + nz // 2
    types[c] = O.WALL
    wu[1, c] = 0.02
    sim.set_geometry(torch.from_numpy(types), torch.from_numpy(wu), None)
    ref = O.Simulation(cfg, "ref", cell_types=types, wall_u=wu)
    sim.step(9)
    ref.step(9)
    assert np.abs(sim.populations().cpu().numpy() - ref.populations()).max() <= TOL


@pytest.mark.parametrize("layout", ("soa", "aos", "blocked"))
@pytest.mark.parametrize("q,coll", [(19, "bgk"), (19, "trt"), (27, "rr")])
def test_box_aa_fp64_matches_oracle(lbm, monkeypatch, q, coll, layout):
    """AA with the position-driven odd step: odd and even step counts, graph
    replays, a lid moving in all three directions."""
    nx, ny, nz, omega, lid = 12, 10, 14, 1.73, (0.04, -0.015, 0.01)
    print(f"case: box aa q={q} {coll} {layout}", flush=True)
    sim = lattice(lbm, monkeypatch, "box", q, nx, ny, nz, scheme="aa", collision=coll, omega=omega, layout=layout,
                  lid_velocity=lid)
    ref = O.Simulation(O.Config(q=q, nx=nx, ny=ny, nz=nz, model=O.MODELS[coll], omega=omega, u_lid=lid), "ref")
    for n in (1, 6, 70, 3):
        sim.step(n)
        ref.step(n)
        assert np.abs(sim.populations().cpu().numpy() - ref.populations()).max() <= TOL, n


@pytest.mark.parametrize("dtype", ("f32", "f16"))
@pytest.mark.parametrize("q,coll", [(19, "trt"), (27, "rr")])
def test_box_aa_equals_flag_aa(lbm, monkeypatch, q, coll, dtype):
    nx, ny, nz = 13, 11, 66
    kw = dict(scheme="aa", collision=coll, omega=1.91, dtype=dtype, lid_velocity=(0.05, 0.01, 0.0))
    got = {}
    for kernel in ("box", "flag"):
        sim = lattice(lbm, monkeypatch, kernel, q, nx, ny, nz, **kw)
        sim.step(37)
        got[kernel] = sim.populations().cpu()
        sim.step(64)
        got[kernel + "_later"] = sim.populations().cpu()
    assert torch.equal(got["box"], got["flag"])
    assert torch.equal(got["box_later"], got["flag_later"])


@pytest.mark.parametrize("scheme", ("2pop_pull", "aa"))
@pytest.mark.parametrize("layout", ("soa", "aos", "blocked"))
@pytest.mark.parametrize("q,coll", [(19, "bgk"), (19, "trt"), (27, "rr")])
def test_wrap_kernels_fp64_match_oracle(lbm, monkeypatch, q, coll, layout, scheme):
    """The position-driven kernels of the periodic box (wraps from the cell's
    position): random flow on ragged boxes, one of them a single cell thick
    in x and y, odd and even step counts and graph replays."""
    for nx, ny, nz in ((12, 10, 14), (1, 1, 9), (3, 70, 5)):
        n = nx * ny * nz
        u0 = W.random_velocity(211, n, amp=0.04).T.copy()
        print(f"case: wrap {scheme} q={q} {coll} {layout} {nx}x{ny}x{nz}", flush=True)
        sim = lattice(lbm, monkeypatch, "box", q, nx, ny, nz, scheme=scheme, collision=coll, omega=1.7,
                      layout=layout, geometry="periodic")
        sim.init_equilibrium(None, torch.from_numpy(u0))
        ref = O.Simulation(O.Config(q=q, nx=nx, ny=ny, nz=nz, geometry=O.PERIODIC, model=O.MODELS[coll], omega=1.7),
                           "ref", u=u0)
        for steps in (1, 6, 70, 3):
            sim.step(steps)
            ref.step(steps)
            assert np.abs(sim.populations().cpu().numpy() - ref.populations()).max() <= TOL, (nx, ny, nz, steps)


@pytest.mark.parametrize("dtype", ("f32", "f16"))
@pytest.mark.parametrize("scheme", ("2pop_pull", "aa"))
@pytest.mark.parametrize("layout", ("soa", "blocked"))
def test_wrap_kernels_equal_flag_kernels(lbm, monkeypatch, layout, scheme, dtype):
    n = 66
    u0 = torch.from_numpy(W.taylor_green_velocity(n, n, n, W.TGV_U0))
    got = {}
    for kernel in ("box", "flag"):
        sim = lattice(lbm, monkeypatch, kernel, 19, n, scheme=scheme, collision="bgk",
                      omega=W.omega_from_nu(W.TGV_NU), layout=layout, dtype=dtype, geometry="periodic")
        sim.init_equilibrium(None, u0)
        sim.step(41)
        got[kernel] = sim.populations().cpu()
    assert torch.equal(got["box"], got["flag"])


@pytest.mark.parametrize("scheme", ("2pop_pull", "aa"))
@pytest.mark.parametrize("q,coll", [(19, "trt"), (27, "rr")])
def test_box_kernels_rows_of_one_run(lbm, monkeypatch, q, coll, scheme):
    """Blocked layout with rows of exactly one run (nz = 256): the
    position-driven kernels address neighbours as the cell's own index plus a
    constant; FP64 against the oracle, FP16 bit for bit against the
    flag-driven kernels."""
    nx, ny, nz, omega, lid = 6, 5, 256, 1.8, (0.04, 0.01, 0.0)
    print(f"case: rows of one run, {scheme} q={q} {coll}", flush=True)
    sim = lattice(lbm, monkeypatch, "box", q, nx, ny, nz, scheme=scheme, collision=coll, omega=omega,
                  layout="blocked", lid_velocity=lid)
    ref = O.Simulation(O.Config(q=q, nx=nx, ny=ny, nz=nz, model=O.MODELS[coll], omega=omega, u_lid=lid), "ref")
    for n in (1, 4, 3):
        sim.step(n)
        ref.step(n)
        assert np.abs(sim.populations().cpu().numpy() - ref.populations()).max() <= TOL, n
    got = {}
    for kernel in ("box", "flag"):
        s16 = lattice(lbm, monkeypatch, kernel, q, nx, ny, nz, scheme=scheme, collision=coll, omega=omega,
                      layout="blocked", lid_velocity=lid, dtype="f16")
        s16.step(23)
        got[kernel] = s16.populations().cpu()
    assert torch.equal(got["box"], got["flag"])


@pytest.mark.parametrize("dtype", ("f64", "f32", "f16"))
@pytest.mark.parametrize("scheme,layout", [("2pop_pull", "blocked"), ("2pop_pull", "soa"), ("aa", "soa")])
def test_launch_shapes_change_no_result(lbm, scheme, layout, dtype):
    """The library's own launch shapes (FP64 pull: blocks of 128, three per
    CU; FP16 pull and FP32 / FP16 AA: blocks of 512) against fixed blocks of
    256 and 64: the same bits."""
    dims = (9, 7, 256) if layout == "blocked" else (13, 11, 70)
    got = []
    for block in (0, 256, 64):
        sim = lbm.Lattice(19, *dims, scheme=scheme, collision="trt", omega=1.85, lid_velocity=(0.05, 0.01, 0.0),
                          layout=layout, dtype=dtype, block_size=block)
        sim.step(21)
        got.append(sim.populations().cpu())
    assert torch.equal(got[0], got[1])
    assert torch.equal(got[0], got[2])
