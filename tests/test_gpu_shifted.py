"""Shifted storage (g = f - t_k stored in FP32 or FP16, collision and moments
in FP32) under every scheme, layout and lattice, against the FP64 oracle.

Bounds on the velocity field, relative L2 against FP64: 1e-5 with FP32
storage and 1e-3 with FP16 storage. What else holds exactly:
  - SoA and AoS hold the same values in a different order, so each scheme
    gives the same bits in both layouts, in FP16 as in FP32.
  - In FP32 every scheme gives the same bits (tested beside the FP64 sweep).
    In FP16 they do not: a bounce-back adds the wall term w_k to f_out_k,
    and the schemes round that sum to the storage type at different points
    (2Pop push and the AA odd push round f_out_k + w_k once; the pull
    gathers and the swap stream add w_k to an f_out_k already rounded).
    Each FP16 scheme is therefore checked against the oracle on its own.
  - A checkpoint (natural FP64 populations, then set) is bit exact in FP16
    when the natural state is a stored value (2Pop push, swap, AA after an
    even count). In pull form (AA after an odd count, 2Pop pull) a natural
    population across a wall is the FP32 sum of two stored FP16 values,
    which set_populations must round to FP16 again; the restored run then
    stays within the FP16 bound of the uninterrupted one.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2010_11751_amd import workloads as W

pytestmark = pytest.mark.gpu

SCHEMES = ("2pop", "swap", "aa", "2pop_pull")
BOUND = {"f32": 1e-5, "f16": 1e-3}


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def cfg(q, nx, ny, nz, coll, omega, u_lid=0.0, geometry=O.CAVITY):
    return O.Config(q=q, nx=nx, ny=ny, nz=nz, geometry=geometry, model=O.MODELS[coll], omega=omega,
                    u_lid=(u_lid, 0.0, 0.0))


@pytest.mark.parametrize("dtype", ("f32", "f16"))
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q,coll", [(19, "bgk"), (19, "trt"), (27, "bgk"), (27, "rr")])
def test_shifted_cavity_every_scheme_matches_oracle(lbm, q, coll, scheme, dtype):
    """Ragged 12x10x14 cavity (several blocks and a partial one, every cell
    type): eager steps of odd and even count, velocity against FP64."""
    nx, ny, nz, omega, u_lid = 12, 10, 14, 1.71, 0.05
    print(f"case: shifted cavity q={q} {coll} {scheme} {dtype}", flush=True)
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision=coll, omega=omega, u_lid=u_lid, dtype=dtype)
    ref = O.Simulation(cfg(q, nx, ny, nz, coll, omega, u_lid), "ref")
    for n in (21, 1, 40):
        sim.step(n)
        ref.step(n)
        _, u = sim.macroscopic()
        _, ur = ref.macroscopic()
        err = rel_l2(u.cpu().numpy(), ur)
        df = float(np.abs(sim.populations().cpu().numpy() - ref.populations()).max())
        print(f"  after +{n}: velocity rel L2 {err:.2e}, max |df| {df:.2e}", flush=True)
        assert err <= BOUND[dtype], n
    m, _ = sim.invariants()
    rm, _ = ref.invariants()
    assert abs(m - rm) <= 1e-3 * rm


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q,coll", [(19, "trt"), (27, "rr")])
def test_fp16_layouts_agree_bit_exactly(lbm, q, coll, scheme):
    """SoA, AoS and blocked FP16 storage: same values in another order, same
    bits. The lid moves in x and y and the run is long enough (40 steps) for
    a value whose FP32 result lies near an FP16 rounding boundary to turn up:
    a kernel that rounds such a value once instead of twice (a mixed-precision
    instruction with an FP16 result) stores a different last bit."""
    got = {}
    for layout in ("soa", "aos", "blocked"):
        sim = lbm.Lattice(q, 11, 9, 13, scheme=scheme, collision=coll, omega=1.83, lid_velocity=(0.05, 0.01, 0.0),
                          layout=layout, dtype="f16")
        sim.step(40)
        got[layout] = sim.populations().cpu()
    assert torch.equal(got["soa"], got["aos"])
    assert torch.equal(got["soa"], got["blocked"])


@pytest.mark.parametrize("scheme,first,exact", [
    ("2pop", 51, True), ("swap", 51, True), ("aa", 50, True),
    ("aa", 51, False), ("2pop_pull", 51, False)])
def test_fp16_checkpoint_round_trip(lbm, scheme, first, exact):
    """first steps, save natural populations, destroy, create, restore,
    100 - first steps, against 100 uninterrupted steps."""
    kw = dict(scheme=scheme, collision="trt", omega=1.8, u_lid=0.04, dtype="f16")
    a = lbm.Lattice(19, 13, 11, 12, **kw)
    a.step(100)
    want = a.populations().cpu()
    _, u_want = a.macroscopic()
    b = lbm.Lattice(19, 13, 11, 12, **kw)
    b.step(first)
    saved = b.populations().cpu()
    b.close()
    c = lbm.Lattice(19, 13, 11, 12, **kw)
    c.set_populations(saved)
    if exact:
        assert torch.equal(c.populations().cpu(), saved)
    c.step(100 - first)
    got = c.populations().cpu()
    if exact:
        assert torch.equal(got, want)
    else:
        _, u_got = c.macroscopic()
        err = rel_l2(u_got.cpu().numpy(), u_want.cpu().numpy())
        print(f"{scheme} restored after {first}: velocity rel L2 vs uninterrupted {err:.2e}", flush=True)
        assert err <= BOUND["f16"]


@pytest.mark.parametrize("dtype", ("f32", "f16"))
@pytest.mark.parametrize("scheme", ("aa", "2pop_pull"))
@pytest.mark.parametrize("q", (19, 27))
@pytest.mark.parametrize("chunk", (40, 100))
def test_shifted_taylor_green_periodic(lbm, q, scheme, dtype, chunk):
    """Periodic 32^3 Taylor-Green vortex (u0 = 0.04, nu = 0.01), 200 steps.
    Chunks of 40 steps run eagerly, so every odd (AA) or every (pull) step
    takes the fast kernel with the z-wrap index correction on the z faces;
    chunks of 100 replay 64-step graphs of the fused kernels in between."""
    n, steps, omega = 32, 200, W.omega_from_nu(W.TGV_NU)
    u0 = W.taylor_green_velocity(n, n, n, W.TGV_U0)
    print(f"case: tgv 32^3 q={q} {scheme} {dtype} chunk {chunk}", flush=True)
    sim = lbm.Lattice(q, n, scheme=scheme, collision="bgk", omega=omega, geometry="periodic", dtype=dtype)
    sim.init_equilibrium(None, torch.from_numpy(u0))
    ref = O.Simulation(cfg(q, n, n, n, "bgk", omega, geometry=O.PERIODIC), "ref", u=u0)
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        done += k
    ref.step(steps)
    _, u = sim.macroscopic()
    _, ur = ref.macroscopic()
    err = rel_l2(u.cpu().numpy(), ur)
    print(f"  velocity rel L2 = {err:.3e}", flush=True)
    assert err <= BOUND[dtype]


@pytest.mark.parametrize("scheme", ("aa", "2pop_pull"))
def test_taylor_green_256_storage_accuracy(lbm, scheme):
    """The 256^3 Taylor-Green workload after 200 steps: FP32 and FP16 shifted
    storage against the FP64 run of the same kernels (whose steps match the
    oracle on sampled cells at this size), velocity relative L2."""
    n = W.TGV_N
    omega = W.omega_from_nu(W.TGV_NU)
    u0 = torch.from_numpy(W.taylor_green_velocity(n, n, n, W.TGV_U0))
    fields = {}
    for dtype in ("f64", "f32", "f16"):
        print(f"case: tgv 256^3 {scheme} {dtype}", flush=True)
        sim = lbm.Lattice(19, n, scheme=scheme, collision="bgk", omega=omega, geometry="periodic", dtype=dtype)
        sim.init_equilibrium(None, u0)
        sim.step(200)
        _, u = sim.macroscopic()
        fields[dtype] = u.cpu().numpy()
        del sim, u
        torch.cuda.empty_cache()
    for dtype in ("f32", "f16"):
        err = rel_l2(fields[dtype], fields["f64"])
        print(f"  {dtype}: velocity rel L2 vs FP64 = {err:.3e}", flush=True)
        assert err <= BOUND[dtype]
