"""GPU parity of the moment-space collision models (BGK-NW4, RM, HM, CM, CHM
and cumulant; Sec. 2.2, Sec. 2.6 Eq. RMcoll, Eq. bulk) against the FP64
oracle, through the C ABI.

FP64 storage: max |df| <= 1e-12 after 22 steps of a ragged 12x10x14 cavity
with a moving lid (several blocks and a ragged tail), every scheme, both
layouts on D3Q19 and D3Q27 (the cumulant model is D3Q19 only), with distinct
rates omega, omega_bulk, omega3, omega4 so that each relaxation path is
exercised. Shifted FP32 / FP16 storage: velocity relative L2 against the
GPU's FP64 run (itself held to the oracle above) on a Taylor-Green vortex.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2010_11751_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
SCHEMES = ("2pop", "swap", "aa", "2pop_pull")
MODELS = ("nw4", "rm", "hm", "cm", "chm", "k")
RATES = dict(omega=1.71, omega_bulk=1.3, omega3=1.2, omega4=0.9)


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def max_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def cases():
    out = []
    for q in (19, 27):
        for model in MODELS:
            if model == "k" and q == 27:
                continue
            for scheme in SCHEMES:
                for layout in ("soa", "aos"):
                    if layout == "aos" and scheme != "aa":
                        continue
                    out.append((q, model, scheme, layout))
    return out


@pytest.mark.parametrize("q,model,scheme,layout", cases())
def test_moment_space_models_match_oracle(lbm, q, model, scheme, layout):
    nx, ny, nz = 12, 10, 14
    print(f"case: q={q} {model} {scheme} {layout} {nx}x{ny}x{nz}", flush=True)
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision=model, u_lid=0.05, layout=layout, **RATES)
    cfg = O.Config(q=q, nx=nx, ny=ny, nz=nz, geometry=O.CAVITY, model=O.MODELS[model], u_lid=(0.05, 0.0, 0.0),
                   **RATES)
    ref = O.Simulation(cfg, "ref")
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= 1e-15
    for n in (21, 1):   # odd, then even step count (AA phase read-out both ways)
        sim.step(n)
        ref.step(n)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, n


@pytest.mark.parametrize("q", (19, 27))
def test_default_rates_and_velocity_field(lbm, q):
    """Periodic box started from the NW4 equilibrium of a random velocity
    field; omega3 = omega4 = 1 by default (the high orders equilibrate)."""
    n = 9
    u0 = W.random_velocity(65, n ** 3, amp=0.05).T.copy()
    for model in ("cm", "k") if q == 19 else ("cm", "hm"):
        sim = lbm.Lattice(q, n, scheme="aa", collision=model, omega=1.9, geometry="periodic")
        sim.init_equilibrium(None, torch.from_numpy(u0))
        cfg = O.Config(q=q, nx=n, ny=n, nz=n, geometry=O.PERIODIC, model=O.MODELS[model], omega=1.9)
        ref = O.Simulation(cfg, "ref", u=u0)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= 1e-15
        sim.step(9)
        ref.step(9)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL


def test_cumulant_model_rejects_d3q27(lbm):
    with pytest.raises(lbm.LBMError):
        lbm.Lattice(27, 8, collision="k", omega=1.5)


def relative_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("model", MODELS)
def test_shifted_storage_taylor_green(lbm, model):
    """Shifted FP32 and FP16 storage with FP32 arithmetic: velocity relative
    L2 against FP64 on a periodic Taylor-Green vortex (u0 = 0.04, nu = 0.01)
    after 200 AA steps, <= 1e-5 (FP32) and <= 1e-3 (FP16)."""
    n, steps, omega = 32, 200, W.omega_from_nu(0.01)
    u0 = torch.from_numpy(W.taylor_green_velocity(n, n, n, W.TGV_U0))
    us = {}
    for dtype in ("f64", "f32", "f16"):
        sim = lbm.Lattice(19, n, scheme="aa", collision=model, omega=omega, geometry="periodic", dtype=dtype,
                          omega3=1.0, omega4=1.0)
        sim.init_equilibrium(None, u0)
        sim.step(steps)
        us[dtype] = sim.macroscopic()[1].cpu().numpy()
    e32 = relative_l2(us["f32"], us["f64"])
    e16 = relative_l2(us["f16"], us["f64"])
    print(f"{model}: velocity rel L2 f32 {e32:.3e} f16 {e16:.3e}", flush=True)
    assert e32 <= 1e-5
    assert e16 <= 1e-3


@pytest.mark.parametrize("q,model", [(19, "cm"), (19, "k"), (27, "chm")])
@pytest.mark.parametrize("dtype", ("f64", "f32"))
def test_schemes_and_layouts_agree_bit_exactly(lbm, q, model, dtype):
    base = None
    for layout in ("soa", "aos"):
        for scheme in SCHEMES:
            sim = lbm.Lattice(q, 11, 9, 13, scheme=scheme, collision=model, u_lid=0.05, layout=layout, dtype=dtype,
                              **RATES)
            sim.step(17)
            f = sim.populations().cpu()
            if base is None:
                base = f
            else:
                assert torch.equal(f, base), (layout, scheme)
