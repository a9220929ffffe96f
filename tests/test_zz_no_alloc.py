"""The no-allocation invariants entry point (lbm_invariants_noalloc) against
lbm_invariants, through the C ABI: same kernels and summation order, so the
two agree bit for bit, also when a smaller lattice follows a larger one on
the same GPU (the fixed device array keeps the previous call's partials)."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def noalloc(lbm, sim):
    res = torch.full((2,), float("nan"), dtype=torch.float64, device=sim.device)
    with torch.cuda.stream(sim.stream):
        rc = lbm.lib().lbm_invariants_noalloc(sim.h, ctypes.c_void_p(res.data_ptr()))
    assert rc == lbm.OK, lbm.last_error()
    sim.sync()
    return res.cpu().numpy()


CASES = [  # (edge, scheme, collision, storage, steps): each call smaller than the one before
    (40, "aa", "trt", "f64", 7),
    (17, "2pop_pull", "bgk", "f32", 5),
    (9, "2pop", "rr", "f16", 4),
]


def test_noalloc_invariants_equal_lbm_invariants(lbm):
    for n, scheme, coll, dtype, steps in CASES:
        print(f"case: noalloc invariants {n}^3 {scheme} {coll} {dtype}, {steps} steps", flush=True)
        sim = lbm.Lattice(19, n, n + 1, n - 1, scheme=scheme, collision=coll, omega=1.7, u_lid=0.08, dtype=dtype)
        sim.step(steps)
        got = noalloc(lbm, sim)
        m, e = sim.invariants()
        assert np.isfinite(got).all() and e > 0.0
        assert got[0] == m and got[1] == e, (got, m, e)
        # the state is unchanged by the read-out: a second call gives the same
        assert np.array_equal(noalloc(lbm, sim), got)
        sim.close()


def test_noalloc_invariants_reject_lattices_beyond_the_scratch_maximum(lbm):
    n = 324  # 324^3 = 34 012 224 cells > 2^25
    print(f"case: noalloc invariants size limit {n}^3 f16 aa", flush=True)
    sim = lbm.Lattice(19, n, scheme="aa", collision="bgk", omega=1.8, dtype="f16")
    res = torch.zeros(2, dtype=torch.float64, device=sim.device)
    assert lbm.lib().lbm_invariants_noalloc(sim.h, ctypes.c_void_p(res.data_ptr())) == lbm.EINVAL
    assert "2^25" in lbm.last_error()
    sim.close()
