"""Batched ensemble on the GPU: each cavity of one batched launch equals the
same cavity run alone (bit for bit, same storage type) under every launch
shape the autotuner can pick, graph replay equals the eager loop,
per-cavity sequential launches equal the batched launch, and FP64 batches
match the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2010_11751_amd import workloads as W

pytestmark = pytest.mark.gpu

MEMBERS = [(8, 1.95, 0.03), (13, 1.6, 0.05), (17, 1.85, 0.02), (5, 1.2, 0.01), (22, 1.99, 0.03), (11, 0.9, 0.04)]


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def make_batch(lbm, dtype, scheme="aa", coll="trt", **kw):
    cav = [lbm.Cavity(n, w, u) for n, w, u in MEMBERS]
    return lbm.Batch(cav, scheme=scheme, collision=coll, dtype=dtype, **kw)


SCHEMES = ("aa", "2pop", "2pop_pull")


def edge_cells(n):
    """Fluid cells of a cubic cavity of edge n (walls included) that lie next
    to two or more walls: m = n - 2 fluid cells per edge, two boundary values
    per axis (one when m = 1)."""
    m = n - 2
    if m <= 2:
        return m ** 3
    return 3 * 4 * (m - 2) + 8


@pytest.mark.parametrize("dtype", ("f64", "f32", "f16"))
@pytest.mark.parametrize("scheme", SCHEMES)
def test_batch_equals_single_runs(lbm, dtype, scheme):
    print(f"case: batch {scheme} {dtype}", flush=True)
    b = make_batch(lbm, dtype, scheme=scheme, use_graph=False)
    b.step(11)
    for j, (n, w, u) in enumerate(MEMBERS):
        s = lbm.Lattice(19, n, scheme=scheme, collision="trt", omega=w, u_lid=u, dtype=dtype)
        s.step(11)
        assert torch.equal(b.populations(j).cpu(), s.populations().cpu()), j


@pytest.mark.parametrize("block,cpt,waves,xcd", [(64, 1, -1, 1), (256, 2, 0, 0), (128, 4, 3, 1), (1024, 1, 6, 0),
                                                 (512, 4, -1, 1)])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_launch_shapes_equal_single_runs(lbm, scheme, block, cpt, waves, xcd):
    """Every launch shape the autotuner may choose (block size, runs of cells
    per block, residency cap, tiles dealt to the XCDs in parts or in order)
    gives the single runs' bits."""
    print(f"case: batch shape {scheme} block {block} cpt {cpt} waves {waves} xcd {xcd}", flush=True)
    b = make_batch(lbm, "f32", scheme=scheme, use_graph=False, block_size=block, cells_per_thread=cpt,
                   waves_per_simd=waves, xcd_split=xcd)
    shape = b.launch_shape()
    assert shape[:4] == (block, cpt, waves, xcd)
    assert shape[4] == sum(edge_cells(n) for n, _, _ in MEMBERS)
    b.step(9)
    for j, (n, w, u) in enumerate(MEMBERS):
        s = lbm.Lattice(19, n, scheme=scheme, collision="trt", omega=w, u_lid=u, dtype="f32")
        s.step(9)
        assert torch.equal(b.populations(j).cpu(), s.populations().cpu()), j


@pytest.mark.parametrize("scheme", SCHEMES)
def test_graph_replay_equals_eager(lbm, scheme):
    a = make_batch(lbm, "f32", scheme=scheme, use_graph=False)
    g = make_batch(lbm, "f32", scheme=scheme, use_graph=True, graph_steps=4)
    for n in (12, 3, 9):   # graph replays, odd remainders and a phase change
        a.step(n)
        g.step(n)
        a.sync()
        g.sync()
        for j in range(len(MEMBERS)):
            assert torch.equal(a.populations(j).cpu(), g.populations(j).cpu()), (n, j)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_sequential_equals_batched(lbm, scheme):
    a = make_batch(lbm, "f32", scheme=scheme, use_graph=False)
    s = make_batch(lbm, "f32", scheme=scheme, use_graph=False)
    a.step(7)
    s.step_sequential(7)
    for j in range(len(MEMBERS)):
        assert torch.equal(a.populations(j).cpu(), s.populations(j).cpu()), j


@pytest.mark.parametrize("scheme", SCHEMES)
def test_fp64_batch_matches_oracle(lbm, scheme):
    b = make_batch(lbm, "f64", scheme=scheme)
    b.step(20)
    masses, kes = b.invariants()
    for j, (n, w, u) in enumerate(MEMBERS):
        ref = O.Simulation(O.Config(q=19, nx=n, ny=n, nz=n, model=O.TRT, omega=w, u_lid=(u, 0, 0)), "ref")
        m0, _ = ref.invariants()
        ref.step(20)
        assert np.abs(b.populations(j).cpu().numpy() - ref.populations()).max() <= 1e-12, j
        rm, re_ = ref.invariants()
        assert abs(masses[j] - rm) <= 1e-12 * rm
        assert abs(masses[j] - m0) <= 1e-12 * m0
        assert abs(kes[j] - re_) <= 1e-10 * max(re_, 1e-30)
        rho, uu = b.macroscopic(j)
        rr, ur = ref.macroscopic()
        assert np.abs(uu.cpu().numpy() - ur).max() <= 1e-12


def test_autotuned_batch_is_still_correct(lbm):
    b = make_batch(lbm, "f64", autotune=True)
    cells, fluid, blk = b.info()
    assert cells == sum(n ** 3 for n, _, _ in MEMBERS)
    assert fluid == sum((n - 2) ** 3 for n, _, _ in MEMBERS)
    assert blk in (64, 128, 256, 512, 1024)
    shape = b.launch_shape()
    assert shape[0] == blk and shape[1] in (1, 2, 4) and shape[2] in (-1, 0, 2, 3, 4, 6) and shape[3] in (0, 1)
    b.step(6)
    n, w, u = MEMBERS[1]
    ref = O.Simulation(O.Config(q=19, nx=n, ny=n, nz=n, model=O.TRT, omega=w, u_lid=(u, 0, 0)), "ref")
    ref.step(6)
    assert np.abs(b.populations(1).cpu().numpy() - ref.populations()).max() <= 1e-12


def test_autotune_cache_round_trip(lbm, tmp_path):
    """The first autotuned creation appends its launch shape (block size,
    cells per thread, residency cap, XCD split) under the ensemble's key; the second
    finds it and uses it without trial runs."""
    path = tmp_path / "tune.txt"
    cav = [lbm.Cavity(n, w, u) for n, w, u in MEMBERS]
    a = lbm.Batch(cav, scheme="aa", collision="trt", dtype="f32", autotune=True, autotune_cache=path)
    shape = a.launch_shape()[:4]
    a.close()
    lines = path.read_text().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    key, *values = lines[0].split()
    assert tuple(int(v) for v in values) == shape and key.startswith("gfx")
    b = lbm.Batch(cav, scheme="aa", collision="trt", dtype="f32", autotune=True, autotune_cache=path)
    assert b.launch_shape()[:4] == shape
    b.step(4)
    b.close()
    assert len([l for l in path.read_text().split("\n") if l.strip()]) == 1


@pytest.mark.parametrize("coll", ("cm", "k", "rr"))
def test_batch_other_collisions_match_oracle(lbm, coll):
    """The ensemble with other collision models (moment-space models at
    omega3 = omega4 = 1, omega_bulk = omega), FP64, against the oracle."""
    b = make_batch(lbm, "f64", coll=coll)
    b.step(10)
    for j, (n, w, u) in enumerate(MEMBERS):
        ref = O.Simulation(O.Config(q=19, nx=n, ny=n, nz=n, model=O.MODELS[coll], omega=w, u_lid=(u, 0, 0)), "ref")
        ref.step(10)
        assert np.abs(b.populations(j).cpu().numpy() - ref.populations()).max() <= 1e-12, j
