"""GPU parity: the HIP path against the FP64 CPU oracle, through the C ABI.

FP64 storage must match the oracle to max |df| <= 1e-12 (populations are of
order 0.05-0.4, so this is a few hundred ulps of headroom for the different
but algebraically equal operation order). Flags and neighbour indices are
compared bit for bit. Small cases span several 256-thread blocks and a
ragged tail; every scheme x collision x layout x lattice is covered.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2010_11751_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
SCHEMES = ("2pop", "swap", "aa", "2pop_pull")
COLLS = ("bgk", "trt", "reg", "rr")
GEOM = {"cavity": O.CAVITY, "periodic": O.PERIODIC, "channel": O.CHANNEL}


@pytest.fixture(scope="module")
def lbm(hiplib):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hiplib


def oracle_cfg(q, nx, ny, nz, coll, omega, u_lid=(0.0, 0.0, 0.0), geometry="cavity", omega_bulk=None, lam=0.25):
    return O.Config(q=q, nx=nx, ny=ny, nz=nz, geometry=GEOM[geometry], model=O.MODELS[coll], omega=omega,
                    trt_lambda=lam, omega_bulk=omega_bulk, u_lid=tuple(u_lid))


def max_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def test_config_small_cavity_matches_oracle(lbm):
    """D3Q19 BGK 32^3 cavity, FP64 2Pop SoA, lid 0.02, Re 100, 100 steps."""
    cav = W.CAVITY_SMALL
    print(f"case: 32^3 BGK 2pop f64 omega={cav.omega:.6f}", flush=True)
    sim = lbm.Lattice(19, cav.n, scheme="2pop", collision="bgk", omega=cav.omega, u_lid=cav.u_lid)
    cfg = oracle_cfg(19, cav.n, cav.n, cav.n, "bgk", cav.omega, (cav.u_lid, 0, 0))
    ref = O.Simulation(cfg, "2pop")
    assert np.array_equal(sim.flags().cpu().numpy(), ref.flags)
    sim.step(100)
    ref.step(100)
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL
    rho, u = sim.macroscopic()
    rr, ur = ref.macroscopic()
    assert max_err(rho.cpu().numpy(), rr) <= TOL
    assert max_err(u.cpu().numpy(), ur) <= TOL
    info = sim.info()
    assert info.fluid_cells == 30 ** 3 and info.steps_done == 100


@pytest.mark.parametrize("q", (19, 27))
@pytest.mark.parametrize("layout", ("soa", "aos", "blocked"))
@pytest.mark.parametrize("coll", COLLS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_scheme_collision_layout_sweep(lbm, q, layout, coll, scheme):
    nx, ny, nz, omega = 12, 10, 14, 1.71
    ob = 1.3 if coll in ("reg", "rr") else None
    print(f"case: q={q} {scheme} {coll} {layout} {nx}x{ny}x{nz}", flush=True)
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision=coll, omega=omega, u_lid=0.05, layout=layout,
                      omega_bulk=ob)
    ref = O.Simulation(oracle_cfg(q, nx, ny, nz, coll, omega, (0.05, 0, 0), omega_bulk=ob), "ref")
    for n in (21, 1):   # odd, then even step count (AA phase read-out both ways)
        sim.step(n)
        ref.step(n)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, n


@pytest.mark.parametrize("q", (19, 27))
@pytest.mark.parametrize("geometry", ("periodic", "channel"))
@pytest.mark.parametrize("scheme", SCHEMES)
def test_wrapping_geometries_from_a_velocity_field(lbm, q, geometry, scheme):
    nx, ny, nz = 9, 8, 11
    u0 = W.random_velocity(61, nx * ny * nz, amp=0.04).T.copy()
    rho0 = W.random_density(62, nx * ny * nz, 0.98, 1.02)
    print(f"case: q={q} {geometry} {scheme}", flush=True)
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision="trt", omega=1.4, geometry=geometry,
                      lid_velocity=(0.03, -0.01, 0.0))
    sim.init_equilibrium(torch.from_numpy(rho0), torch.from_numpy(u0))
    cfg = oracle_cfg(q, nx, ny, nz, "trt", 1.4, (0.03, -0.01, 0.0), geometry=geometry)
    ref = O.Simulation(cfg, "ref", rho=rho0, u=u0)
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= 1e-15
    sim.step(13)
    ref.step(13)
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL


@pytest.mark.parametrize("layout", ("soa", "aos", "blocked"))
@pytest.mark.parametrize("scheme", ("aa", "2pop_pull"))
@pytest.mark.parametrize("q", (19, 27))
def test_periodic_z_faces_on_the_fast_path(lbm, q, scheme, layout):
    """Periodic boxes: z-face cells whose x and y lie inside the box take
    the fast AA odd / pull kernels with a per-lane +-nz index correction
    (eager steps). nz = 3 is the smallest box with such cells; nz = 70 puts
    row ends inside waves."""
    for n3 in ((7, 6, 3), (6, 5, 70)):
        nx, ny, nz = n3
        print(f"case: periodic z faces q={q} {scheme} {layout} {nx}x{ny}x{nz}", flush=True)
        u0 = W.random_velocity(67, nx * ny * nz, amp=0.04).T.copy()
        sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision="trt", omega=1.6, geometry="periodic",
                          layout=layout)
        sim.init_equilibrium(None, torch.from_numpy(u0))
        ref = O.Simulation(oracle_cfg(q, nx, ny, nz, "trt", 1.6, geometry="periodic"), "ref", u=u0)
        for n in (5, 1):   # odd, then even step count
            sim.step(n)
            ref.step(n)
            assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, (n3, n)


@pytest.mark.parametrize("q", (19, 27))
def test_rr_equilibrium_initialisation(lbm, q):
    n = 7
    u0 = W.random_velocity(63, n ** 3, amp=0.05).T.copy()
    sim = lbm.Lattice(q, n, scheme="aa", collision="rr", omega=1.9, geometry="periodic")
    sim.init_equilibrium(None, torch.from_numpy(u0))
    ref = O.Simulation(oracle_cfg(q, n, n, n, "rr", 1.9, geometry="periodic"), "ref", u=u0)
    assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= 1e-15


def test_flags_and_neighbour_indices_bit_exact(lbm):
    for geometry, dims in (("cavity", (9, 7, 11)), ("periodic", (5, 6, 7)), ("channel", (6, 5, 8))):
        for q in (19, 27):
            sim = lbm.Lattice(q, *dims, geometry=geometry)
            cfg = oracle_cfg(q, *dims, "bgk", 1.0, geometry=geometry)
            assert np.array_equal(sim.flags().cpu().numpy(), O.flags(cfg))
            n = dims[0] * dims[1] * dims[2]
            cells = np.arange(n)
            fl = O.flags(cfg)
            got = sim.neighbor_index(cells).cpu().numpy()
            for i in cells:
                if fl[i] != O.FLUID and geometry == "cavity":
                    continue   # wall cells never stream; their neighbours may lie outside the box
                for k in range(q):
                    assert got[i, k] == O.neighbour_index(cfg, int(i), k), (geometry, q, i, k)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dtype", ("f64", "f32"))
def test_checkpoint_round_trip_is_bit_exact(lbm, scheme, dtype):
    """51 steps, save, destroy, create, restore, 49 steps == 100 steps."""
    kw = dict(scheme=scheme, collision="trt", omega=1.8, u_lid=0.04, dtype=dtype)
    a = lbm.Lattice(19, 13, 11, 12, **kw)
    a.step(100)
    want = a.populations().cpu()
    b = lbm.Lattice(19, 13, 11, 12, **kw)
    b.step(51)
    saved = b.populations().cpu()
    b.close()
    c = lbm.Lattice(19, 13, 11, 12, **kw)
    c.set_populations(saved)
    c.step(49)
    assert torch.equal(c.populations().cpu(), want)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_invariants_match_oracle(lbm, scheme):
    sim = lbm.Lattice(19, 16, 14, 15, scheme=scheme, collision="bgk", omega=1.6, u_lid=0.06)
    ref = O.Simulation(oracle_cfg(19, 16, 14, 15, "bgk", 1.6, (0.06, 0, 0)), "ref")
    m0, _ = sim.invariants()
    sim.step(31)
    ref.step(31)
    m, e = sim.invariants()
    rm, re_ = ref.invariants()
    assert abs(m - rm) <= 1e-12 * rm
    assert abs(e - re_) <= 1e-10 * re_
    assert abs(m - m0) <= 1e-12 * m0    # closed cavity conserves mass


def test_monitor_reports_non_finite_step(lbm):
    """A NaN planted from the host is caught by the invariant monitor at the
    first check after it appears; the kernels themselves run normally."""
    sim = lbm.Lattice(19, 10, scheme="aa", collision="bgk", omega=1.2, check_every=4)
    sim.step(4)
    f = sim.populations().cpu()
    f[3, 5 * 100 + 5 * 10 + 5] = float("nan")
    sim.set_populations(f)
    sim.step(3)
    with pytest.raises(lbm.LBMError) as e:
        sim.step(2)
    assert e.value.code == lbm.ENONFINITE
    assert sim.info().first_nonfinite == 4


def test_host_pointer_path_and_library_buffers(lbm):
    """lbm_create_ex with library-owned buffers, the null stream and host pointers."""
    import ctypes
    L = lbm.lib()
    d = lbm.Desc()
    L.lbm_desc_default(ctypes.byref(d))
    d.nx, d.ny, d.nz, d.scheme, d.collision, d.omega = 10, 9, 11, 0, 1, 1.5
    d.lid_velocity[0] = 0.05
    d.ptr_kind = 1
    h = L.lbm_create_ex(ctypes.byref(d))
    assert h, lbm.last_error()
    try:
        assert L.lbm_step(h, 9) == 0
        f = np.zeros((19, 990))
        assert L.lbm_get_populations(h, f.ctypes.data) == 0
        ref = O.Simulation(oracle_cfg(19, 10, 9, 11, "trt", 1.5, (0.05, 0, 0)), "ref")
        ref.step(9)
        assert max_err(f, ref.populations()) <= TOL
        rho, u = np.zeros(990), np.zeros((3, 990))
        assert L.lbm_macroscopic(h, rho.ctypes.data, u.ctypes.data) == 0
        rr, ur = ref.macroscopic()
        assert max_err(rho, rr) <= TOL and max_err(u, ur) <= TOL
        cells = np.array([0, 5, 989, 990], np.int64)
        out = np.zeros((4, 19), np.int64)
        assert L.lbm_neighbor_index(h, cells.ctypes.data, 4, out.ctypes.data) == lbm.EINVAL
    finally:
        L.lbm_destroy(h)


def relative_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("dtype,bound", [("f32", 1e-5), ("f16", 1e-3)])
def test_shifted_storage_taylor_green(lbm, dtype, bound):
    """Shifted storage g = f - t_k with FP32 arithmetic vs the FP64 oracle:
    velocity relative L2 on a periodic Taylor-Green vortex (u0 = 0.04)."""
    n, steps, omega = 32, 200, W.omega_from_nu(0.01)
    u0 = W.taylor_green_velocity(n, n, n, W.TGV_U0)
    sim = lbm.Lattice(19, n, scheme="aa", collision="bgk", omega=omega, geometry="periodic", dtype=dtype)
    sim.init_equilibrium(None, torch.from_numpy(u0))
    ref = O.Simulation(oracle_cfg(19, n, n, n, "bgk", omega, geometry="periodic"), "2pop", u=u0)
    sim.step(steps)
    ref.step(steps)
    _, u = sim.macroscopic()
    _, ur = ref.macroscopic()
    err = relative_l2(u.cpu().numpy(), ur)
    print(f"{dtype}: velocity rel L2 = {err:.3e}", flush=True)
    assert err <= bound


@pytest.mark.parametrize("dtype,bound", [("f32", 1e-5), ("f16", 1e-3)])
def test_shifted_storage_cavity(lbm, dtype, bound):
    cav = W.CAVITY_SMALL
    sim = lbm.Lattice(19, cav.n, scheme="aa", collision="bgk", omega=cav.omega, u_lid=cav.u_lid, dtype=dtype)
    ref = O.Simulation(oracle_cfg(19, cav.n, cav.n, cav.n, "bgk", cav.omega, (cav.u_lid, 0, 0)), "2pop")
    sim.step(100)
    ref.step(100)
    _, u = sim.macroscopic()
    _, ur = ref.macroscopic()
    err = relative_l2(u.cpu().numpy(), ur)
    print(f"{dtype}: cavity velocity rel L2 = {err:.3e}", flush=True)
    assert err <= bound


@pytest.mark.parametrize("q,coll", [(19, "bgk"), (19, "trt"), (19, "reg"), (27, "rr")])
@pytest.mark.parametrize("dtype", ("f64", "f32"))
def test_gpu_schemes_and_layouts_agree_bit_exactly(lbm, q, coll, dtype):
    """The six strategies (three schemes x two layouts) produce identical
    results (Sec. 2.3) on the GPU too: the collision is the same arithmetic
    in every kernel, streaming only moves values."""
    base = None
    for layout in ("soa", "aos", "blocked"):
        for scheme in SCHEMES:
            sim = lbm.Lattice(q, 11, 9, 13, scheme=scheme, collision=coll, omega=1.83, u_lid=0.05,
                              layout=layout, dtype=dtype)
            sim.step(17)
            f = sim.populations().cpu()
            if base is None:
                base = f
            else:
                assert torch.equal(f, base), (layout, scheme)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q,layout", [(19, "soa"), (19, "aos"), (27, "soa"), (19, "blocked")])
def test_captured_step_graphs_match_oracle(lbm, scheme, q, layout):
    """Small lattices replay steps from a captured HIP graph (64 steps, one
    fused kernel per kind on D3Q19 SoA). Odd eager steps in between move the
    AA phase and the 2Pop buffers, which forces a fresh capture."""
    nx, ny, nz, omega = 12, 10, 14, 1.71
    print(f"case: graph q={q} {scheme} {layout}", flush=True)
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision="trt", omega=omega, u_lid=0.05, layout=layout)
    ref = O.Simulation(oracle_cfg(q, nx, ny, nz, "trt", omega, (0.05, 0, 0)), "ref")
    for n in (130, 1, 64, 3):
        sim.step(n)
        ref.step(n)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, n


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("q,dims,geometry", [
    (19, (3, 3, 3), "cavity"),        # one fluid cell, every neighbour a wall
    (27, (3, 4, 3), "cavity"),        # a line of two fluid cells
    (19, (1, 1, 1), "periodic"),      # one cell whose neighbours are all itself
    (27, (1, 1, 1), "periodic"),
    (19, (7, 1, 5), "periodic"),      # one-cell-thick periodic axis
    (19, (5, 4, 3), "channel"),       # a single fluid layer between the walls
])
def test_degenerate_lattices_match_oracle(lbm, scheme, q, dims, geometry):
    nx, ny, nz = dims
    print(f"case: degenerate q={q} {dims} {geometry} {scheme}", flush=True)
    u0 = W.random_velocity(67, nx * ny * nz, amp=0.04).T.copy()
    sim = lbm.Lattice(q, nx, ny, nz, scheme=scheme, collision="trt", omega=1.6, u_lid=0.05, geometry=geometry)
    cfg = oracle_cfg(q, nx, ny, nz, "trt", 1.6, (0.05, 0, 0), geometry=geometry)
    fl = O.flags(cfg)
    u0[:, fl != O.FLUID] = 0.0
    sim.init_equilibrium(None, torch.from_numpy(u0))
    ref = O.Simulation(cfg, "ref", u=u0)
    for n in (0, 9, 1):
        sim.step(n)
        ref.step(n)
        assert max_err(sim.populations().cpu().numpy(), ref.populations()) <= TOL, n
    m, e = sim.invariants()
    mr, er = ref.invariants()
    assert abs(m - mr) <= 1e-12 * max(mr, 1.0)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_lattice_without_fluid_cells(lbm, scheme):
    """A geometry of walls only: steps change nothing, invariants are zero."""
    n = 6
    sim = lbm.Lattice(19, n, scheme=scheme, collision="bgk", omega=1.5, u_lid=0.05)
    cfg = oracle_cfg(19, n, n, n, "bgk", 1.5, (0.05, 0, 0))
    wall = np.full(n ** 3, O.WALL, np.uint8)
    sim.set_geometry(torch.from_numpy(wall))
    assert sim.info().fluid_cells == 0
    before = sim.populations().cpu()
    sim.step(5)
    assert torch.equal(sim.populations().cpu(), before)
    assert sim.invariants() == (0.0, 0.0)
    rho, u = sim.macroscopic()
    assert float(rho.abs().max()) == 0.0 and float(u.abs().max()) == 0.0


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dims", [(110, 100, 96), (12, 10, 14)])
def test_reverse_traversal_order_is_bit_identical(lbm, scheme, dims, monkeypatch):
    """Race check on the GPU (Sec. 2.3: each scheme is independent of the
    order in which cells are visited): the step kernels run their blocks and
    edge-cell lists backwards and must produce identical populations. The
    large box takes the fast + edge-cell kernels, the small one the captured
    graph of fused kernels."""
    nx, ny, nz = dims
    out = []
    for rev in (False, True):
        if rev:
            monkeypatch.setenv("LBM_REVERSE_BLOCKS", "1")
        else:
            monkeypatch.delenv("LBM_REVERSE_BLOCKS", raising=False)
        sim = lbm.Lattice(19, nx, ny, nz, scheme=scheme, collision="trt", omega=1.8, u_lid=0.05)
        sim.step(130 if nx < 20 else 9)
        out.append(sim.populations().cpu())
        sim.close()
    monkeypatch.delenv("LBM_REVERSE_BLOCKS", raising=False)
    assert torch.equal(out[0], out[1])


def test_divergence_is_caught_and_resume_reproduces_it(lbm):
    """BGK at omega = 1.999 with a fast lid (0.3) blows up within a few hundred
    steps. The monitor (every 10 steps) reports the first check that sees a
    non-finite mass or energy; restoring the last good checkpoint into a new
    handle and stepping again reproduces the same trajectory bit for bit."""
    kw = dict(scheme="aa", collision="bgk", omega=1.999, u_lid=0.3)
    a = lbm.Lattice(19, 16, check_every=10, **kw)
    saved, step = None, 0
    with pytest.raises(lbm.LBMError) as e:
        for _ in range(200):
            saved = a.populations().cpu()
            a.step(10)
            step += 10
    assert e.value.code == lbm.ENONFINITE
    bad = a.info().first_nonfinite
    assert bad == step + 10 and 50 <= bad <= 1000
    b = lbm.Lattice(19, 16, check_every=10, **kw)
    b.set_populations(saved)
    with pytest.raises(lbm.LBMError):
        b.step(10)
    c = lbm.Lattice(19, 16, **kw)
    c.set_populations(saved)
    c.step(10)
    as_bits = lambda t: t.view(torch.int64)
    assert torch.equal(as_bits(b.populations().cpu()), as_bits(c.populations().cpu()))
    assert torch.equal(as_bits(a.populations().cpu()), as_bits(c.populations().cpu()))


@pytest.mark.parametrize("ns", (19, 27))
def test_stream_copy_probe(lbm, ns):
    """The bandwidth probe copies exactly the n values of each stream."""
    n, stride = 3001, 3072
    src = torch.randn(ns * stride, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    lbm.stream_copy(dst, src, ns, n, stride, 46080)
    torch.cuda.synchronize()
    s, d = src.view(ns, stride).cpu(), dst.view(ns, stride).cpu()
    assert torch.equal(d[:, :n], s[:, :n])
    assert float(d[:, n:].abs().max()) == 0.0
    big = torch.zeros(20 * stride, dtype=torch.float64, device="cuda")
    with pytest.raises(lbm.LBMError):      # the library takes 19 or 27 streams only
        lbm.stream_copy(big, big.clone(), 20, n, stride)
    # shifted (AA odd) pattern: stream s read at i - d_s, written at i + d_s
    ny, nz = 4, 5
    halo = ny * nz + nz + 1
    src = torch.randn(ns * stride + 2 * halo, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    lbm.stream_copy(dst, src, ns, n, stride, 0, shift=(ny, nz))
    c, _, _ = O.lattice(ns)
    s_, d_ = src.cpu().numpy(), dst.cpu().numpy()
    i = np.arange(n)
    for k in range(ns):
        off = (int(c[k, 0]) * ny + int(c[k, 1])) * nz + int(c[k, 2])
        assert np.array_equal(d_[halo + k * stride + i + off], s_[halo + k * stride + i - off]), k


@pytest.mark.parametrize("block_log2", (0, 8, 12))
@pytest.mark.parametrize("pattern", (0, 1, 2))
@pytest.mark.parametrize("vec", (1, 2))
def test_pattern_copy_probe(lbm, block_log2, pattern, vec):
    """The memory-pattern probe moves each of the 19 streams as documented:
    value (s, j) at s * stride + j (SoA) or ((j >> b) * 19 + s) * 2^b + (j mod
    2^b) (blocked); read at i (- d_s for patterns 1 and 2), written at i
    (+ d_s for pattern 2)."""
    if block_log2 and vec == 2:
        pytest.skip("two values per lane: SoA only")
    ny, nz = 6, 5
    n = 8192 if block_log2 else 3000
    stride = 3072
    shift = (ny, nz)
    halo = lbm.pattern_halo(block_log2, shift if pattern else None)
    span = 19 * (n if block_log2 else stride)
    src = torch.randn(span + 2 * halo, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    lbm.pattern_copy(dst, src, n, stride, block_log2, pattern, vec, 0, shift)
    torch.cuda.synchronize()
    s_, d_ = src.cpu().numpy(), dst.cpu().numpy()
    c, _, _ = O.lattice(19)

    def at(j, k):
        if block_log2 == 0:
            return halo + k * stride + j
        b = 1 << block_log2
        return halo + ((j // b) * 19 + k) * b + j % b
    i = np.arange(n)
    written = np.zeros(d_.size, bool)
    for k in range(19):
        d = (int(c[k, 0]) * ny + int(c[k, 1])) * nz + int(c[k, 2])
        r = i - d if pattern else i
        w = i + d if pattern == 2 else i
        assert np.array_equal(d_[at(w, k)], s_[at(r, k)]), k
        written[at(w, k)] = True
    assert float(np.abs(d_[~written]).max(initial=0.0)) == 0.0   # nothing else is written
