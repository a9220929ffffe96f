"""Thin ctypes binding of ``liblbm.so`` (C ABI in ``include/lbm.h``).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch supplies device memory (population, flag and output buffers are
torch tensors handed to the library as caller-owned buffers) and the stream
(the handle runs on ``torch.cuda.current_stream()`` at creation). The
library must have been built (``python -m paper_2010_11751_amd.build``);
importing this module on a machine without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch  # loads the HIP runtime the library then binds to

HERE = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY may name another build of the same library (tuning variants).
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(HERE, "liblbm.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SCHEMES = {"2pop": 0, "swap": 1, "aa": 2, "2pop_pull": 3}
COLLISIONS = {"bgk": 0, "trt": 1, "reg": 2, "rr": 3,
              "nw4": 4, "rm": 5, "hm": 6, "cm": 7, "chm": 8, "k": 9}
DTYPES = {"f64": 0, "f32": 1, "f16": 2}
LAYOUTS = {"soa": 0, "aos": 1, "blocked": 2}
GEOMETRIES = {"cavity": 0, "periodic": 1, "channel": 2}
FLUID, WALL, LID, PRESSURE = 0, 1, 2, 3


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("scheme", ctypes.c_int), ("collision", ctypes.c_int), ("storage_dtype", ctypes.c_int),
                ("layout", ctypes.c_int), ("geometry", ctypes.c_int), ("ptr_kind", ctypes.c_int),
                ("check_every", ctypes.c_int), ("block_size", ctypes.c_int),
                ("omega", ctypes.c_double), ("trt_lambda", ctypes.c_double), ("omega_bulk", ctypes.c_double),
                ("omega3", ctypes.c_double), ("omega4", ctypes.c_double),
                ("lid_velocity", ctypes.c_double * 3), ("stream", ctypes.c_void_p),
                ("pop", ctypes.c_void_p), ("out", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("pop_bytes", ctypes.c_size_t), ("out_bytes", ctypes.c_size_t), ("flags_bytes", ctypes.c_size_t)]


class Info(ctypes.Structure):
    _fields_ = [("ntot", ctypes.c_int64), ("fluid_cells", ctypes.c_int64), ("pop_stride", ctypes.c_int64),
                ("steps_done", ctypes.c_int64), ("first_nonfinite", ctypes.c_int64),
                ("bytes_per_update", ctypes.c_int64), ("aa_phase", ctypes.c_int), ("block_size", ctypes.c_int)]


class CavityDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("omega", ctypes.c_double), ("u_lid", ctypes.c_double), ("trt_lambda", ctypes.c_double)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int), ("graph_steps", ctypes.c_int), ("autotune", ctypes.c_int),
                ("block_size", ctypes.c_int), ("stream", ctypes.c_void_p), ("autotune_cache", ctypes.c_char_p),
                ("cells_per_thread", ctypes.c_int), ("waves_per_simd", ctypes.c_int), ("xcd_split", ctypes.c_int)]


SYMBOLS = [
    "lbm_desc_default", "lbm_required_bytes", "lbm_create", "lbm_create_ex", "lbm_destroy",
    "lbm_init_equilibrium", "lbm_set_geometry", "lbm_set_wall_distances", "lbm_step", "lbm_macroscopic", "lbm_get_populations", "lbm_get_populations_at",
    "lbm_set_populations",
    "lbm_get_flags", "lbm_invariants", "lbm_invariants_noalloc", "lbm_neighbor_index", "lbm_get_info", "lbm_lattice", "lbm_device_copy",
    "lbm_sync", "lbm_stream_copy", "lbm_pattern_copy",
    "lbm_last_error", "lbm_batch_create", "lbm_batch_step", "lbm_batch_step_sequential",
    "lbm_batch_macroscopic", "lbm_batch_get_populations", "lbm_batch_invariants", "lbm_batch_info",
    "lbm_batch_launch_shape",
    "lbm_batch_sync", "lbm_batch_destroy",
]

_lib = None


def lib() -> ctypes.CDLL:
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_11751_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.lbm_desc_default.argtypes = [ctypes.POINTER(Desc)]
    L.lbm_desc_default.restype = None
    L.lbm_required_bytes.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)]
    L.lbm_create.argtypes = [I, I, I, I, I, I, D, D, I]
    L.lbm_create.restype = P
    L.lbm_create_ex.argtypes = [ctypes.POINTER(Desc)]
    L.lbm_create_ex.restype = P
    L.lbm_destroy.argtypes = [P]
    L.lbm_destroy.restype = None
    L.lbm_init_equilibrium.argtypes = [P, P, P]
    L.lbm_set_geometry.argtypes = [P, P, P, P]
    L.lbm_set_wall_distances.argtypes = [P, P]
    L.lbm_step.argtypes = [P, I]
    L.lbm_macroscopic.argtypes = [P, P, P]
    L.lbm_get_populations.argtypes = [P, P]
    L.lbm_get_populations_at.argtypes = [P, P, I, P]
    L.lbm_set_populations.argtypes = [P, P]
    L.lbm_get_flags.argtypes = [P, P]
    L.lbm_invariants.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D)]
    L.lbm_invariants_noalloc.argtypes = [P, P]
    L.lbm_neighbor_index.argtypes = [P, P, I, P]
    L.lbm_get_info.argtypes = [P, ctypes.POINTER(Info)]
    L.lbm_lattice.argtypes = [I, P, P, P]
    L.lbm_sync.argtypes = [P]
    L.lbm_device_copy.argtypes = [P, P, ctypes.c_size_t, P]
    L.lbm_stream_copy.argtypes = [P, P, I, ctypes.c_size_t, ctypes.c_size_t, I, I, I, P]
    L.lbm_pattern_copy.argtypes = [P, P, ctypes.c_size_t, ctypes.c_size_t, I, I, I, I, I, I, P]
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = ctypes.c_char_p
    L.lbm_batch_create.argtypes = [I, ctypes.POINTER(CavityDesc), I, I, I, ctypes.POINTER(BatchOpts)]
    L.lbm_batch_create.restype = P
    L.lbm_batch_step.argtypes = [P, I]
    L.lbm_batch_step_sequential.argtypes = [P, I]
    L.lbm_batch_macroscopic.argtypes = [P, I, P, P]
    L.lbm_batch_get_populations.argtypes = [P, I, P]
    L.lbm_batch_invariants.argtypes = [P, P, P]
    L.lbm_batch_info.argtypes = [P, P, P, P]
    L.lbm_batch_launch_shape.argtypes = [P, P, P, P, P, P]
    L.lbm_batch_sync.argtypes = [P]
    L.lbm_batch_destroy.argtypes = [P]
    L.lbm_batch_destroy.restype = None
    _lib = L
    return L


def last_error() -> str:
    return lib().lbm_last_error().decode()


def check(rc: int) -> int:
    if rc != OK:
        raise LBMError(rc, last_error())
    return rc


def lattice(q: int):
    """(c[q][3], t[q], opp[q]) as the kernels use them (no device needed)."""
    import numpy as np
    c = np.zeros((q, 3), np.int32)
    t = np.zeros(q)
    opp = np.zeros(q, np.int32)
    check(lib().lbm_lattice(q, c.ctypes.data, t.ctypes.data, opp.ctypes.data))
    return c, t, opp


def stream_copy(dst: torch.Tensor, src: torch.Tensor, nstreams: int, n: int, stride: int, lds_bytes: int = 0,
                shift=None) -> None:
    """Copy nstreams FP64 streams of n values (stream s at element s * stride)
    from src to dst with the library's multi-stream kernel on the current
    stream (the step kernels' memory pattern without arithmetic). With
    shift = (ny, nz) stream s is read at i - d_s and written at i + d_s (the AA
    odd step's pattern); the tensors then start ny*nz + nz + 1 values before
    element 0 and end as far after the last stream."""
    ny, nz = (0, 0) if shift is None else shift
    halo = ny * nz + nz + 1 if shift is not None else 0
    for t in (dst, src):
        if t.dtype != torch.float64 or t.numel() < (nstreams - 1) * stride + n + 2 * halo:
            raise ValueError("float64 tensors of at least (nstreams - 1) * stride + n (+ 2 halo) values needed")
    off = halo * 8
    check(lib().lbm_stream_copy(ctypes.c_void_p(dst.data_ptr() + off), ctypes.c_void_p(src.data_ptr() + off),
                                nstreams, n, stride, lds_bytes, ny, nz,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


def pattern_halo(block_log2: int, shift) -> int:
    """Values the pattern-copy buffers extend before value (0, 0) and after
    the last value."""
    if shift is None:
        return 0
    h = shift[0] * shift[1] + shift[1] + 1
    if block_log2 == 0:
        return h
    b = 1 << block_log2
    return -(-h // b) * 19 * b


def pattern_copy(dst: torch.Tensor, src: torch.Tensor, n: int, stride: int, block_log2: int = 0, pattern: int = 0,
                 vec: int = 1, lds_bytes: int = 0, shift=None) -> None:
    """The library's memory-pattern probe over 19 FP64 streams on the current
    stream: SoA (block_log2 0, stream s at s * stride) or blocks of 2^8 / 2^12
    cells; pattern 0 local, 1 pull (read i - d_s), 2 AA odd (read i - d_s,
    write i + d_s) with d_s from shift = (ny, nz). The tensors hold the halo
    of pattern_halo() before value (0, 0) and after the last value."""
    halo = pattern_halo(block_log2, shift if pattern else None)
    span = 19 * (n if block_log2 else stride)
    for t in (dst, src):
        if t.dtype != torch.float64 or t.numel() < span + 2 * halo:
            raise ValueError("float64 tensors of the layout's size plus twice the halo needed")
    ny, nz = (0, 0) if not pattern else shift
    off = halo * 8
    check(lib().lbm_pattern_copy(ctypes.c_void_p(dst.data_ptr() + off), ctypes.c_void_p(src.data_ptr() + off), n,
                                 stride, block_log2, pattern, vec, lds_bytes, ny, nz,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


def device_copy(dst: torch.Tensor, src: torch.Tensor) -> None:
    """Copy src into dst (same byte size) with the library's streaming kernel
    on the current stream."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    check(lib().lbm_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, n, device):
    if t is None:
        return None
    t = torch.as_tensor(t, dtype=dtype, device=device).contiguous()
    if t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return t


class Lattice:
    """One simulation on one GPU, backed by the C handle.

    Buffers are torch tensors owned by this object (caller-owned from the
    library's point of view); the handle runs on the current torch stream."""

    def __init__(self, lattice: int = 19, nx: int = 8, ny: int | None = None, nz: int | None = None,
                 scheme: str = "aa", collision: str = "bgk", omega: float = 1.0, u_lid: float = 0.0,
                 dtype: str = "f64", layout: str = "soa", geometry: str = "cavity", trt_lambda: float = 0.25,
                 omega_bulk: float | None = None, lid_velocity=None, check_every: int = 0,
                 block_size: int = 0, device: int | str | torch.device = 0,
                 omega3: float | None = None, omega4: float | None = None):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        d = Desc()
        lib().lbm_desc_default(ctypes.byref(d))
        d.lattice, d.nx, d.ny, d.nz = lattice, nx, ny, nz
        d.scheme, d.collision = SCHEMES[scheme], COLLISIONS[collision]
        d.storage_dtype, d.layout, d.geometry = DTYPES[dtype], LAYOUTS[layout], GEOMETRIES[geometry]
        d.omega, d.trt_lambda = omega, trt_lambda
        d.omega_bulk = 0.0 if omega_bulk is None else omega_bulk
        d.omega3 = 0.0 if omega3 is None else omega3
        d.omega4 = 0.0 if omega4 is None else omega4
        lv = (u_lid, 0.0, 0.0) if lid_velocity is None else tuple(lid_velocity)
        for a in range(3):
            d.lid_velocity[a] = lv[a]
        d.check_every, d.block_size = check_every, block_size
        req = (ctypes.c_size_t * 3)()
        check(lib().lbm_required_bytes(ctypes.byref(d), req))
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self._pop = torch.empty(max(int(req[0]), 1), dtype=torch.uint8, device=self.device)
            self._out = torch.empty(int(req[1]), dtype=torch.uint8, device=self.device) if req[1] else None
            self._flags = torch.empty(max(int(req[2]), 1), dtype=torch.uint8, device=self.device)
            d.stream = self.stream.cuda_stream
            d.pop, d.out, d.flags = self._pop.data_ptr(), (self._out.data_ptr() if self._out is not None else None), \
                self._flags.data_ptr()
            d.pop_bytes, d.flags_bytes = self._pop.numel(), self._flags.numel()
            d.out_bytes = self._out.numel() if self._out is not None else 0
            h = lib().lbm_create_ex(ctypes.byref(d))
        if not h:
            raise LBMError(EINVAL, last_error())
        self.h = ctypes.c_void_p(h)
        self.q, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.ntot = nx * ny * nz
        self.scheme, self.collision, self.dtype, self.layout = scheme, collision, dtype, layout

    def close(self) -> None:
        if getattr(self, "h", None):
            lib().lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- simulation -----------------------------------------------------------
    def step(self, n: int = 1) -> None:
        check(lib().lbm_step(self.h, int(n)))

    def init_equilibrium(self, rho=None, u=None) -> None:
        r = _dev(rho, torch.float64, self.ntot, self.device)
        v = _dev(u, torch.float64, 3 * self.ntot, self.device)
        check(lib().lbm_init_equilibrium(self.h, _ptr(r), _ptr(v)))

    def set_geometry(self, cell_types, wall_velocity=None, wall_density=None) -> None:
        """Caller cell types (uint8 FLUID / WALL / LID / PRESSURE per cell) with per-cell
        wall velocity [3][Ntot] and wall density [Ntot] of the wall cells."""
        t = _dev(cell_types, torch.uint8, self.ntot, self.device)
        wu = _dev(wall_velocity, torch.float64, 3 * self.ntot, self.device)
        wr = _dev(wall_density, torch.float64, self.ntot, self.device)
        check(lib().lbm_set_geometry(self.h, _ptr(t), _ptr(wu), _ptr(wr)))

    def set_wall_distances(self, q) -> None:
        """Curved walls: q[k][Ntot], the wall's fraction of the link from each
        fluid cell x to its wall neighbour x - c_k (1/2: half-way)."""
        t = _dev(q, torch.float64, self.q * self.ntot, self.device)
        check(lib().lbm_set_wall_distances(self.h, _ptr(t)))

    def sync(self) -> None:
        check(lib().lbm_sync(self.h))

    # -- read-outs --------------------------------------------------------------
    def macroscopic(self):
        rho = torch.empty(self.ntot, dtype=torch.float64, device=self.device)
        u = torch.empty(3, self.ntot, dtype=torch.float64, device=self.device)
        check(lib().lbm_macroscopic(self.h, _ptr(rho), _ptr(u)))
        return rho, u

    def populations(self) -> torch.Tensor:
        f = torch.empty(self.q, self.ntot, dtype=torch.float64, device=self.device)
        check(lib().lbm_get_populations(self.h, _ptr(f)))
        return f

    def populations_at(self, cells) -> torch.Tensor:
        """Natural populations of the listed cells: f[j][k] (FP64)."""
        c = torch.as_tensor(cells, dtype=torch.int64, device=self.device).contiguous()
        if c.numel() and (int(c.min()) < 0 or int(c.max()) >= self.ntot):
            raise ValueError("cell index out of range")
        f = torch.empty(c.numel(), self.q, dtype=torch.float64, device=self.device)
        check(lib().lbm_get_populations_at(self.h, _ptr(c), c.numel(), _ptr(f)))
        return f

    def set_populations(self, f) -> None:
        t = _dev(f, torch.float64, self.q * self.ntot, self.device)
        check(lib().lbm_set_populations(self.h, _ptr(t)))

    def flags(self) -> torch.Tensor:
        fl = torch.empty(self.ntot, dtype=torch.uint8, device=self.device)
        check(lib().lbm_get_flags(self.h, _ptr(fl)))
        return fl

    def invariants(self):
        m, e = ctypes.c_double(), ctypes.c_double()
        check(lib().lbm_invariants(self.h, ctypes.byref(m), ctypes.byref(e)))
        return m.value, e.value

    def neighbor_index(self, cells) -> torch.Tensor:
        c = torch.as_tensor(cells, dtype=torch.int64, device=self.device).contiguous()
        if c.numel() and (int(c.min()) < 0 or int(c.max()) >= self.ntot):
            raise ValueError("cell index out of range")
        out = torch.empty(c.numel(), self.q, dtype=torch.int64, device=self.device)
        check(lib().lbm_neighbor_index(self.h, _ptr(c), c.numel(), _ptr(out)))
        return out

    def info(self) -> Info:
        i = Info()
        check(lib().lbm_get_info(self.h, ctypes.byref(i)))
        return i


@dataclass
class Cavity:
    n: int
    omega: float
    u_lid: float
    trt_lambda: float = 0.25


class Batch:
    """Ensemble of independent D3Q19 cavities advanced by one launch per step."""

    def __init__(self, cavities, scheme: str = "aa", collision: str = "trt", dtype: str = "f32",
                 use_graph: bool = True, graph_steps: int = 100, autotune: bool = False, block_size: int = 0,
                 autotune_cache=None, cells_per_thread: int = 0, waves_per_simd: int = -1, xcd_split: int = 1):
        arr = (CavityDesc * len(cavities))()
        self.sizes = []
        for j, c in enumerate(cavities):
            n = c.n
            arr[j] = CavityDesc(n, n, n, c.omega, c.u_lid, c.trt_lambda)
            self.sizes.append(n ** 3)
        self.stream = torch.cuda.current_stream()
        opts = BatchOpts(int(use_graph), graph_steps, int(autotune), block_size, self.stream.cuda_stream,
                         None if autotune_cache is None else str(autotune_cache).encode(),
                         cells_per_thread, waves_per_simd, 1 if xcd_split else 2)
        b = lib().lbm_batch_create(len(cavities), arr, SCHEMES[scheme], COLLISIONS[collision], DTYPES[dtype],
                                   ctypes.byref(opts))
        if not b:
            raise LBMError(EINVAL, last_error())
        self.b = ctypes.c_void_p(b)
        self.count = len(cavities)

    def close(self):
        if getattr(self, "b", None):
            lib().lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        check(lib().lbm_batch_step(self.b, int(n)))

    def step_sequential(self, n: int = 1):
        check(lib().lbm_batch_step_sequential(self.b, int(n)))

    def sync(self):
        check(lib().lbm_batch_sync(self.b))

    def macroscopic(self, idx: int):
        n = self.sizes[idx]
        rho = torch.empty(n, dtype=torch.float64, device="cuda")
        u = torch.empty(3, n, dtype=torch.float64, device="cuda")
        check(lib().lbm_batch_macroscopic(self.b, idx, _ptr(rho), _ptr(u)))
        return rho, u

    def populations(self, idx: int):
        f = torch.empty(19, self.sizes[idx], dtype=torch.float64, device="cuda")
        check(lib().lbm_batch_get_populations(self.b, idx, _ptr(f)))
        return f

    def invariants(self):
        import numpy as np
        m = np.zeros(self.count)
        e = np.zeros(self.count)
        check(lib().lbm_batch_invariants(self.b, m.ctypes.data, e.ctypes.data))
        return m, e

    def info(self):
        cells, fluid, blk = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        check(lib().lbm_batch_info(self.b, ctypes.byref(cells), ctypes.byref(fluid), ctypes.byref(blk)))
        return cells.value, fluid.value, blk.value

    def launch_shape(self):
        """(block size, cells per thread, residency cap, XCD split, edge
        cells) of the fast kernel in use."""
        blk, cpt, waves, xcd, edge = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        check(lib().lbm_batch_launch_shape(self.b, ctypes.byref(blk), ctypes.byref(cpt), ctypes.byref(waves),
                                           ctypes.byref(xcd), ctypes.byref(edge)))
        return blk.value, cpt.value, waves.value, xcd.value, edge.value
