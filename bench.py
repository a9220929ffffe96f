"""Benchmark of the lattice Boltzmann collide-and-stream step on one MI355X.

Workload: D3Q19 lid-driven cavity 256^3 (wall layer included; Re = 1000,
u_lid = 0.05), synthetic state at rest, populations resident in HBM. A step
is one full time step of the method (gather, decode, moments, collision,
encode, stream with bounce-back) over the whole lattice.

Headline: FP64 storage, BGK, the fastest scheme on this workload, the
two-population scheme in pull form (SoA; MLUPS over fluid cells). The same
JSON line carries the FP32-shifted run, the AA pattern (the paper's fastest
scheme) in FP64 and FP32, the twelve FP64 scheme x collision combinations,
the schemes under FP32/FP16 storage, the measured copy-kernel bandwidth, the
roofline of the dominant kernel and the CPU oracle baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-sweep] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak
HEAD_SCHEME = "2pop_pull"
HEAD_LAYOUT = "blocked"  # the 19 streams of each run of 256 cells kept together (the fastest pull layout)
KERNEL_LABEL = {"2pop_pull": "2Pop pull", "aa": "AA even/odd"}


def kernel_label(r) -> str:
    """The step kernel a headline run times (D3Q19, 256^3). On the built-in
    cavity the library takes the position-driven pull kernel (FP64: blocks of
    128 threads, three per CU) and the position-driven AA odd kernel in SoA
    and the blocked layout, where they measured faster than the flag-driven
    ones."""
    label = KERNEL_LABEL[r["scheme"]]
    if r["scheme"] == "2pop_pull" and r["layout"] in ("soa", "blocked"):
        label += ", position-driven"
    if r["scheme"] == "aa" and r["layout"] in ("soa", "blocked"):
        label += " (odd step position-driven)"
    return f"k_step<19,BGK,{r['dtype']},{LAYOUT_NAME[r['layout']]},{label}>"
TRAFFIC_KEY = {"2pop_pull": "pull", "aa": "aa"}
LAYOUT_NAME = {"soa": "SoA", "aos": "AoS", "blocked": "blocked"}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2010_11751_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def traffic_key(r) -> str:
    """Key of a run in profiles/hbm_traffic.md: scheme, layout (SoA unnamed), collision, storage, size."""
    lay = "" if r.get("layout", "soa") == "soa" else "_" + r["layout"]
    return f"{TRAFFIC_KEY[r['scheme']]}{lay}_bgk_{r['dtype']}_256"


def stored_traffic(key: str):
    """HBM bytes per launch measured with rocprofv3 counters, if recorded for
    the current kernel sources (profiles/hbm_traffic.md)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    src = kernel_source_hash()
    for line in open(path):
        m = re.match(r"\|\s*" + re.escape(key) + r"\s*\|\s*([0-9a-f]+)\s*\|\s*([0-9.eE+]+)\s*\|", line)
        if m and m.group(1) == src:
            return float(m.group(2))
    return None


def time_steps(sim, steps: int, warmup: int):
    import torch
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall  # ms per step (events), wall seconds


def copy_ceiling_gbs(nbytes: int = 2 << 30, reps: int = 20) -> float:
    import torch
    from paper_2010_11751_amd import lbm
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    lbm.device_copy(b, a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lbm.device_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def stream_copy_ceiling(cav, reps: int = 20):
    """GB/s of the library's 19-stream FP64 copy over the 256^3 cavity's cell
    count (19 loads then 19 stores per thread, no arithmetic): the memory
    pattern of the AA-even and swap-collide kernels alone, uncapped and at two
    and three resident waves per SIMD (the step kernels' FP64 caps), and the
    AA-odd pattern (stream s read at i - d_s, written at i + d_s) at several."""
    import torch
    from paper_2010_11751_amd import lbm
    n = cav.cells
    stride = (n + 1023) // 1024 * 1024
    halo = cav.n * cav.n + cav.n + 1
    a = torch.zeros(19 * stride + 2 * halo, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for label, lds, shift in (("uncapped", 0, None), ("3_waves", 46080, None), ("2_waves", 65536, None),
                              ("odd_pattern_uncapped", 0, (cav.n, cav.n)), ("odd_pattern_4_waves", 35840, (cav.n, cav.n)),
                              ("odd_pattern_3_waves", 46080, (cav.n, cav.n)), ("odd_pattern_2_waves", 65536, (cav.n, cav.n))):
        lbm.stream_copy(b, a, 19, n, stride, lds, shift=shift)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            lbm.stream_copy(b, a, 19, n, stride, lds, shift=shift)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[label] = round(2 * 19 * n * 8 / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def pattern_probe(cav, reps: int = 20):
    """The library's memory-pattern probe on the 256^3 cavity's cell count: 19
    FP64 streams in the SoA layout of the step kernels (stride as the handle
    pads it for this size) or in blocks of 2^8 / 2^12 cells holding all 19
    streams, under the local, pull and AA-odd patterns, one or two values per
    lane, uncapped and at 4 / 3 / 2 resident waves per SIMD. GB/s of moved
    bytes (2 x 19 x 8 B per cell); the step kernels' algorithmic rates are
    over the same bytes plus one flag byte per cell."""
    import torch
    from paper_2010_11751_amd import lbm
    n = cav.cells
    stride = (n + 1023) // 1024 * 1024
    shift = (cav.n, cav.n)
    size = 19 * stride + 2 * lbm.pattern_halo(12, shift)
    a = torch.zeros(size, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    caps = {"uncapped": 0, "4_waves": 35840, "3_waves": 46080, "2_waves": 65536}
    rows = []
    for layout in (0, 8, 12):
        for pattern in (0, 1, 2):
            for vec in ((1, 2) if layout == 0 else (1,)):
                for cap, lds in caps.items():
                    def go():
                        lbm.pattern_copy(b, a, n, stride, layout, pattern, vec, lds, shift)
                    go()
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        go()
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    rows.append({"layout": "soa" if layout == 0 else f"blocks_of_{1 << layout}",
                                 "pattern": ("local", "pull", "aa_odd")[pattern], "values_per_lane": vec,
                                 "residency": cap, "ms": round(ms, 4),
                                 "gbs": round(2 * 19 * n * 8 / (ms * 1e-3) / 1e9, 1)})
                    print(f"# probe {rows[-1]}", file=sys.stderr, flush=True)
    del a, b
    torch.cuda.empty_cache()
    return rows


def mall_probe(reps: int = 20):
    """The step kernels' memory patterns on footprints around the 256 MB
    last-level cache (MALL): 19 FP64 streams of N^3 values (SoA), the local
    pattern in place in one array (the AA even step), the local and pull
    patterns between two arrays (2Pop), for N = 64 .. 256. GB/s of moved
    bytes, 2 x 19 x 8 B per cell."""
    import torch
    from paper_2010_11751_amd import lbm
    rows = []
    for n3 in (64, 80, 96, 112, 128, 144, 160, 192, 256):
        n = n3 ** 3
        stride = (n + 1023) // 1024 * 1024
        shift = (n3, n3)
        size = 19 * stride + 2 * lbm.pattern_halo(0, shift)
        a = torch.zeros(size, dtype=torch.float64, device="cuda")
        b = torch.zeros_like(a)
        for label, dst, pattern in (("one_array_local", a, 0), ("two_arrays_local", b, 0), ("two_arrays_pull", b, 1)):
            def go():
                lbm.pattern_copy(dst, a, n, stride, 0, pattern, 1, 65536, shift)
            go()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                go()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            arrays = 1 if dst is a else 2
            rows.append({"n": n3, "pattern": label, "footprint_mb": round(arrays * 19 * 8 * n / 2 ** 20, 1),
                         "gbs": round(2 * 19 * 8 * n / (ms * 1e-3) / 1e9, 1)})
            print(f"# mall probe {rows[-1]}", file=sys.stderr, flush=True)
        del a, b
        torch.cuda.empty_cache()
    return rows


def run_case(scheme, coll, dtype, steps, warmup, cav, reps=1, layout="soa"):
    """One handle; `reps` timed runs of `steps` steps each (the first after
    `warmup` untimed steps); the median run is reported."""
    from paper_2010_11751_amd import lbm
    sim = lbm.Lattice(19, cav.n, scheme=scheme, collision=coll, omega=cav.omega, u_lid=cav.u_lid, dtype=dtype,
                      layout=layout)
    info = sim.info()
    runs = [time_steps(sim, steps, warmup if r == 0 else 0) for r in range(reps)]
    ms, wall = sorted(runs)[len(runs) // 2]
    m, e = sim.invariants()
    sim.close()
    fluid = info.fluid_cells
    launches = 2 if scheme == "swap" else 1
    return {
        "scheme": scheme, "collision": coll, "dtype": dtype, "layout": layout,
        "ms_per_step": ms, "wall_s": wall,
        "mlups": fluid / (ms * 1e-3) / 1e6,
        "mlups_all_cells": info.ntot / (ms * 1e-3) / 1e6,
        "bytes_per_update": info.bytes_per_update,
        "algorithmic_gbs": fluid * info.bytes_per_update / (ms * 1e-3) / 1e9,
        "kernel_avg_ms": ms / launches,
        "fluid_cells": fluid,
        "finite": bool(m == m and e == e),
        "block_size": info.block_size,
        "runs_ms_per_step": [round(r[0], 5) for r in runs],
    }


def run_d3q27_rr(steps, warmup, scheme="aa", layout="soa"):
    """512^3 D3Q27 cavity, recursive regularized, FP32-shifted (Re 5000); the
    workload names the AA pattern, and 2Pop pull runs beside it."""
    from paper_2010_11751_amd import lbm, workloads as W
    cav = W.CAVITY_512
    sim = lbm.Lattice(27, cav.n, scheme=scheme, collision="rr", omega=cav.omega, u_lid=cav.u_lid, dtype="f32",
                      layout=layout)
    info = sim.info()
    ms, _ = time_steps(sim, steps, warmup)
    m, e = sim.invariants()
    sim.close()
    gbs = info.fluid_cells * info.bytes_per_update / (ms * 1e-3) / 1e9
    return {"workload": f"D3Q27 lid-driven cavity 512^3, RR, FP32-shifted {scheme} {LAYOUT_NAME[layout]}, Re=5000, "
                        "u_lid=0.05",
            "scheme": scheme,
            "mlups": round(info.fluid_cells / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "bytes_per_update": info.bytes_per_update, "hbm_gbs": round(gbs, 1),
            "roofline_frac": round(gbs / PEAK_HBM_GBS, 4), "steps": steps, "finite": bool(m == m and e == e)}


def run_taylor_green(steps, scheme, layout="soa"):
    """256^3 periodic Taylor-Green vortex (u0 = 0.04, nu = 0.01), BGK under
    one scheme and layout, FP64 vs FP32- and FP16-shifted storage: MLUPS,
    velocity relative L2 against the FP64 run, and the decay of the (k,k,k)
    mode against exp(-3 nu k^2 t)."""
    import math
    import torch
    from paper_2010_11751_amd import lbm, workloads as W
    n = W.TGV_N
    omega = W.omega_from_nu(W.TGV_NU)
    u0 = torch.from_numpy(W.taylor_green_velocity(n, n, n, W.TGV_U0))
    mode = u0[0].to("cuda")
    out, ref = {}, None
    for dtype in ("f64", "f32", "f16"):
        sim = lbm.Lattice(19, n, scheme=scheme, collision="bgk", omega=omega, geometry="periodic", dtype=dtype,
                          layout=layout)
        sim.init_equilibrium(None, u0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        _, u = sim.macroscopic()
        info = sim.info()
        sim.close()
        # projection of u_x on the initial field: the mode's amplitude relative to t = 0
        amp = float((u[0] * mode).sum() / (mode * mode).sum())
        r = {"mlups": round(info.ntot / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
             "hbm_gbs": round(info.ntot * info.bytes_per_update / (ms * 1e-3) / 1e9, 1),
             "mode_amplitude_ratio": amp}
        if ref is None:
            ref = u
        else:
            r["velocity_rel_l2_vs_f64"] = float(torch.linalg.vector_norm(u - ref) / torch.linalg.vector_norm(ref))
        out[dtype] = r
    k = 2 * math.pi / n
    return {"workload": f"D3Q19 BGK triply periodic Taylor-Green 256^3, u0=0.04, nu=0.01, {scheme} "
                        f"{LAYOUT_NAME[layout]}",
            "scheme": scheme, "steps": steps, "analytic_exp_minus_3nuk2t": math.exp(-3 * W.TGV_NU * k * k * steps), **out}


def run_ensemble(steps, seq_steps, scheme="aa", warmup=100):
    """512 independent D3Q19 TRT cavities (edge U{16..64}, Re U[100,1000],
    u_lid 0.03), FP32-shifted storage under one scheme: one step is one fast
    kernel over the (cavity, tile) table plus the edge-cell kernel on a second
    stream, replayed from a HIP graph with the autotuned launch shape, vs one
    launch per cavity per step. Timed with events on the batch's stream."""
    import torch
    from paper_2010_11751_amd import lbm, workloads as W
    members = W.ensemble(512)
    cav = [lbm.Cavity(m.n, m.omega, m.u_lid) for m in members]
    res = {}
    stream = torch.cuda.Stream()  # the batch runs on this stream (the null stream would get a private one)
    for mode in ("graph", "sequential"):
        with torch.cuda.stream(stream):
            b = lbm.Batch(cav, scheme=scheme, collision="trt", dtype="f32", use_graph=(mode == "graph"),
                          graph_steps=100, autotune=(mode == "graph"))
        cells, fluid, blk = b.info()
        shape = b.launch_shape()
        n = steps if mode == "graph" else seq_steps
        run = b.step if mode == "graph" else b.step_sequential
        run(warmup if mode == "graph" else 2)
        b.sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        run(n)
        e1.record(stream)
        b.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1) / n
        masses, _ = b.invariants()
        gbs = fluid * 153 / (ms * 1e-3) / 1e9
        res[mode] = {"mlups": round(fluid / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5), "steps": n,
                     "wall_s": round(wall, 3), "hbm_gbs_algorithmic": round(gbs, 1),
                     "roofline_frac": round(gbs / PEAK_HBM_GBS, 4),
                     "nonfinite_cavities": int(sum(1 for m in masses if m != m))}
        if mode == "graph":
            res[mode]["launch_shape"] = {"block": shape[0], "cells_per_thread": shape[1],
                                         "waves_per_simd": shape[2], "xcd_split": shape[3], "edge_cells": shape[4]}
        b.close()
        del b
        torch.cuda.empty_cache()
    return {"workload": f"512 D3Q19 TRT cavities, L~U{{16..64}}, Re~U[100,1000], u_lid=0.03, FP32-shifted {scheme}",
            "scheme": scheme, "cells": int(cells), "fluid_cells": int(fluid), "bytes_per_update": 153, **res,
            "speedup_graph_vs_sequential": round(res["graph"]["mlups"] / res["sequential"]["mlups"], 2)}


COLLISION_MODELS = ("bgk", "trt", "reg", "rr", "nw4", "rm", "hm", "cm", "chm", "k")


def run_collision_models(steps, warmup, cav):
    """The ten collision models (BGK-W2, TRT, REG, RR, BGK-NW4, RM, HM, CM,
    CHM, cumulant; high-order rates 1) on the 256^3 cavity, AA-SoA, in FP64
    and FP32-shifted storage; the paper finds the slowest within 2x of the
    fastest (Sec. 3.2.3)."""
    out = {}
    for dtype in ("f64", "f32"):
        rows = []
        for coll in COLLISION_MODELS:
            r = run_case("aa", coll, dtype, steps, warmup, cav)
            rows.append({"collision": coll, "mlups": round(r["mlups"], 1),
                         "algorithmic_gbs": round(r["algorithmic_gbs"], 1), "block_size": r["block_size"],
                         "finite": r["finite"]})
            print(f"# model {coll} {dtype}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        m = [r["mlups"] for r in rows]
        out[dtype] = {"runs": rows, "slowest_over_fastest": round(min(m) / max(m), 3)}
    return out


DOMAIN_SIZES = (16, 24, 32, 48, 64, 96, 128, 192, 256, 320, 400)


def domain_sweep():
    """MLUPS against cavity size N (walls included) for AA vs 2Pop (push and
    pull) and BGK vs RR, FP64 D3Q19 SoA, as in the domain-size study of
    Sec. 3.2.4; steps per size chosen for about 0.3 s of timed work."""
    from paper_2010_11751_amd import lbm, workloads as W
    rows = []
    for n in DOMAIN_SIZES:
        omega = W.omega_from_nu(0.05 * n / 1000.0)
        for scheme in ("aa", "2pop", "2pop_pull"):
            for coll in ("bgk", "rr"):
                fluid = (n - 2) ** 3
                steps = int(min(2000, max(20, 0.3 / (fluid / 15e9))))
                steps += steps % 2
                sim = lbm.Lattice(19, n, scheme=scheme, collision=coll, omega=omega, u_lid=0.05)
                ms, _ = time_steps(sim, steps, max(steps // 10, 10))
                info = sim.info()
                sim.close()
                r = {"n": n, "scheme": scheme, "collision": coll, "steps": steps,
                     "ms_per_step": round(ms, 5), "mlups": round(info.fluid_cells / (ms * 1e-3) / 1e6, 1),
                     "algorithmic_gbs": round(info.fluid_cells * info.bytes_per_update / (ms * 1e-3) / 1e9, 1)}
                rows.append(r)
                print(f"# N={n} {scheme} {coll}: {r['mlups']} MLUPS", file=sys.stderr, flush=True)
    print(json.dumps({"domain_sweep": rows, "dtype": "f64", "lattice": "D3Q19", "layout": "SoA"}), flush=True)


def validation(re=100.0, u=0.1, grids=(32, 64, 128), tstar=20.0, scheme="aa", coll="bgk"):
    """Self-convergence of the lid-driven cavity (Sec. 3.1 validation case;
    the spectral and experimental reference data are not available): FP64
    D3Q19, M fluid cells per edge on nested grids (cell centres of the coarse
    grid are midpoints of fine ones), lid u along +x, nu = u M / Re, run to
    t = tstar M / u. Centreline u_x(z) and u_z(x) through the cavity centre
    (the four nearest cell columns averaged), their change over the last
    tenth of the run (steadiness), and the differences between successive
    grids with the coarse values compared to pair averages of the fine."""
    import math
    import numpy as np
    from paper_2010_11751_amd import lbm, workloads as W
    prof = {}
    for m in grids:
        n = m + 2
        sim = lbm.Lattice(19, n, scheme=scheme, collision=coll, omega=W.omega_from_nu(u * m / re), u_lid=u)
        steps = int(round(tstar * m / u))
        steps += steps % 2
        chunk = max(2, (steps // 20) // 2 * 2)

        def centrelines():
            _, v = sim.macroscopic()
            v = v.cpu().numpy().reshape(3, n, n, n) / u
            c = (m // 2, m // 2 + 1)
            ux = np.mean([v[0, a, b, 1:n - 1] for a in c for b in c], axis=0)
            uz = np.mean([v[2, 1:n - 1, b, d] for b in c for d in c], axis=0)
            return ux, uz
        done, prev = 0, None
        t0 = time.perf_counter()
        while done < steps:
            k = min(chunk, steps - done)
            sim.step(k)
            done += k
            if steps - done <= steps // 10 and prev is None:
                prev = centrelines()
            sim.sync()
            print(f"# validation Re={re:g} M={m}: {done}/{steps} steps, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
        ux, uz = centrelines()
        m_, _ = sim.invariants()
        finite = bool(np.isfinite(ux).all() and np.isfinite(uz).all() and m_ == m_)
        drift = float(max(np.abs(ux - prev[0]).max(), np.abs(uz - prev[1]).max())) if prev is not None else None
        sim.close()
        prof[m] = (ux, uz, steps, drift, finite)
        print(f"# validation M={m}: min u_x/U {ux.min():.5f}, max u_z/U {uz.max():.5f}, drift {drift}",
              file=sys.stderr, flush=True)

    def coarsen(a):
        return 0.5 * (a[0::2] + a[1::2])
    out = {"workload": f"D3Q19 lid-driven cavity, Re {re:g}, u_lid {u}, FP64 {scheme} {coll}, t = {tstar:g} M / u_lid",
           "grids": {}}
    for m in grids:
        ux, uz, steps, drift, finite = prof[m]
        out["grids"][m] = {"steps": steps, "finite": finite, "min_ux": round(float(ux.min()), 6),
                           "max_uz": round(float(uz.max()), 6), "min_uz": round(float(uz.min()), 6),
                           "last_tenth_max_change": drift,
                           "ux_centreline": [round(float(x), 6) for x in ux[:: max(1, m // 32)]],
                           "uz_centreline": [round(float(x), 6) for x in uz[:: max(1, m // 32)]]}
    for key, idx in (("ux", 0), ("uz", 1)):
        diffs = []
        for a, b in zip(grids[:-1], grids[1:]):
            d = float(np.abs(prof[a][idx] - coarsen(prof[b][idx])).max())
            out[f"{key}_max_diff_{a}_{b}"] = d
            diffs.append(d)
        if len(diffs) >= 2 and diffs[-1] > 0:
            out[f"{key}_observed_order"] = round(math.log2(diffs[-2] / diffs[-1]), 3)
    print(json.dumps({"validation": out}), flush=True)


def stability(n=400, re=10000.0, steps=20000, coll="rr", scheme="aa"):
    """The paper's turbulent case (Sec. 3.1, 3.2: recursive regularized
    collision, Re 10000, N = 400), FP64 D3Q19, nu = u n / Re, under three
    settings: lid 0.05 with omega_bulk = omega, lid 0.05 with the bulk
    relaxation set to 1 (Eq. bulk: a larger bulk viscosity), and lid 0.03.
    Each run must stay finite and keep the closed cavity's mass; a run that
    turns non-finite is reported with the step it did so at."""
    import math
    from paper_2010_11751_amd import lbm, workloads as W
    out = []
    for u, ob in ((0.05, None), (0.05, 1.0), (0.03, None)):
        omega = W.omega_from_nu(u * n / re)
        sim = lbm.Lattice(19, n, scheme=scheme, collision=coll, omega=omega, u_lid=u, omega_bulk=ob)
        m0, _ = sim.invariants()
        rows = []
        done, chunk = 0, 2000
        t0 = time.perf_counter()
        while done < steps:
            sim.step(chunk)
            done += chunk
            m, e = sim.invariants()
            rows.append({"step": done, "mass_rel_change": (m - m0) / m0, "kinetic_energy": e})
            print(f"# stability {coll} Re={re:g} N={n} u={u} omega_bulk={ob}: step {done}, mass change "
                  f"{(m - m0) / m0:.3e}, KE {e:.6e}, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
            if not (math.isfinite(m) and math.isfinite(e)):
                break
        sim.close()
        finite = all(math.isfinite(r["kinetic_energy"]) for r in rows)
        out.append({"u_lid": u, "omega": round(omega, 6), "omega_bulk": ob if ob is not None else round(omega, 6),
                    "steps": done, "lid_traversals": round(done * u / (n - 2), 3), "finite": finite,
                    "nonfinite_at_step": None if finite else done,
                    "max_abs_mass_rel_change": max(abs(r["mass_rel_change"]) for r in rows) if finite else None,
                    "kinetic_energy_last": rows[-1]["kinetic_energy"] if finite else None})
    print(json.dumps({"stability": {"workload": f"D3Q19 cavity {n}^3, {coll} FP64 {scheme}, Re {re:g}", "runs": out}}),
          flush=True)


def traffic_run(cav):
    import torch
    from paper_2010_11751_amd import lbm
    nbytes = 1 << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    lbm.device_copy(b, a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()
    for scheme, dtype, layout in (("aa", "f64", "soa"), ("aa", "f32", "soa"), ("aa", "f16", "soa"),
                                  ("2pop", "f64", "soa"), ("swap", "f64", "soa"), ("2pop_pull", "f64", "soa"),
                                  ("2pop_pull", "f32", "soa"), ("2pop_pull", "f16", "soa"),
                                  ("2pop_pull", "f64", "blocked"), ("2pop_pull", "f32", "blocked"),
                                  ("2pop_pull", "f16", "blocked")):
        sim = lbm.Lattice(19, cav.n, scheme=scheme, collision="bgk", omega=cav.omega, u_lid=cav.u_lid, dtype=dtype,
                          layout=layout)
        sim.step(4)
        sim.sync()
        info = sim.info()
        print(json.dumps({"traffic_run": f"{scheme}/{dtype}/{layout}", "fluid_cells": info.fluid_cells,
                          "algorithmic_bytes_per_update": info.bytes_per_update, "copy_bytes": 2 * nbytes}),
              flush=True)
        sim.close()
    # The 512-cavity ensemble (FP32-shifted TRT) at fixed launch shapes, 4 steps each.
    from paper_2010_11751_amd import workloads as W
    members = W.ensemble(512)
    ens = [lbm.Cavity(m.n, m.omega, m.u_lid) for m in members]
    stream = torch.cuda.Stream()
    for scheme, shape in (("aa", (1024, 1, 4, 0)), ("2pop_pull", (512, 1, 0, 0))):
        with torch.cuda.stream(stream):
            b = lbm.Batch(ens, scheme=scheme, collision="trt", dtype="f32", use_graph=False, block_size=shape[0],
                          cells_per_thread=shape[1], waves_per_simd=shape[2], xcd_split=shape[3])
        b.step(4)
        b.sync()
        cells, fluid, _ = b.info()
        print(json.dumps({"traffic_run": f"ensemble/{scheme}/f32", "fluid_cells": fluid, "cells": cells,
                          "launch_shape": list(b.launch_shape()), "algorithmic_bytes_per_update": 153}), flush=True)
        b.close()
        del b
        torch.cuda.empty_cache()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cav, budget_s: float = 6.0, max_steps: int = 20, single_budget_s: float = 4.0):
    """The FP64 oracle on the host cores (OpenMP over cells), on bounded
    samples of every workload (whole steps, one to a few per case, about
    30 s in all on 16 threads): the headline case (256^3 cavity, 2Pop pull
    BGK) as `value`, then the 32^3 correctness cavity (100 steps), the nine
    scheme x collision runs of the 256^3 cavity (one step each), D3Q27 RR AA
    on a 40^3 cavity (the oracle's RR takes seconds per million cells; the
    workload's 512^3 would need 29 GB of FP64 host memory per array), the
    256^3 Taylor-Green AA run and the 512-cavity ensemble stepped cavity by
    cavity; one thread on the headline case and the small cavity."""
    import numpy as np
    import oracle as O
    from paper_2010_11751_amd import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    O.set_threads(threads)

    def timed(sim, fluid, budget, cap, first=True):
        if first:
            sim.step(1)  # first touch of the pages
        n, t0 = 0, time.perf_counter()
        while n < cap and (n == 0 or (time.perf_counter() - t0) < budget):
            sim.step(1)
            n += 1
        dt = time.perf_counter() - t0
        return round(fluid * n / dt / 1e6, 3), n, round(dt, 2)

    def cavity_cfg(n, q=19, model=O.BGK, omega=cav.omega, u=cav.u_lid):
        return O.Config(q=q, nx=n, ny=n, nz=n, model=model, omega=omega, u_lid=(u, 0.0, 0.0))

    t_all = time.perf_counter()
    sim = O.Simulation(cavity_cfg(cav.n), HEAD_SCHEME)
    head, n, dt = timed(sim, cav.fluid_cells, budget_s, max_steps)
    O.set_threads(1)
    head1, n1, dt1 = timed(sim, cav.fluid_cells, single_budget_s, max_steps, first=False)
    O.set_threads(threads)
    del sim
    per = {}
    small = W.CAVITY_SMALL
    sim = O.Simulation(cavity_cfg(small.n, omega=small.omega, u=small.u_lid), "2pop")
    per["cavity_32_bgk_2pop_100_steps"] = timed(sim, small.fluid_cells, 1e9, 100, first=False)[0]
    O.set_threads(1)
    sim = O.Simulation(cavity_cfg(small.n, omega=small.omega, u=small.u_lid), "2pop")
    per["cavity_32_bgk_2pop_100_steps_1_thread"] = timed(sim, small.fluid_cells, 1e9, 100, first=False)[0]
    O.set_threads(threads)
    for scheme in ("2pop", "swap", "aa"):
        for coll in ("bgk", "trt", "reg"):
            sim = O.Simulation(cavity_cfg(cav.n, model=O.MODELS[coll]), scheme)
            per[f"cavity_256_{scheme}_{coll}"] = timed(sim, cav.fluid_cells, 0.0, 1)[0]
            del sim
    c3 = W.CAVITY_512
    sim = O.Simulation(cavity_cfg(40, q=27, model=O.RR, omega=c3.omega, u=c3.u_lid), "aa")
    per["cavity_40_d3q27_rr_aa (the 512^3 workload's case on 40^3)"] = timed(sim, 38 ** 3, 0.0, 2)[0]
    del sim
    n_tg = W.TGV_N
    u0 = W.taylor_green_velocity(n_tg, n_tg, n_tg, W.TGV_U0)
    sim = O.Simulation(O.Config(q=19, nx=n_tg, ny=n_tg, nz=n_tg, geometry=O.PERIODIC, omega=W.omega_from_nu(W.TGV_NU)),
                       "aa", u=u0)
    del u0
    per["taylor_green_256_aa"] = timed(sim, n_tg ** 3, 0.0, 1)[0]
    del sim
    members = W.ensemble(512)
    sims = [O.Simulation(O.Config(q=19, nx=m.n, ny=m.n, nz=m.n, model=O.TRT, omega=m.omega,
                                  u_lid=(m.u_lid, 0.0, 0.0)), "aa") for m in members]
    fluid = sum((m.n - 2) ** 3 for m in members)
    t0 = time.perf_counter()
    for _ in range(2):
        for sm in sims:
            sm.step(1)
    per["ensemble_512_trt_aa_serial"] = round(fluid * 2 / (time.perf_counter() - t0) / 1e6, 3)
    del sims
    return {"value": head, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} whole {HEAD_SCHEME} BGK FP64 steps of the 256^3 cavity ({dt:.1f} s), OpenMP over cells",
            "single_core": {"value": head1, "unit": "MLUPS", "cores": 1,
                            "sample": f"{n1} whole steps ({dt1:.1f} s) on one thread"},
            "per_workload_mlups": per,
            "total_s": round(time.perf_counter() - t_all, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--reps", type=int, default=5,
                    help="timed runs of --steps steps for the headline and FP32 figures; the median is reported")
    ap.add_argument("--no-sweep", action="store_true", help="skip the nine FP64 scheme x collision runs and the ten-model sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 512^3 D3Q27, Taylor-Green and ensemble workloads")
    ap.add_argument("--domain-sweep", action="store_true",
                    help="only the MLUPS-vs-cavity-size sweep (N = 16..400; AA vs 2Pop push / pull, BGK vs RR, FP64)")
    ap.add_argument("--jsonl", default=None,
                    help="also append one JSON record per measured run to this file")
    ap.add_argument("--taylor-green", action="store_true",
                    help="only the periodic 256^3 Taylor-Green workload (2Pop pull and AA; FP64 / FP32 / FP16)")
    ap.add_argument("--validation", action="store_true",
                    help="only the cavity self-convergence study (Re 100, M = 32 / 64 / 128)")
    ap.add_argument("--validation-re1000", action="store_true",
                    help="only the cavity self-convergence study at Re 1000 (BGK, lid 0.05, M = 64 / 128 / 256, "
                         "t = 40 M / u_lid)")
    ap.add_argument("--stability", action="store_true",
                    help="only the RR stability run of the paper's turbulent case (Re 10000, N = 400, 20000 steps)")
    ap.add_argument("--pattern-probe", action="store_true",
                    help="only the memory-pattern probe (19 FP64 streams, SoA and blocked layouts, local / pull / "
                         "AA-odd patterns) beside the FP64 step kernels of the 256^3 cavity")
    ap.add_argument("--mall-probe", action="store_true",
                    help="only the memory patterns of the step kernels on footprints around the 256 MB last-level "
                         "cache (19 FP64 streams, N = 64 .. 256, one array in place or two arrays), at 2 waves per SIMD")
    ap.add_argument("--ensemble", action="store_true",
                    help="only the 512-cavity ensemble (AA and 2Pop pull; --steps graph steps, --warmup warm-up steps)")
    ap.add_argument("--traffic", action="store_true",
                    help="short run for hardware byte counters: one 1 GiB device copy, then 4 BGK steps of "
                         "the 256^3 cavity each for AA FP64 / FP32- / FP16-shifted, 2Pop FP64, swap FP64 and 2Pop "
                         "pull FP64 / FP32- / FP16-shifted, then 4 steps each of the 512-cavity ensemble (AA and "
                         "2Pop pull, FP32-shifted TRT)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the cavity step runs on a single MI355X; "
              "multi-GPU slab decomposition is not built (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_11751_amd import workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    cav = W.CAVITY_256
    print(f"# device: {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)
    if args.traffic:
        traffic_run(cav)
        return
    if args.domain_sweep:
        domain_sweep()
        return
    if args.validation:
        validation()
        return
    if args.validation_re1000:
        validation(re=1000.0, u=0.05, grids=(64, 128, 256), tstar=40.0)
        return
    if args.stability:
        stability()
        return
    if args.pattern_probe:
        rows = pattern_probe(cav)
        kernels = {f"{sch}/f64": round(run_case(sch, "bgk", "f64", 200, 20, cav, reps=3)["algorithmic_gbs"], 1)
                   for sch in ("2pop_pull", "aa", "2pop")}
        print(json.dumps({"pattern_probe": rows, "step_kernels_algorithmic_gbs": kernels}), flush=True)
        return
    if args.mall_probe:
        print(json.dumps({"mall_probe": mall_probe()}), flush=True)
        return
    if args.ensemble:
        seq = max(2, min(100, args.steps // 10))
        print(json.dumps({"ensemble_512": run_ensemble(args.steps, seq, "aa", args.warmup),
                          "ensemble_512_pull": run_ensemble(args.steps, seq, HEAD_SCHEME, args.warmup)}), flush=True)
        return
    if args.taylor_green:
        print(json.dumps({"taylor_green_256": run_taylor_green(args.steps, HEAD_SCHEME, HEAD_LAYOUT),
                          "taylor_green_256_aa": run_taylor_green(args.steps, "aa")}), flush=True)
        return

    head = run_case(HEAD_SCHEME, "bgk", "f64", args.steps, args.warmup, cav, reps=args.reps, layout=HEAD_LAYOUT)
    print(f"# f64 {HEAD_SCHEME} {HEAD_LAYOUT} bgk: {head['mlups']:.0f} MLUPS, {head['algorithmic_gbs']:.0f} GB/s",
          file=sys.stderr, flush=True)
    f32 = run_case(HEAD_SCHEME, "bgk", "f32", args.steps, args.warmup, cav, reps=args.reps, layout=HEAD_LAYOUT)
    print(f"# f32 {HEAD_SCHEME} {HEAD_LAYOUT} bgk: {f32['mlups']:.0f} MLUPS, {f32['algorithmic_gbs']:.0f} GB/s",
          file=sys.stderr, flush=True)
    soa64 = run_case(HEAD_SCHEME, "bgk", "f64", args.steps, args.warmup, cav, reps=args.reps)
    print(f"# f64 {HEAD_SCHEME} soa bgk: {soa64['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    soa32 = run_case(HEAD_SCHEME, "bgk", "f32", args.steps, args.warmup, cav, reps=args.reps)
    print(f"# f32 {HEAD_SCHEME} soa bgk: {soa32['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    aa64 = run_case("aa", "bgk", "f64", args.steps, args.warmup, cav, reps=args.reps)
    print(f"# f64 aa bgk: {aa64['mlups']:.0f} MLUPS, {aa64['algorithmic_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    aa32 = run_case("aa", "bgk", "f32", args.steps, args.warmup, cav, reps=args.reps)
    print(f"# f32 aa bgk: {aa32['mlups']:.0f} MLUPS, {aa32['algorithmic_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    sweep = []
    if not args.no_sweep:
        for scheme in ("2pop", "swap", "aa", "2pop_pull"):
            for coll in ("bgk", "trt", "reg"):
                r = run_case(scheme, coll, "f64", max(args.steps // 5, 20), max(args.warmup // 5, 10), cav)
                sweep.append({k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()
                              if k in ("scheme", "collision", "mlups", "algorithmic_gbs", "ms_per_step")})
                print(f"# sweep {scheme} {coll}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    shifted_schemes = []
    if not args.no_sweep:
        for dtype in ("f32", "f16"):
            for scheme in ("2pop", "aa", "2pop_pull"):
                r = run_case(scheme, "bgk", dtype, max(args.steps // 5, 20), max(args.warmup // 5, 10), cav)
                shifted_schemes.append({k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()
                                        if k in ("scheme", "collision", "dtype", "mlups", "algorithmic_gbs",
                                                 "ms_per_step")})
                print(f"# {dtype} {scheme} bgk: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    models = None
    if not args.no_sweep:
        models = run_collision_models(max(args.steps // 5, 20), max(args.warmup // 5, 10), cav)
    workloads = {}
    if not args.no_configs:
        workloads["cavity_512_d3q27_rr_f32"] = run_d3q27_rr(max(args.steps // 5, 20), 10)
        print(f"# d3q27 rr 512: {workloads['cavity_512_d3q27_rr_f32']['mlups']} MLUPS", file=sys.stderr, flush=True)
        workloads["cavity_512_d3q27_rr_f32_pull"] = run_d3q27_rr(max(args.steps // 5, 20), 10, HEAD_SCHEME)
        print(f"# d3q27 rr 512 {HEAD_SCHEME}: {workloads['cavity_512_d3q27_rr_f32_pull']['mlups']} MLUPS", file=sys.stderr,
              flush=True)
        workloads["taylor_green_256"] = run_taylor_green(2000, HEAD_SCHEME, HEAD_LAYOUT)
        workloads["taylor_green_256_aa"] = run_taylor_green(2000, "aa")
        print("# taylor-green done", file=sys.stderr, flush=True)
        workloads["ensemble_512"] = run_ensemble(1000, 100)
        print(f"# ensemble: {workloads['ensemble_512']['graph']['mlups']} MLUPS (graph)", file=sys.stderr, flush=True)
        workloads["ensemble_512_pull"] = run_ensemble(1000, 100, HEAD_SCHEME)
        print(f"# ensemble {HEAD_SCHEME}: {workloads['ensemble_512_pull']['graph']['mlups']} MLUPS (graph)",
              file=sys.stderr, flush=True)
    copy_gbs = copy_ceiling_gbs()
    print(f"# copy kernel: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    streams_gbs = stream_copy_ceiling(cav)
    print(f"# 19-stream copy: {streams_gbs} GB/s", file=sys.stderr, flush=True)

    def roofline(r):
        achieved = r["fluid_cells"] * r["bytes_per_update"] / (r["kernel_avg_ms"] * 1e-3) / 1e9
        traffic = stored_traffic(traffic_key(r))
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                "kernel": kernel_label(r),
                "bytes_per_launch": r["fluid_cells"] * r["bytes_per_update"],
                "frac_of_copy": round(achieved / copy_gbs, 4)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cav)
        print(f"# cpu oracle: {cpu['value']} MLUPS on {cpu['cores']} threads", file=sys.stderr, flush=True)

    out = {
        "metric": "MLUPS + HBM GB/s vs peak, D3Q19 256^3 cavity: FP64 vs FP32-shifted storage",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "repetitions": len(head["runs_ms_per_step"]),
        "runs_ms_per_step": head["runs_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "D3Q19 lid-driven cavity 256^3 incl. walls, Re=1000, u_lid=0.05, "
                               "BGK, two-population scheme in pull form, blocked layout (the 19 streams of each "
                               "run of 256 cells together), position-driven kernel, FP64 populations",
                   "scheme": HEAD_SCHEME, "layout": HEAD_LAYOUT,
                   "cells": cav.cells, "fluid_cells": cav.fluid_cells, "omega": round(cav.omega, 6),
                   "parallelism": "single GPU"},
        "hbm_gbs": round(head["algorithmic_gbs"], 1),
        "roofline": roofline(head),
        "fp32_shifted": {"value": round(f32["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(f32["ms_per_step"], 5),
                         "hbm_gbs": round(f32["algorithmic_gbs"], 1), "speedup_vs_f64": round(f32["mlups"] / head["mlups"], 3),
                         "roofline": roofline(f32)},
        "soa_layout": {d: {"value": round(r["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 5),
                           "hbm_gbs": round(r["algorithmic_gbs"], 1), "roofline": roofline(r)}
                       for d, r in (("f64", soa64), ("f32", soa32))},
        "aa_pattern": {d: {"value": round(r["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 5),
                           "hbm_gbs": round(r["algorithmic_gbs"], 1), "runs_ms_per_step": r["runs_ms_per_step"],
                           "roofline": roofline(r)} for d, r in (("f64", aa64), ("f32", aa32))},
        "copy_kernel_gbs": round(copy_gbs, 1),
        "stream_copy_19_gbs": streams_gbs,
        "sweep_f64": sweep,
        "schemes_shifted_bgk": shifted_schemes,
        "collision_models": models,
        "workloads": workloads,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.jsonl:
        write_records(args.jsonl, out, (head, f32, soa64, soa32, aa64, aa32), copy_gbs)


def write_records(path, out, heads, copy_gbs):
    """One record per measured run: workload, scheme, collision, dtype,
    MLUPS (fluid and all cells), algorithmic GB/s and its fraction of the HBM
    peak and of the measured copy rate, host cores of the CPU baseline."""
    cores = (out.get("cpu_baseline") or {}).get("cores")
    recs = []
    for r in heads:
        recs.append({"workload": "cavity_256", "scheme": r["scheme"], "collision": r["collision"], "dtype": r["dtype"],
                     "layout": "soa", "mlups_fluid": round(r["mlups"], 1), "mlups_total": round(r["mlups_all_cells"], 1),
                     "gbs_algorithmic": round(r["algorithmic_gbs"], 1)})
    for r in out["sweep_f64"]:
        recs.append({"workload": "cavity_256", "scheme": r["scheme"], "collision": r["collision"], "dtype": "f64",
                     "layout": "soa", "mlups_fluid": r["mlups"], "gbs_algorithmic": r["algorithmic_gbs"]})
    for r in out.get("schemes_shifted_bgk") or []:
        recs.append({"workload": "cavity_256", "scheme": r["scheme"], "collision": r["collision"], "dtype": r["dtype"],
                     "layout": "soa", "mlups_fluid": r["mlups"], "gbs_algorithmic": r["algorithmic_gbs"]})
    for dtype, block in (out.get("collision_models") or {}).items():
        for r in block["runs"]:
            recs.append({"workload": "cavity_256", "scheme": "aa", "collision": r["collision"], "dtype": dtype,
                         "layout": "soa", "mlups_fluid": r["mlups"], "gbs_algorithmic": r["algorithmic_gbs"]})
    w = out.get("workloads") or {}
    for key in ("cavity_512_d3q27_rr_f32", "cavity_512_d3q27_rr_f32_pull"):
        if key in w:
            r = w[key]
            recs.append({"workload": "cavity_512_d3q27", "scheme": r["scheme"], "collision": "rr", "dtype": "f32",
                         "layout": "soa", "mlups_fluid": r["mlups"], "gbs_algorithmic": r["hbm_gbs"]})
    for key in ("taylor_green_256", "taylor_green_256_aa"):
        if key not in w:
            continue
        for dtype in ("f64", "f32", "f16"):
            r = w[key][dtype]
            recs.append({"workload": "taylor_green_256", "scheme": w[key]["scheme"], "collision": "bgk", "dtype": dtype,
                         "layout": "soa", "mlups_fluid": r["mlups"], "gbs_algorithmic": r["hbm_gbs"],
                         "velocity_rel_l2_vs_f64": r.get("velocity_rel_l2_vs_f64")})
    for key in ("ensemble_512", "ensemble_512_pull"):
        if key not in w:
            continue
        for mode in ("graph", "sequential"):
            r = w[key][mode]
            recs.append({"workload": "ensemble_512", "scheme": w[key]["scheme"], "collision": "trt", "dtype": "f32",
                         "layout": "soa", "mode": mode, "mlups_fluid": r["mlups"],
                         "gbs_algorithmic": r["hbm_gbs_algorithmic"]})
    with open(path, "a") as f:
        for r in recs:
            g = r.get("gbs_algorithmic")
            if g:
                r["pct_peak"] = round(100 * g / PEAK_HBM_GBS, 2)
                r["pct_copy"] = round(100 * g / copy_gbs, 2)
            r["host_cores"] = cores
            f.write(json.dumps(r) + "\n")


if __name__ == "__main__":
    main()
