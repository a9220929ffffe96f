"""The oracle under AddressSanitizer (host code only): a copy built with
-fsanitize=address runs every entry point (both lattices, every collision
model, every scheme and layout, caller geometry, sampled reference cells,
read-outs) in a child process with the sanitizer runtime preloaded. Any
out-of-bounds or use-after-free access aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle as O
O.LIB = sys.argv[2]
rng = np.random.default_rng(5)
for q in (19, 27):
    c, t, opp = O.lattice(q)
    for model in O.MODELS:
        if model == "k" and q == 27:
            continue
        cfg = O.Config(q=q, nx=6, ny=5, nz=7, model=O.MODELS[model], omega=1.6, omega_bulk=1.2, omega3=1.1,
                       omega4=0.9, u_lid=(0.04, 0.0, 0.0))
        O.collide(cfg, rng.uniform(0.01, 0.1, q))
        O.equilibrium(q, 1.02, np.array([0.01, -0.02, 0.03]), O.MODELS[model])
        for layout in (O.SOA, O.AOS):
            cfg.layout = layout
            for scheme in ("ref", "2pop", "swap", "aa", "2pop_pull"):
                s = O.Simulation(cfg, scheme)
                s.step(3)
                s.macroscopic()
                s.invariants()
    for geo in (O.PERIODIC, O.CHANNEL):
        cfg = O.Config(q=q, nx=5, ny=4, nz=6, geometry=geo, model=O.TRT, omega=1.7, u_lid=(0.03, 0.0, 0.0))
        fl = O.flags(cfg).copy()
        fl[7] = O.WALL
        wu = rng.uniform(-0.02, 0.02, (3, cfg.ntot))
        s = O.Simulation(cfg, "aa", cell_types=fl, wall_u=wu, wall_rho=rng.uniform(0.9, 1.1, cfg.ntot))
        s.step(4)
        O.reference_cells(cfg, s.flags, s.natural(), [0, cfg.ntot - 1, 11])
        for i in (0, cfg.ntot - 1):
            for k in range(q):
                O.neighbour_index(cfg, i, k)
print("asan child ok")
"""


def test_oracle_under_address_sanitizer(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no AddressSanitizer runtime for gcc")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
                           "-ffp-contract=off", "-fPIC", "-fopenmp", "-shared",
                           os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-o", lib, "-lm"])
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, lib], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "asan child ok" in r.stdout, r.stderr[-3000:]
