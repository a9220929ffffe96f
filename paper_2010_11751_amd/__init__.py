"""MI355X-native lattice Boltzmann collide-and-stream (arXiv:2010.11751).

The compute path is the HIP library ``liblbm.so`` (``csrc/``) behind the C ABI
declared in ``include/lbm.h``; :mod:`paper_2010_11751_amd.lbm` is its thin
ctypes binding. Importing the package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
__all__ = ["lbm", "workloads"]
