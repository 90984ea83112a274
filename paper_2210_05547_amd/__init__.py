"""Reacting-flow right-hand side and Runge-Kutta stage on AMD MI355X (gfx950).

The compute path is the HIP library ``libhrx.so`` (sources in ``csrc/``, C-ABI in
``include/hrx.h``); ``hrx`` is its ctypes binding and ``fields`` the seeded
synthetic workload generator.
"""
