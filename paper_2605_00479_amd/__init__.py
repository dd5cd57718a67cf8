"""MI355X-native ensemble Gillespie direct method in FP64, mixed 16-bit and
uniform 16-bit precision (Kimpson, Flegg & Flegg, "Reduced-Precision
Stochastic Simulation for Mathematical Biology").

The compute path is the HIP library ``libssa_rp.so`` built from ``csrc/``;
``ssa`` is its thin ctypes binding. Importing this package loads nothing:
``workloads`` (input descriptions) and ``stats`` (ensemble statistics) are
plain host modules.
"""
