"""MI355X-native (gfx950 HIP, FP64) hot path of the particle filter for the
viscous stochastic Camassa-Holm (SALT) equation of Cotter, Crisan & Singh
(arXiv 2402.06927).

``sch`` is the ctypes binding of the C-ABI in ``include/sch.h``;
``workloads`` holds the seeded synthetic inputs.  Importing the package does
not load the HIP library; the first call into ``sch`` does, and raises if it
is not built.
"""

__all__ = ["sch", "workloads"]
