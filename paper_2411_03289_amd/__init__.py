"""MI355X (gfx950) HIP implementation of the GP-augmented chance-constrained
MPPI rollout (arXiv 2411.03289).

Submodules:
  gpmppi     ctypes binding of libgpmppi.so (the C ABI of include/gpmppi.h)
  workloads  seeded synthetic problem instances
  build      hipcc build of libgpmppi.so

Importing the package loads nothing; the library is loaded on first use.
"""
