"""MI355X (gfx950) Barnes-Hut force step after Bedorf, Gaburov & Portegies Zwart,
"Bonsai: A GPU Tree-Code" (arXiv:1204.2280).

Submodules:
  mibh       ctypes binding of the HIP library libmibh.so (C ABI in include/mibh.h)
  workloads  seeded synthetic particle sets (Plummer, Hernquist, ensembles)
  build      hipcc build of libmibh.so
"""

__all__ = ["mibh", "workloads", "build"]
