"""MI355X-native diffuse-interface multiphysics step (arXiv 2009.14555).

Submodules:
  problems  seeded synthetic inputs (primitive fields) and material constants
  dimp      ctypes binding of the HIP C-ABI library libdimp.so
  solver    Grid / PatchSet objects holding device state in torch tensors
The HIP library is loaded on first use of `dimp` and fails loudly when absent.
"""
__all__ = ["problems"]
