"""NENO6 on MI355X: the six-point neuron-based ENO reconstruction (Li, Fu &
Adams, arXiv 2207.08500) as hand-written HIP kernels for gfx950 behind a C-ABI
library (``libneno6.so``), with a thin ctypes binding.

Submodules:
  native   -- ctypes binding of the C-ABI (same names as ``include/neno6.h``)
  solver   -- torch-facing helpers (device buffers, streams, workspaces)
  autograd -- torch.autograd.Function wrappers (classifier, fixed-mask adjoint)
  inputs   -- seeded synthetic workloads (no method arithmetic)
"""
__all__ = ["native", "solver", "autograd", "inputs"]
