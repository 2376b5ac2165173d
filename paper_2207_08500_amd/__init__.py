"""NENO6 on MI355X: the six-point neuron-based ENO reconstruction (Li, Fu &
Adams, arXiv 2207.08500) as hand-written HIP kernels for gfx950 behind a C-ABI
library (``libneno6.so``), with a thin ctypes binding.

Submodules:
  native          -- ctypes binding of the C ABI (same names as ``include/neno6.h``),
                     plus the Problem / Mlp helpers that hold device buffers and
                     workspaces
  autograd        -- torch.autograd.Function wrappers (classifier gradient,
                     fixed-label right-hand-side adjoints)
  autotune        -- launch-shape cache around neno6_autotune
  datagen         -- training data after Alg. 1 on the GPU path
  inputs          -- seeded synthetic workloads (no method arithmetic)
  build           -- hipcc build of libneno6.so
  profile_kernels -- driver for rocprofv3 kernel summaries
"""
__all__ = ["native", "autograd", "autotune", "datagen", "inputs", "build", "profile_kernels"]
