"""MI355X (gfx950) engine for fixed-step RK4 integration of coupled
Hodgkin-Huxley networks (Mohanta & Assisi, arXiv 1906.03958).

``psst``      -- binding of the C ABI in include/psst.h (libpsst.so, HIP)
``workloads`` -- seeded synthetic antennal-lobe-shaped inputs
``autograd``  -- torch.autograd.Function over the discrete adjoint
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "psst"]
