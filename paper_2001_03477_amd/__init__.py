"""pcvof: geometric PLIC-VOF advection with conservative thermal-energy advection
and the two-step phase-change shift (arXiv 2001.03477, sections 3.3 and 3.4.1) as
hand-written HIP kernels for MI355X (gfx950) behind a C-ABI library.

``pcvof`` is the ctypes binding of ``include/pcvof.h``; ``workloads`` draws the
seeded synthetic inputs."""
from . import workloads  # noqa: F401

__all__ = ["pcvof", "workloads"]
