"""MI355X hot path of self-learning determinantal QMC (arXiv:1612.03804).

The arithmetic lives in the HIP library ``libslq.so`` (C ABI in include/slq.h);
``paper_1612_03804_amd.slq`` is a thin ctypes binding with the same entry-point
names.  PyTorch supplies device memory and streams only.
"""
from .slq import *  # noqa: F401,F403
