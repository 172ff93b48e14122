"""MI355X (gfx950) truncated-Newton entropic optimal transport.

The computation lives in the HIP library libeot.so (C ABI: include/eot.h);
:mod:`paper_2504_02067_amd.eot` is its ctypes binding, taking torch GPU
tensors. :mod:`paper_2504_02067_amd.workloads` builds seeded synthetic
instances.
"""
from . import eot  # noqa: F401
from .eot import (eot_hvp, eot_marginals, eot_newton_cg, eot_solve,  # noqa: F401
                  default_solve_opts, EotError)

__all__ = ["eot", "eot_marginals", "eot_hvp", "eot_newton_cg", "eot_solve",
           "default_solve_opts", "EotError"]
