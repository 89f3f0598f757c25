"""libism: the Intermediate State Method (ISM) hot path on AMD Instinct MI355X.

The compute path is the HIP library ``libism.so`` (built in-tree for gfx950);
this package only marshals arguments to it (``_lib``), wraps its hand-written
adjoint in a ``torch.autograd.Function`` (``autograd``) and runs a
continuous-batching solve server on top of it (``serve``).
"""
from ._lib import (FP32_MIXED, FP64, GATE, STATE, IsmError, Problem, Server,  # noqa: F401
                   footprint, from_problem, lib)

__all__ = ["Problem", "Server", "IsmError", "from_problem", "footprint", "lib", "FP64",
           "FP32_MIXED", "STATE", "GATE"]
