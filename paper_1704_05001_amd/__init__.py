"""nAIR (Neumann approximate ideal restriction AMG) on MI355X.

The hierarchy build and the V-cycle solve run in the HIP kernels of
libnair_hip.so, reached through the C ABI of include/nair.h; `nair` is the
ctypes binding.
"""
from .nair import (Hierarchy, Params, Result, NairError, lib, LIB_PATH, EXPORTED, STATUS, KERNELS, TUNE_KINDS,
                   pool_trim, timer_select, timer_read, grad_vals, NOALLOC_SCRATCH_BYTES)
from .autograd import NairSolve, solve

__all__ = ["Hierarchy", "Params", "Result", "NairError", "lib", "LIB_PATH", "EXPORTED", "STATUS", "KERNELS", "TUNE_KINDS",
           "pool_trim", "timer_select", "timer_read", "grad_vals", "NOALLOC_SCRATCH_BYTES", "NairSolve", "solve"]
