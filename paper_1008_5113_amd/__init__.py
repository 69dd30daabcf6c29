"""MI355X-native determinant ratios of consecutive sparse Slater matrices.

The hot path (proposal, Slater row, ILUTP-preconditioned GMRES, ratio,
Metropolis decision, preconditioner updates, reorder and refactor) and the
kinetic energy through the same solver run in the HIP library
``libvmcdet.so``; ``vmcdet`` is its ctypes binding.
"""
from .vmcdet import (Context, STEP_RECORD_DTYPE, VmcError, default_params, params_from_workload,
                     PREC_FP64, PREC_MIXED, FLAG_ACCEPTED, FLAG_REORDERED, FLAG_REFACTORED,
                     FLAG_CONVERGED, FLAG_SINGULAR, FLAG_CAPACITY, FLAG_TRIG_N, FLAG_TRIG_NOCONV,
                     FLAG_TRIG_ITERS, FLAG_TRIG_FORCED, FLAG_NOCONV, LIB_PATH, load_library, lib,
                     VMC_ESTATE, VMC_ENOCONV, VMC_ESINGULAR, VMC_EINVAL)

__all__ = ["Context", "STEP_RECORD_DTYPE", "VmcError", "default_params", "params_from_workload",
           "PREC_FP64", "PREC_MIXED", "FLAG_ACCEPTED", "FLAG_REORDERED", "FLAG_REFACTORED",
           "FLAG_CONVERGED", "FLAG_SINGULAR", "FLAG_CAPACITY", "FLAG_TRIG_N", "FLAG_TRIG_NOCONV",
           "FLAG_TRIG_ITERS", "FLAG_TRIG_FORCED", "FLAG_NOCONV", "VMC_ESTATE", "VMC_ENOCONV",
           "VMC_ESINGULAR", "VMC_EINVAL", "LIB_PATH",
           "load_library", "lib"]
