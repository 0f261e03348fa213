"""MI355X RI-LVL exact-exchange build: thin Python layer over libexx.so."""
from ._lib import (PREC_BF16X3, PREC_FP32, PREC_MIXED, PREC_FP64, ExxError, Plan, lib)  # noqa: F401


def exchange_energy(plan, C, V, D, precision=PREC_FP64):
    """Differentiable E_x per system (see paper_2403_10343_amd.autograd)."""
    from .autograd import exchange_energy as f
    return f(plan, C, V, D, precision)


def spin_exchange_energy(plan, C, V, D):
    """Differentiable collinear-spin E_x per system (D: spin 0 then spin 1)."""
    from .autograd import spin_exchange_energy as f
    return f(plan, C, V, D)


def exchange_forces(plan, C, V, D, c_decay=1.5, v_2s2=8.0, gE=1.0):
    from .autograd import exchange_forces as f
    return f(plan, C, V, D, c_decay, v_2s2, gE)


__all__ = ["Plan", "ExxError", "PREC_FP64", "PREC_MIXED", "PREC_FP32", "PREC_BF16X3", "lib", "exchange_energy",
           "spin_exchange_energy", "exchange_forces"]
