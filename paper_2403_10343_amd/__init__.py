"""MI355X RI-LVL exact-exchange build: thin Python layer over libexx.so."""
from ._lib import (PREC_FP32, PREC_FP64, ExxError, Plan, lib)  # noqa: F401

__all__ = ["Plan", "ExxError", "PREC_FP64", "PREC_FP32", "lib"]
