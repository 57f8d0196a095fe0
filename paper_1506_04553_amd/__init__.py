"""MI355X (gfx950) long-range tree force of the P3T scheme.

The compute path is the HIP library ``libp3t.so`` (C ABI in ``include/p3t.h``);
this package is its thin binding.  Importing the package does not load the
library; ``P3T(...)`` does, and raises if it is not built.
"""
from .p3t import (P3T, P3TError, Params, PREC_FP64, PREC_MIXED, check_params,  # noqa: F401
                  load_library, make_params)

__all__ = ["P3T", "P3TError", "Params", "PREC_FP64", "PREC_MIXED", "check_params",
           "load_library", "make_params", "LongForceFn", "long_force"]


def __getattr__(name):
    if name in ("LongForceFn", "long_force"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
