"""MI355X-native Rotne-Prager-Blake mobility products and Brownian dynamics steps.

The computation lives in the HIP library ``librpb.so`` (C ABI in ``include/rpb.h``);
``Context`` is its thin Python binding (torch tensors for device memory and streams).
"""
from ._lib import Context, RpbError, StepState, load  # noqa: F401

__all__ = ["Context", "RpbError", "StepState", "load"]
