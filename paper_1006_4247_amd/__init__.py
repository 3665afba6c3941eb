"""hsgpt: MI355X-native parallel tempering for the 3D Heisenberg spin glass.

The hot path (checkerboard heat-bath + overrelaxation sweeps, FP64 energies,
replica exchange, annealed exchange, overlap measurements) runs in hand-written
HIP kernels behind the C ABI of include/hsgpt.h (libhsgpt.so, built in-tree).
This package is the thin Python binding: PyTorch supplies device memory and
streams only.  There is no CPU fallback: importing the binding without the
built library raises.
"""
from ._abi import HsgError, lib  # noqa: F401
from .ensemble import (Ensemble, device_to_natural, geometric_betas,  # noqa: F401
                       natural_to_device, natural_to_device_index)

__all__ = ["Ensemble", "HsgError", "lib", "geometric_betas", "device_to_natural",
           "natural_to_device", "natural_to_device_index"]
