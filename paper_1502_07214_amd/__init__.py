"""MI355X-native parallel multicanonical (MUCA) sampling of the 3D Blume-Capel model.

The compute path is libmuca.so (HIP kernels for gfx950 + C ABI, include/muca.h);
`muca` is its ctypes binding.  PyTorch provides device memory and streams only.
"""
from .muca import (REC_ACCUMULATED, REC_EXTRAPOLATE, MucaBatch, MucaError, MucaJob, OBS_FIELDS, lib,  # noqa: F401
                   muca_flatness, muca_host_order, muca_host_tables, muca_query_sizes)

__all__ = ["MucaBatch", "MucaError", "MucaJob", "OBS_FIELDS", "REC_ACCUMULATED", "REC_EXTRAPOLATE", "lib",
           "muca_flatness", "muca_host_order", "muca_host_tables", "muca_query_sizes"]
