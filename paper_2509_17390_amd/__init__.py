"""MI355X-native batched LiDAR ray casting (FGGS-LiDAR, arXiv 2509.17390, Sec. IV-C).

The compute path is the HIP library ``_lib/librcast.so`` (C ABI in
``include/rcast.h``); ``rcast`` is its thin ctypes binding.
"""
from .rcast import (Context, Job, RcastError, load, LIB_PATH, RC_NODE_FP32, RC_NODE_Q8)  # noqa: F401

__all__ = ["Context", "Job", "RcastError", "load", "LIB_PATH", "RC_NODE_FP32", "RC_NODE_Q8"]
