"""MI355X-native matrix-free Newton-Stokes operator engine.

The compute path lives in the HIP library built from ``csrc/`` (C ABI in
``include/nsmf.h``); ``nsmf.Engine`` is its Python binding.
"""
from .nsmf import Engine, NsmfError, load_library, FP64, FP32, FP32_BF16OPS

__all__ = ["Engine", "NsmfError", "load_library", "FP64", "FP32", "FP32_BF16OPS"]
