"""Ensemble transfer entropy (KSG estimator) on AMD MI355X: Python binding of libte.

The computation runs in libte.so (HIP kernels for gfx950 behind the C interface
in include/te.h).  This package only marshals arguments; PyTorch supplies
device memory and streams.
"""
from ._lib import LIB_PATH, TEError, lib
from .api import (Plan, Server, autotune, knn_counts, knn_counts_noalloc, profile_enable, ragwitz, profile_read, profile_work, profile_work_all, tune_clear, tune_load, tune_save,
                  version)

__all__ = ["LIB_PATH", "Plan", "Server", "TEError", "autotune", "knn_counts", "knn_counts_noalloc", "lib", "ragwitz", "profile_enable", "profile_read", "profile_work", "profile_work_all",
           "tune_clear", "tune_load", "tune_save", "version"]
