"""DPM score estimation on AMD MI355X: direct and tensor-form (shared
feature-mode basis) filter responses, distance transform and star-model
scores, through the C ABI of libdpmt (include/dpmt.h).

Importing the package does not load the library; the first call does, and it
raises ImportError if libdpmt.so has not been built.
"""
from ._abi import LIB_PATH, MODES, DIRECT_FP32, TENSOR_FP32, TENSOR_BF16, TENSOR_FP8  # noqa: F401
from .api import (Context, DpmtError, Layout, distance_transform, tile_config_count,  # noqa: F401
                  tile_config_name)
