"""MI355X-native RI-HF hot path (arXiv 2407.19614): Python binding of libri.

Every step of the computation runs in the HIP kernels of ``libri.so``; this
package only marshals arguments (PyTorch supplies device memory and streams).
Importing it does not load the library; the first call does, and raises if
the library has not been built.
"""
from .binding import (FP64, FP32, BF16X3, BF16X6, COMPRESSED, FINAL_FP64, RIError, RIProblem, lib, load_library,  # noqa: F401
                      ri_status_str, workspace_bytes, packed_b_bytes, MLP, MLP_FP32, MLP_BF16,
                      pack_params, unpack_params, NPARAM)
