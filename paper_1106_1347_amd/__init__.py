"""MI355X (gfx950) library for dense FP64 matrix multiplication by the
methods of Hedtke, "Methods of Matrix Multiplication" (arXiv:1106.1347).

Python binding of the C ABI in ``include/mmm.h``: argument marshalling
only.  Every entry of every result is computed by the HIP kernels in
``libmmm.so``; PyTorch provides device memory (CUDA/HIP tensors) and the
stream the work is enqueued on.  There is no CPU fallback: importing the
module fails when ``libmmm.so`` is missing.

    import torch, paper_1106_1347_amd as mmm
    C = mmm.multiply(A, B, "winograd_scaled")      # A, B: float64 on cuda
"""
from ._lib import (  # noqa: F401
    METHODS,
    TILES,
    Batch,
    Config,
    MmmError,
    lib_path,
    minus,
    multiply,
    multiply_noalloc,
    noalloc_scratch_bytes,
    multiply_with_scalar,
    norm_inf,
    plus,
    timer_start,
    timer_stop,
    version,
    winograd_lambda,
    workspace_bytes,
)
