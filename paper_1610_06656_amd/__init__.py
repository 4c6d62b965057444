"""SMP-PCA (single-pass PCA of matrix products, arXiv 1610.06656) on AMD
Instinct MI355X: hand-written HIP kernels for gfx950 behind the C-ABI of
include/smp.h, with a thin torch/ctypes binding.

    import paper_1610_06656_amd as smp
    U, sigma, V = smp.solve(A, B, k=400, r=10)      # A: d x n1, B: d x n2 (GPU, FP32)

Importing the package does not load the library; the first call does, and it
raises if libsmp.so has not been built (there is no CPU fallback).
"""

from ._lib import (SMP_B_IS_A, SMP_OMEGA_REUSE, SMP_OMEGA_SPLIT, SMP_PREC_BF16, SMP_PREC_FP32,  # noqa: F401
                   LIB_PATH, SmpOmega, SmpParams, load)


def __getattr__(name):
    # the torch-facing binding is imported lazily so that `import paper_1610_06656_amd`
    # stays light (the build step imports the package without touching a GPU)
    if name in ("Context", "Omega", "SmpError", "make_params", "default_m", "solve",
                "smp_check_params", "smp_workspace_size"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
