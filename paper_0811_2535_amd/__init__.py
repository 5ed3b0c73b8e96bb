"""liftfft: the dimension-lifted 1-D complex FFT of Hunt, Mullin, Rosenkrantz
and Raynolds (Sections 2-4 of their paper) as HIP kernels for MI355X (gfx950).

The compute path is the C-ABI library ``libliftfft.so`` (``include/liftfft.h``);
this package holds its sources, the in-tree build and a thin Python binding.

    import torch, paper_0811_2535_amd as lf
    y = lf.fft(x)            # x: complex64/complex128 CUDA tensor, last dim n = 2^t
    z = lf.fft(y, sign=+1)   # unnormalized: z == n * x
    g = lf.LiftFFT.apply(x, -1)   # differentiable; backward is the adjoint transform
"""
from .binding import (FFTError, LibraryNotBuilt, Plan, cached_plan, clear_plan_cache,  # noqa: F401
                      fft, lib, strerror)
from .autograd import LiftFFT, fft_autograd  # noqa: F401

__all__ = ["fft", "Plan", "FFTError", "LibraryNotBuilt", "LiftFFT", "fft_autograd", "lib",
           "strerror", "cached_plan", "clear_plan_cache"]
