"""MI355X-native TNLM 4DCT reconstruction (arXiv:1009.1351): Python front-end.

Thin wrapper over the C ABI in include/tnlm.h (libtnlm.so): torch CUDA
tensors carry device memory and the current stream; every computation runs in
the library's HIP kernels. Importing ``Recon`` requires the built library.
"""
from __future__ import annotations

__all__ = ["Recon", "Batch", "TnlmError"]


def __getattr__(name):
    if name in ("Recon", "Batch", "TnlmError"):
        from . import recon
        return getattr(recon, name)
    raise AttributeError(name)
