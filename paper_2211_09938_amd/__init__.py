"""MI355X-native progressive saliency-guided hologram generation (arXiv 2211.09938).

The compute path lives in the HIP/C library ``libcgh.so`` built from ``csrc/``;
``cgh`` is its thin ctypes binding.  Importing this package does not load the
library; the first call that needs it does, and fails loudly if it is missing.
"""

__all__ = ["cgh", "scenes"]
