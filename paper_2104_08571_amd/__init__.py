"""MI355X-native padded-tile finite-volume Euler step (HIP kernels for gfx950).

The compute path lives in ``libripple_fv.so`` (C ABI declared in
``include/ripple_fv.h``); ``paper_2104_08571_amd.ripple_fv`` is its thin ctypes
binding.  Importing this package loads nothing: the binding loads the shared
library on first use and raises if it is missing, and ``initial_states``
holds the seeded input generators.
"""
__all__ = ["ripple_fv", "initial_states"]
