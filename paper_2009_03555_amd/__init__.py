"""MI355X-native screened exchange-matrix builder (HIP kernels behind a C ABI).

The compute path is ``libhfx.so`` (hand-written gfx950 HIP kernels);
``paper_2009_03555_amd.hfx`` is its ctypes binding.  Importing this package
does not load the library; ``hfx.lib()`` does, and raises if it is missing.
"""
from .hfx import (  # noqa: F401
    HFX_SYNC,
    HFX_TIMING,
    HfxError,
    Plan,
    build_K_multi,
    hfx_footprint,
    hfx_last_error,
    lib,
    unpack_quartets,
)
