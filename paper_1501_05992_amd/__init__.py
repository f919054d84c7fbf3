"""corrx: an MI355X-native X-engine for the MWA correlator (Ord et al., arXiv 1501.05992).

The hot path lives in the HIP library ``libcorrx.so`` behind the C ABI declared
in ``include/corrx.h``; ``paper_1501_05992_amd.corrx`` is its thin ctypes
binding.  Importing this package does not load the GPU library.
"""

__all__ = ["corrx", "synth", "model"]
