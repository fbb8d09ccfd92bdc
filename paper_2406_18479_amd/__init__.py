"""MI355X-native GW self-energy hot path (Iskakov et al., Green/WeakCoupling, Sec. 2).

The compute lives in ``libgreen_gw.so`` (hand-written HIP for gfx950, C ABI in
include/green_gw.h).  ``paper_2406_18479_amd.gw.Plan`` is the torch-facing
binding.  Importing ``gw`` raises ImportError when the library is not built.
"""
__all__ = ["gw"]
