"""MesonGS++ size-aware quantization search hot path on AMD MI355X (gfx950).

The compute path is the C-ABI library ``libmgs.so`` (hand-written HIP kernels
plus the host 0-1 ILP); ``paper_2604_26799_amd.mgs`` is its thin ctypes
binding.  Importing this package loads nothing; the binding loads the library
on first use and raises if it is missing.
"""
__all__ = ["mgs", "synth"]
