"""MI355X-native TT-rounding and TT orthogonalization (CGS, MGS, CGS2, MGS2, Gram).

The compute path is the C-ABI library ``libttortho.so`` (hand-written HIP for
gfx950); :mod:`paper_2211_08770_amd.tt` is its thin Python binding.  Importing
this package loads nothing: the binding loads the library on first use and
raises if it is missing.
"""
__all__ = ["tt", "synth"]
