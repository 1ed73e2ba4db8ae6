"""MI355X-native VR-NeRF renderer hot path (arXiv 2311.02542).

The renderer lives in a C-ABI shared library (``libvrn.so``, built from
``csrc/`` with hipcc for gfx950); ``capi`` is its thin ctypes binding and
``serve`` the serving loop.  ``synth`` draws the seeded synthetic inputs.
Nothing is loaded at import time.
"""
__all__ = ["capi", "synth", "serve"]
