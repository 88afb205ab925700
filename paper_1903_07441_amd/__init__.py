"""MI355X-native harmonic potential fields on time-warped grids.

The compute path is the HIP library ``libtwg.so`` built from ``csrc/`` for
gfx950; ``twg`` binds its C ABI with ctypes.  Importing this package loads
nothing: ``from paper_1903_07441_amd import twg`` does.
"""
__all__ = ["twg", "scenarios"]
