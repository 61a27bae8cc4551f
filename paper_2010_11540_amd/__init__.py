"""scpic: MI355X-native 2D particle-in-cell space-charge tracking (arXiv:2010.11540).

The compute path is a HIP library for gfx950 (``libscpic.so``) behind a C ABI
(``include/scpic.h``); ``paper_2010_11540_amd.scpic`` is its thin ctypes binding
over PyTorch device tensors.  ``paper_2010_11540_amd.inputs`` builds seeded
synthetic beams, grids and lattices.
"""
__version__ = "0.1.0"
