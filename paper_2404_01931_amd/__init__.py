"""MI355X-native FLIP timestep (arXiv 2404.01931).

The compute path is the C-ABI library ``libflipmi.so`` built from ``csrc/``
(hand-written HIP for gfx950); ``flip`` is its thin Python binding and
``inputs`` holds the seeded synthetic scenes. Importing this package loads
nothing; ``paper_2404_01931_amd.flip`` loads the library on first use and
raises if it has not been built.
"""

__all__ = ["flip", "inputs"]
