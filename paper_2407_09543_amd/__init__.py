"""libntbc: Neural Texture Block Compression (BC1/BC4) on MI355X (gfx950).

The compute path lives in the HIP shared library ``libntbc.so`` built from ``csrc/``; ``ntbc`` is its
thin ctypes binding.  ``synth`` holds the seeded synthetic inputs.
"""
