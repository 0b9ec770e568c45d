"""MI355X-native DIAM: P periodically synchronised adaptive-Metropolis chains
on hand-written HIP kernels for gfx950.

The compute path lives in ``libdiam.so`` (C ABI, see ``include/diam.h``);
``paper_1506_05741_amd.diam`` is its thin ctypes binding and
``paper_1506_05741_amd.synth`` draws seeded inputs.  Importing the package
does not load the library; ``diam.load()`` does, and raises if it is missing.
"""
__all__ = ["synth", "diam"]
