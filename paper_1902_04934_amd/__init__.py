"""MI355X-native ILE likelihood hot path (arXiv:1902.04934, Sec. II).

``paper_1902_04934_amd.ile``   ctypes binding of libile.so (the C ABI in
                               include/ile.h; HIP kernels for gfx950)
``paper_1902_04934_amd.synth`` seeded synthetic workloads (inputs only)
``paper_1902_04934_amd.build`` builds libile.so in-tree with hipcc

Importing the package loads nothing; ``ile.lib()`` loads the library and
raises if it has not been built.
"""
__all__ = ["ile", "synth", "build"]
