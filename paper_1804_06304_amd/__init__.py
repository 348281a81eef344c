"""MI355X (gfx950) evolution of 3D/2D snakuscules (arXiv 1804.06304): HIP kernels behind a C ABI.

``paper_1804_06304_amd.snk`` is the ctypes binding of ``libsnk.so`` (include/snk.h);
``paper_1804_06304_amd.build`` compiles it with hipcc.
"""
__version__ = "0.1.0"
