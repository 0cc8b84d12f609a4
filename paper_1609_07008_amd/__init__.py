"""MFBC (maximal frontier betweenness centrality) on MI355X.

The compute path lives in ``libmfbc.so`` (HIP kernels for gfx950 behind a
C ABI declared in ``include/mfbc.h``); ``paper_1609_07008_amd.mfbc`` is its
thin ctypes binding.  ``paper_1609_07008_amd.graphgen`` makes seeded
synthetic inputs.  Submodules are imported on demand so that importing the
generators never loads the GPU library.
"""
__all__ = ["graphgen", "mfbc"]
