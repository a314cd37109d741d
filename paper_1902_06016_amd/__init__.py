"""MI355X IP-GFCC solver: shifted Green's-function linear solves and their reduced-order model.

The compute lives in ``libgfcc.so`` (HIP, gfx950); ``paper_1902_06016_amd.gfcc`` is its ctypes
binding. Build with ``python -m paper_1902_06016_amd.build``.
"""
__all__ = ["gfcc", "build"]
