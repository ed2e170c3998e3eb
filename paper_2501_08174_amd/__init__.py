"""MI355X-native hot path of object-centric 2D Gaussian splatting.

Submodules are loaded on demand so that the seeded scene generators can be
used without the compiled library:
  scenes     seeded synthetic inputs (no renderer arithmetic)
  _lib       ctypes binding of the C-ABI library libsurfelrast.so
  raster     torch-facing wrappers and the autograd.Function
"""
__all__ = ["scenes"]
