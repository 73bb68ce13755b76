"""MI355X-native 4D Gaussian Splatting renderer (HIP, gfx950) with a C ABI.

`g4d` is the ctypes binding of libg4d.so; `build` compiles it.
"""
from . import g4d  # noqa: F401
from .g4d import Render4DGS, Renderer, render  # noqa: F401
