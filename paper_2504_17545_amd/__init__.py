"""MI355X (gfx950) render library for Gaussian-enhanced surfels.

The render and its gradient run in hand-written HIP kernels behind the C ABI
of include/ges.h (libges.so); `_lib` binds that ABI with ctypes and `render`
adds torch buffers, streams and autograd.
"""
from . import _lib
from ._lib import GESError
from .render import Frame, PlannedFrame, Renderer, render_differentiable
from .translucent import TranslucentFrame, TranslucentRenderer

__all__ = ["_lib", "GESError", "Frame", "PlannedFrame", "Renderer", "render_differentiable", "TranslucentFrame",
           "TranslucentRenderer"]
