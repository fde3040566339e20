"""MI355X (gfx950) implementation of the per-frame 3D Gaussian Splatting
render path of "Visionary" (arXiv 2512.08478, Section 3.2 and Algorithm 1):
EWA projection, SH colour, (tile, depth) keys, a GPU radix sort and
front-to-back tile compositing, with a hand-written backward pass.

The compute path is the C-ABI library ``libgs.so`` (include/gs.h), built
in-tree by ``paper_2512_08478_amd.build``; ``render`` and ``Renderer`` wrap
it for PyTorch.  Importing this package does not load the library;
the first render call does, and raises if it is missing.
"""
__version__ = "0.1.0"


def __getattr__(name):
    if name in ("Renderer", "GaussianParams", "Frame", "render", "GsRender"):
        from . import render as _render
        return getattr(_render, name)
    raise AttributeError(name)
