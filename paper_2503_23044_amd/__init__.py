"""MI355X-native batched differentiable RGB-D-N Gaussian rasterizer
(CityGS-X, arXiv 2503.23044, Sec. 3.2-3.3).

The compute path is libcgx.so (hand-written HIP for gfx950) behind the C ABI
in include/cgx.h; `binding` marshals arguments to it with the same names and
`render` wraps it with torch tensors and autograd.  Nothing here computes on
the CPU; a missing library raises on first use.
"""
from . import binding  # noqa: F401

__all__ = ["binding"]
