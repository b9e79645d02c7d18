"""Gaussian-mixture interpolation of scattered points onto a regular grid, for MI355X.

The interpolation (paper, Eq. 1-2) runs in hand-written HIP kernels behind the
C-ABI library ``libgmminterp.so``; this package binds it for PyTorch.  Heavy
imports are lazy so that ``paper_2012_13257_amd.synth`` works without torch.
"""
__all__ = ["interpolate", "InterpFunction", "Server", "lib"]


def __getattr__(name):
    if name in ("interpolate", "InterpFunction", "forward", "backward", "debug_bins"):
        from . import interp
        return getattr(interp, name)
    if name == "Server":
        from .server import Server
        return Server
    if name == "lib":
        from . import _lib
        return _lib.lib()
    raise AttributeError(name)
