"""MI355X-native (gfx950) hot path of linear-scaling LNV density-matrix
minimisation (Sec. II.C.2 of arXiv:2002.07704, the CONQUEST code paper).

  lib     ctypes binding of liblnv.so (C ABI in include/lnv.h)
  system  device-resident patterns, matrices and CG workspace of one geometry
  build   hipcc build of liblnv.so for gfx950
  autograd  LNVEnergy: E(L, S, H) with the hand-written adjoint as backward
"""
from . import lib  # noqa: F401

__all__ = ["lib"]
