"""MI355X (gfx950) implementation of the matrix-free Jacobian / priorconditioned
LSQR path of QPAT with a lagged-diffusivity Perona-Malik prior
(Hannukainen, Hyvonen, Majander, Tarvainen, arXiv:1512.02796).

The compute path is libqpat.so (HIP kernels behind the C ABI of
include/qpat.h); ``qpat`` is its ctypes binding and ``driver`` runs
Algorithm 1 on top of it. Build with ``python -m paper_1512_02796_amd.build``.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqpat.so")


def load():
    """Import the binding (raises ImportError when libqpat.so is missing)."""
    from . import qpat
    return qpat
