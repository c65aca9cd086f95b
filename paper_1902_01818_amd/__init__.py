"""MI355X-native multigrid for multi-patch isogeometric analysis (Takacs,
arXiv:1902.01818): HIP kernels behind the C ABI of include/igamg.h, bound to
Python by ctypes in :mod:`paper_1902_01818_amd.igamg`."""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libigamg.so")


def load():
    """Import the ctypes binding (raises if the library is not built)."""
    from . import igamg
    return igamg
