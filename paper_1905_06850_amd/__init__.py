"""libplcg: deep pipelined CG (p(l)-CG) and classic CG on AMD MI355X (gfx950).

The solver is the HIP library ``libplcg.so`` behind the C ABI of
``include/plcg.h``; ``paper_1905_06850_amd.plcg`` is its ctypes binding.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libplcg.so")


def load():
    """Import the binding (raises ImportError when libplcg.so is not built)."""
    from . import plcg
    return plcg
