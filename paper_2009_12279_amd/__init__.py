"""MI355X-native lattice Boltzmann for Oldroyd-B fluids with complex and moving
boundaries (after Kuron, Stewart, de Graaf, Holm, arXiv 2009.12279).

The compute path is the HIP library ``libvlb.so`` (C-ABI declared in
``include/vlb.h``); ``paper_2009_12279_amd.vlb`` is its thin ctypes binding,
imported on first use so that the input generators load without a GPU.
"""
import importlib

__all__ = ["vlb", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
