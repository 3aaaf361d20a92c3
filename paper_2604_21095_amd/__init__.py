"""MI355X (gfx950) phenotype-panel linear association scan.

The compute path is the HIP library libtgw.so (kernels + C ABI declared in
include/tgw.h); ``paper_2604_21095_amd.tgw`` is its thin ctypes binding.
Importing the binding fails loudly when the library has not been built.
"""
import importlib

__all__ = ["tgw"]


def __getattr__(name):
    if name == "tgw":
        return importlib.import_module(__name__ + ".tgw")
    raise AttributeError(name)
