"""MI355X (gfx950) list-mode OSEM with attenuation and first-order scatter
compensation for 2-D SPECT.

The reconstruction runs in liblmosem.so (HIP kernels behind the C ABI of
include/lmosem.h); ``paper_2002_12471_amd.lmosem`` is its Python binding.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblmosem.so")


def build(verbose: bool = False) -> str:
    from .build import build as _build
    return _build(verbose)
