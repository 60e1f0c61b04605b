"""MI355X-native echellogram renderer (Genoni et al. 2020 hot path).

The product is ``libe2e.so`` (C ABI in ``include/e2e.h``) with hand-written
HIP kernels for gfx950; this package is its thin ctypes binding.
"""
from . import e2e
from .e2e import E2EError, lib
from .host import Loaded, make_req, psf_desc, trace_descs

__all__ = ["e2e", "E2EError", "lib", "Loaded", "make_req", "psf_desc", "trace_descs"]
