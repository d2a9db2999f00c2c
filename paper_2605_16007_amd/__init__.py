"""MI355X-native IVF-RaBitQ search: Python binding of librbq.

The search path (probe, rotation, query quantisation, code scan with the fused
estimator, top-R selection, exact re-rank) runs in hand-written HIP kernels for
gfx950 behind the C ABI of include/rbq.h. This package only marshals arguments.
"""
from .rbq import Index, RbqError, Server, huge_page_rows, lib, version, LIB_PATH, SYMBOLS  # noqa: F401
