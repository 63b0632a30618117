"""mgrw: leading-order event reweighting on AMD Instinct MI355X (gfx950).

The computation lives in libmgrw.so (HIP kernels behind the C ABI of
include/mgrw.h); this package is its Python binding plus the build-time
process generator.
"""
from .binding import (  # noqa: F401
    Process, Params, make_params, MgrwError, LHEFile, multi_reweight, PROCESS_IDS, PRECISIONS, MAX_POINTS, lib,
)
