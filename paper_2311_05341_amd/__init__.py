"""MI355X (gfx950) brute-force incoherent dedispersion.

The transform, its adjoint and a batched multi-beam form run in hand-written
HIP kernels behind the C ABI of include/dd.h; this package is the Python
binding (ctypes + torch device memory and streams).
"""
from .binding import (  # noqa: F401
    DD_F32,
    DD_U16,
    DD_U4,
    DD_U8,
    LIB_PATH,
    BIN_OUT,
    SURVEY_BIN_DTYPE,
    Batch,
    DDError,
    DedisperseFn,
    Plan,
    Survey,
    bin_time,
    corner_turn,
    dedisperse,
)
from .chunks import TimeChunks  # noqa: F401
