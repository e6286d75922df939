"""MI355X batched Stratego engine (arXiv 2511.07312 hot path).

The engine lives in libstratego.so (hand-written HIP for gfx950); this package
is its ctypes binding.  See include/stratego.h for the C ABI.
"""
from .engine import (  # noqa: F401
    Engine,
    StrategoError,
    load_library,
    strerror,
    FUNCTIONS,
    LIB_PATH,
    MASK_WORDS,
    NUM_CHANNELS,
    RECORD_BYTES,
    OBS_BYTES_PER_GAME,
)
from . import engine  # noqa: F401
