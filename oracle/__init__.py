"""CPU rules oracle for the batched Stratego engine (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (built from
``stratego_oracle.c`` with gcc) through ctypes; the arithmetic lives in the C
file, which cites the paper section each function follows.
"""
from .oracle import (  # noqa: F401
    OracleEngine,
    build,
    lib,
    battle,
    philox4x32_10,
    setup_types,
    hidden_prob,
    fnv1a64,
    digest_blocks,
    num_threads,
    REC_BYTES,
    MASK_WORDS,
    NCHAN,
    MAX_LEGAL,
    SAMPLER_UNIFORM,
    SAMPLER_MAGNET,
)
from .history import OracleRolloutBuffer, WindowError  # noqa: F401,E402
