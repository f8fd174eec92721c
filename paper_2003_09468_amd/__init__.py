"""MI355X-native k-point AFQMC walker-batch step (arXiv:2003.09468).

The compute path is the gfx950 shared library ``libafqmc_kpt.so`` built from
``csrc/`` (C ABI declared in ``include/afqmc_kpt.h``).  This package is its thin
Python binding: argument marshalling over ctypes, with torch tensors supplying
device memory and the current HIP stream.  There is no CPU fallback: every
call fails loudly when the library or a gfx950 device is missing.
"""

from .binding import (  # noqa: F401
    AfqmcError,
    KptProblem,
    KptBatch,
    KptGraph,
    KptSpinPair,
    SPIN_CLOSED,
    SPIN_UP,
    SPIN_DOWN,
    lib,
    library_path,
    PREC_FP64,
    PREC_FP32,
    PREC_BF16X3,
    PREC_INT8X5,
    PREC_INT8X4,
    prec_place,
    step_prec,
    energy_prec,
    WALKER_SINGULAR,
    WALKER_NONFINITE,
    WALKER_KILLED,
    ENTRIES,
    local_energy,
    reblock,
    pad_bands,
    unpad_bands,
    timing_enable,
    timing_read,
    KERNEL_CLASSES,
)
