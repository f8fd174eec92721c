"""Seeded synthetic inputs shaped like the paper's diamond-carbon k-point workloads.

This package builds inputs only: one-body blocks, momentum-blocked Cholesky
vectors, trial orbitals, walkers and auxiliary fields.  It holds none of the
method's arithmetic (no Green's function, force bias, potential, propagation or
energy); both the FP64 oracle and the GPU library consume the arrays it returns.
"""

from .kpt_inputs import (  # noqa: F401
    KptSystem,
    CONFIGS,
    make_system,
    make_walkers,
    make_fields,
    config_shapes,
    make_spin_trial,
    spin_view,
    RaggedSystem,
    make_ragged_system,
    make_ragged_walkers,
    pack_ragged,
)
