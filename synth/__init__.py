"""Seeded synthetic line lists (input data only; none of the method's arithmetic).

Shared by the CPU oracle's tests, the GPU parity tests and the benchmark as a
source of input arrays.  Nothing here computes intensities, widths or profiles.
"""
from .linelist import (  # noqa: F401
    WorkloadConfig, CONFIGS, config_by_name, make_states, make_transitions,
    make_broadening_table, make_linelist, make_vibrational_labels, splitmix64_ref, uniform53,
)
