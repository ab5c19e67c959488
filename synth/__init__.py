"""Seeded synthetic inputs for the RT-TDDFT time step.

This package draws random numbers and lays them out; it performs none of the
method's arithmetic (no Hamiltonian, density, potential or propagator).  Both the
CPU oracle and the GPU path take their inputs from here.
"""

from .systems import (  # noqa: F401
    System,
    RunParams,
    make_system,
    make_molecule,
    config_system,
    config_run,
    batch_systems,
    lowpass_orbitals,
    basis_mixing,
    ground_state_start,
    CONFIGS,
)
