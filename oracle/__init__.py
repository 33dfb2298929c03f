"""CPU FP64 oracle for the bosonic PIMD force-and-energy step (test infrastructure).

This package is TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may use it; the GPU library never does.
It wraps ``pimd_oracle.c`` (plain sequential double precision, written from the
paper's Sec. II-III equations) through ctypes and shares nothing with the GPU path.
"""
from .wrapper import (  # noqa: F401
    OracleParams, OracleMD, lib_path, build, load,
    ring_energy, internal_energies, cycle_energies, forward_potentials,
    backward_potentials, connection_probabilities, exchange_forces, interaction,
    compute_forces, step, conserved, density, exact_energy, exact_energy_signed,
    philox4x32_10, init_state,
)
