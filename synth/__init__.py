"""Seeded synthetic workloads for correlated-sampling phaseless AFQMC.

This module only draws and arranges input data: one-body matrices, Cholesky
vectors, trial orbitals, auxiliary-field arrays and the batch recipes of the
benchmark configurations.  It performs none of the method's arithmetic and is
the one module that both the FP64 oracle and the GPU path read their inputs
from.
"""
from .configs import (  # noqa: F401
    Hamiltonian,
    PairConfig,
    config,
    gaussian_fields,
    make_hamiltonian,
    make_expansion,
    make_trial,
    pair_batch_configs,
    perturbation,
    random_walkers,
)
