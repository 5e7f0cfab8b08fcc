"""Seeded synthetic inputs for the posterior engine (test and benchmark data).

This module draws random numbers and nothing else: sphere models, orientation
grids, CTF parameter grids, per-image true parameters and noise fields.  It
holds none of the method's arithmetic (no projection, no transform, no
likelihood), so both the CPU oracle and the GPU path can take their inputs
from it without sharing code.

Every workload has one generator seeded with ``[160906634, k]``; draws happen
in a fixed order: model, orientation grid, per-image orientation, per-image
shift, per-image CTF, noise, and finally the normalisation/offset stream that
only invariance tests use.
"""
from .configs import (  # noqa: F401
    Workload, SizeClass, make_workload, CONFIGS, electron_wavelength_A,
    ctf_abA_from_physical, shoemake_quaternions, proposal_training_images, symmetric_model,
    symmetry_restricted_euler, expand_symmetry,
)
