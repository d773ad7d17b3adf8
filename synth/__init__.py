"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws random numbers and assembles the Wannier-space input
arrays (Hamiltonian H(R_e), force constants D(R_p), vertex g(R_e, R_p), and
for polar materials Born charges and the dielectric tensor, and
third-order force constants for three-phonon processes); it
holds none of the method's arithmetic (no Fourier sums, no eigensolves, no
transition probabilities).  Calibrated scale parameters (band gap offset,
Hamiltonian scale, force-constant scale, chemical potential) are stored in
``configs.json``, written by ``tests/golden/calibrate_configs.py``.
"""
from . import mlp  # noqa: F401
from .materials import (  # noqa: F401
    rset_cube, rset_sphere, make_material, config, config_names, material_for, polar_params,
    MASS_CYCLE, LATTICE_A, ifc3_params,
)
