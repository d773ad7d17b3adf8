"""CPU FP64 oracle for the e-ph transition-probability path (test infrastructure).

This package is a plain, slow, obviously-correct NumPy implementation of what
the electron-phonon path computes, written from the paper's equations:
Wannier-to-Bloch transforms (Eqs. 1-3, 5, 6), transition probabilities
(Eq. 8), RTA scattering rates (Eqs. 12, 21, 25), the coupled drag iteration
(Eqs. 19-27) and the transport tensors (Eqs. 28-30).

It is test infrastructure only: the tests, the smoke check and the CPU
baseline leg of the benchmark import it; the product library never does, and
it shares no code with the HIP path.
"""
from .elph_oracle import *  # noqa: F401,F403
