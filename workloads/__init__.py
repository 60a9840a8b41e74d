"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package holds random draws and workload recipes only -- none of the method's
arithmetic (no Laplacian, no basis, no products).  The vorticity field of every workload is
given by its spherical-harmonic coefficients omega_lm; turning them into a matrix is the
basis assembly of eq. (W0), which each side does with its own code.
"""

from .spectra import omega_coeffs, sigma_law, ensemble_sizes, WORKLOADS

__all__ = ["omega_coeffs", "sigma_law", "ensemble_sizes", "WORKLOADS"]
