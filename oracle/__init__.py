"""FP64 CPU oracle for the Fourier x Chebyshev sparse-tau SBDF2 step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product path.
"""
from . import spectral  # noqa: F401
from .rb import RBOracle, RBParams, ncc_matrix, rk_tableau, sbdf_coefficients, tau_poisson_bvp  # noqa: F401
