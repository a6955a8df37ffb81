"""Pins of the oracle's linear-stability eigenvalue (Sec. IX "Eigenvalue
solver": sigma M X + (L + L') X = 0 about the conduction state, the
eigenvalue nearest a real shift) against closed forms and the classical
onset:

* without buoyancy the temperature modes decouple from the flow:
  sigma = -kappa (n^2 pi^2 + k^2), n >= 1;
* the mean pencil (gauge row) holds the pure diffusion modes of b and u:
  -kappa n^2 pi^2 and -nu n^2 pi^2;
* at the no-slip, fixed-temperature onset (Ra = 1707.76, k = 3.117) the
  growth rate crosses zero;
* the dense and the ARPACK shift-invert routes agree, for one eigenvalue and
  for several (nearest the shift first).
"""
import math

import numpy as np
import pytest

from oracle import RBOracle, RBParams


@pytest.mark.parametrize("n", [1, 2, 3])
def test_temperature_modes_without_buoyancy(n):
    o = RBOracle(8, 32, 2.0, RBParams(1e4, 1.0, buoyancy=0.0))
    kx = 3.0
    s = -o.par.kappa * (n * n * math.pi ** 2 + kx * kx)
    assert abs(o.stability_eigenvalue(kx, 0.0, s * 1.0001) - s) < 1e-12


@pytest.mark.parametrize("Pr", [0.5, 7.0])
def test_mean_pencil_diffusion_modes(Pr):
    o = RBOracle(8, 32, 2.0, RBParams(1e4, Pr))
    kap, nu = o.par.kappa, o.par.nu
    for c in (kap, nu):
        for n in (1, 2):
            s = -c * n * n * math.pi ** 2
            assert abs(o.stability_eigenvalue(0.0, 0.0, s * 1.0001, is_mean=True) - s) < 1e-12


def test_onset_growth_rate_crosses_zero():
    def sig(Ra):
        o = RBOracle(8, 32, 2.0, RBParams(Ra, 1.0))
        return o.stability_eigenvalue(3.117, 0.0, 0.05)
    assert sig(1690.0) < 0 < sig(1725.0)
    assert abs(sig(1707.76)) < 1e-5


def test_dense_and_shift_invert_routes_agree():
    o = RBOracle(16, 64, 2.0, RBParams(1e5, 1.0))
    for kx, tau in ((3.117, 0.5), (6.0, -0.2)):
        a = o.stability_eigenvalue(kx, 0.0, tau, method="dense")
        b = o.stability_eigenvalue(kx, 0.0, tau, method="arpack")
        assert abs(a - b) < 1e-9 * max(1.0, abs(a)), (kx, a, b)


def test_mean_pencil_nearest_modes_in_order():
    """Several eigenvalues at once (the Krylov solver's output): at Pr = 0.5
    the four modes of the mean pencil nearest 0.01 are the diffusion modes
    -nu pi^2, -kappa pi^2, -4 nu pi^2, -4 kappa pi^2 (nu = kappa / 2), in
    that order."""
    o = RBOracle(8, 32, 2.0, RBParams(1e4, 0.5))
    kap, nu = o.par.kappa, o.par.nu
    want = [-nu * math.pi ** 2, -kap * math.pi ** 2, -4 * nu * math.pi ** 2, -4 * kap * math.pi ** 2]
    got = o.stability_eigenvalues(0.0, 0.0, 0.01, nev=4, is_mean=True)
    for g, w in zip(got, want):
        assert abs(g - w) < 1e-12, (got, want)


def test_temperature_modes_3d_without_buoyancy():
    """3-D pencil (kx, ky): without buoyancy the temperature modes are
    -kappa (n^2 pi^2 + kx^2 + ky^2)."""
    o = RBOracle(8, 16, 2.0, RBParams(1e4, 1.0, buoyancy=0.0), dim=3, Ny=8, Ly=2.0)
    kx, ky = 3.0, -2.0
    for n in (1, 2):
        s = -o.par.kappa * (n * n * math.pi ** 2 + kx * kx + ky * ky)
        got = o.stability_eigenvalues(kx, ky, s * 1.0001, nev=1)[0]
        assert abs(got - s) < 1e-12


def test_dense_and_arpack_agree_on_several_modes():
    o = RBOracle(16, 64, 2.0, RBParams(1e5, 1.0))
    for kx, tau in ((3.117, 0.5), (6.0, -0.2)):
        a = o.stability_eigenvalues(kx, 0.0, tau, nev=5, method="dense")
        b = o.stability_eigenvalues(kx, 0.0, tau, nev=5, method="arpack")
        assert np.abs(a - b).max() < 1e-9 * max(1.0, np.abs(a).max()), (kx, a, b)
