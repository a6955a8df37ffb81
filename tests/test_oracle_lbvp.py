"""Pins of the oracle's linear boundary value solve L X = F (Sec. IX "Linear
boundary value solver") against closed-form solutions:

* F = 0: the conduction state b = 1 - z, hydrostatic p = z - z^2/2 - 1/2
  (gauge p(1) = 0), no flow;
* a Fourier pencil with b = sin(pi z) and a manufactured Stokes flow
  w = sin^2(pi z), u = i w'/k (continuity), p from the x momentum equation,
  with F_w from the z momentum equation (buoyancy included);
* the mean pencil with u = sin(pi z) under F_u = nu pi^2 sin(pi z).
"""
import math

import numpy as np
import pytest

from oracle import RBOracle, RBParams, spectral as S


def _coef(o, vals):
    """T coefficients of values on the scale-1 Chebyshev grid."""
    return S.cheb_forward_matrix(o.Nz, o.Nz) @ vals


@pytest.mark.parametrize("Ra,Pr,Nz", [(1e4, 1.0, 32), (1e6, 7.0, 48)])
def test_conduction_state(Ra, Pr, Nz):
    o = RBOracle(8, Nz, 4.0, RBParams(Ra, Pr))
    _, z = o.scale1_grids()
    X = o.lbvp(np.zeros((o.Px, o.ne, Nz), complex))
    vi = o.vi
    np.testing.assert_allclose(X[0, vi["b"]], _coef(o, 1.0 - z), atol=1e-14)
    np.testing.assert_allclose(X[0, vi["bz"]], _coef(o, -np.ones_like(z)), atol=1e-12)
    np.testing.assert_allclose(X[0, vi["p"]], _coef(o, z - z * z / 2 - 0.5), atol=1e-14)
    assert np.abs(X[1:]).max() == 0.0
    assert np.abs(X[0, [vi["u"], vi["w"], vi["uz"], vi["wz"]]]).max() < 1e-15


@pytest.mark.parametrize("Ra,Pr,ix", [(1e4, 1.0, 1), (1e6, 7.0, 3)])
def test_manufactured_stokes_pencil(Ra, Pr, ix):
    Nx, Nz, Lx = 16, 40, 4.0
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    kap, nu = o.par.kappa, o.par.nu
    k = 2 * math.pi * ix / Lx
    _, z = o.scale1_grids()
    pi = math.pi
    b = np.sin(pi * z)
    w = np.sin(pi * z) ** 2
    u = 1j * pi * np.sin(2 * pi * z) / k
    p = -nu * pi * (4 * pi ** 2 + k ** 2) * np.sin(2 * pi * z) / k ** 2
    dp = -nu * pi * (4 * pi ** 2 + k ** 2) * 2 * pi * np.cos(2 * pi * z) / k ** 2
    lap_w = 2 * pi ** 2 * np.cos(2 * pi * z) - k ** 2 * w
    F = np.zeros((o.Px, o.ne, Nz), complex)
    F[ix, 0] = _coef(o, kap * (pi ** 2 + k ** 2) * b)     # -kappa lap b = F_b
    F[ix, 2] = _coef(o, -nu * lap_w + dp - b)              # w equation
    X = o.lbvp(F)
    vi = o.vi
    for name, vals in (("b", b), ("w", w), ("u", u), ("p", p)):
        ref = _coef(o, vals)
        assert np.abs(X[ix, vi[name]] - ref).max() < 1e-11 * max(1.0, np.abs(ref).max()), name
    # other Fourier pencils carry nothing; the mean pencil is conduction
    others = [i for i in range(1, o.Px) if i != ix]
    assert np.abs(X[others]).max() == 0.0
    np.testing.assert_allclose(X[0, vi["b"]], _coef(o, 1.0 - z), atol=1e-14)


def test_mean_pencil_shear():
    Nx, Nz = 8, 32
    o = RBOracle(Nx, Nz, 4.0, RBParams(1e5, 1.0))
    _, z = o.scale1_grids()
    F = np.zeros((o.Px, o.ne, Nz), complex)
    F[0, 1] = _coef(o, o.par.nu * math.pi ** 2 * np.sin(math.pi * z))
    X = o.lbvp(F)
    np.testing.assert_allclose(X[0, o.vi["u"]], _coef(o, np.sin(math.pi * z)), atol=1e-14)
    np.testing.assert_allclose(X[0, o.vi["uz"]], _coef(o, math.pi * np.cos(math.pi * z)), atol=1e-12)
