"""Pins of the oracle's non-constant coefficient (NCC) term Gamma(z) w in
the b equation (Sec. II, non-constant coefficients):

* the product matrix against the Chebyshev product identity
  T_n T_j = (T_{n+j} + T_{|n-j|}) / 2, i.e. <T_i|T_n T_j> = (d_{i,j+n} + d_{i,|j-n|}) / 2;
* the product matrix against pointwise products on a grid (Clenshaw);
* a manufactured stratified Stokes pencil through the linear boundary value
  solve (Gamma w evaluated pointwise in the right-hand side);
* a constant Gamma = g0 shifts the linear-stability problem exactly like a
  conduction gradient changed by g0.
"""
import math

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle import RBOracle, RBParams, ncc_matrix, spectral as S


@pytest.mark.parametrize("N,nt", [(8, 1), (12, 3), (33, 5)])
def test_ncc_matrix_product_identity(N, nt):
    rng = np.random.default_rng(N)
    g = rng.standard_normal(nt)
    G = ncc_matrix(g, N)
    ref = np.zeros((N, N))
    for i in range(N):
        for j in range(N):
            ref[i, j] = 0.5 * sum(g[n] * ((i == j + n) + (i == abs(j - n))) for n in range(nt))
    np.testing.assert_allclose(G, ref, atol=1e-15)


def test_ncc_matrix_pointwise_product():
    N, nt = 24, 4
    rng = np.random.default_rng(5)
    g = rng.standard_normal(nt)
    c = np.zeros(N)
    c[: N - nt] = rng.standard_normal(N - nt)  # product stays inside N modes
    x = np.linspace(-1, 1, 101)
    np.testing.assert_allclose(npc.chebval(x, ncc_matrix(g, N) @ c), npc.chebval(x, g) * npc.chebval(x, c),
                               atol=1e-13)


@pytest.mark.parametrize("gamma", [(0.5, 0.3), (-0.2, 0.4, 0.25)])
def test_stratified_stokes_pencil(gamma):
    Nx, Nz, Lx, ix = 16, 40, 4.0, 1
    o = RBOracle(Nx, Nz, Lx, RBParams(1e4, 1.0, gamma=gamma))
    kap, nu = o.par.kappa, o.par.nu
    k = 2 * math.pi * ix / Lx
    _, z = o.scale1_grids()
    pi = math.pi
    Gam = npc.chebval(2 * z - 1, gamma)
    b = np.sin(pi * z)
    w = np.sin(pi * z) ** 2
    u = 1j * pi * np.sin(2 * pi * z) / k
    p = -nu * pi * (4 * pi ** 2 + k ** 2) * np.sin(2 * pi * z) / k ** 2
    dp = -nu * pi * (4 * pi ** 2 + k ** 2) * 2 * pi * np.cos(2 * pi * z) / k ** 2
    lap_w = 2 * pi ** 2 * np.cos(2 * pi * z) - k ** 2 * w
    Fz = S.cheb_forward_matrix(Nz, Nz)
    F = np.zeros((o.Px, o.ne, Nz), complex)
    F[ix, 0] = Fz @ (kap * (pi ** 2 + k ** 2) * b + Gam * w)
    F[ix, 2] = Fz @ (-nu * lap_w + dp - b)
    X = o.lbvp(F)
    for name, vals in (("b", b), ("w", w), ("u", u), ("p", p)):
        ref = Fz @ vals
        assert np.abs(X[ix, o.vi[name]] - ref).max() < 1e-11 * max(1.0, np.abs(ref).max()), name


def test_constant_ncc_equals_shifted_gradient():
    g0 = 0.35
    a = RBOracle(8, 32, 2.0, RBParams(3000.0, 1.0, gamma=(g0,)))
    b = RBOracle(8, 32, 2.0, RBParams(3000.0, 1.0, b_bottom=1.0 - g0))
    for kx in (2.0, 3.117):
        sa = a.stability_eigenvalue(kx, 0.0, 0.3)
        sb = b.stability_eigenvalue(kx, 0.0, 0.3)
        assert abs(sa - sb) < 1e-12, (kx, sa, sb)
