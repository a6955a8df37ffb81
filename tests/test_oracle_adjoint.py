"""Pins of the oracle's discrete adjoint: dot-product identities of every
linear piece against its forward, exactness of central differences for the
quadratic pieces (the explicit term and the kinetic energy are bilinear /
quadratic in the state), and the full gradient against central finite
differences on tiny problems."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import RBOracle, RBParams
from oracle import adjoint as ADJ


def _rand_state(o, seed):
    X = si.complex_noise(o.state_shape, seed)
    if o.dim == 2:
        X[0] = X[0].real
        X[o.Px - 1] = 0
    else:
        X[:, o.Px - 1] = 0
        X[o.Ny // 2] = 0
        # kx = 0 column must be Hermitian in ky for a real field
        for iy in range(1, o.Ny // 2):
            X[o.Ny - iy, 0] = np.conj(X[iy, 0])
        X[0, 0] = X[0, 0].real
    return X


def _ip(a, b):
    """Real inner product of complex (or real) arrays: Re sum conj(a) b."""
    return float(np.real(np.vdot(a, b)))


@pytest.fixture(params=[2, 3], ids=["2d", "3d"])
def orc(request):
    if request.param == 2:
        return RBOracle(8, 6, 3.0, RBParams(3e4, 1.0))
    return RBOracle(6, 6, 3.0, RBParams(3e4, 1.0), dim=3, Ny=6, Ly=2.0)


def test_transform_adjoints_dot_product(orc):
    o = orc
    rng = np.random.default_rng(0)
    c = _rand_state(o, 1)[..., 1, :]
    gshape = o.to_grid(c).shape
    gbar = rng.standard_normal(gshape)
    assert abs(_ip(gbar, o.to_grid(c)) - _ip(ADJ.to_grid_adjoint(o, gbar), c)) < 1e-12
    g = rng.standard_normal(gshape)
    cbar = _rand_state(o, 2)[..., 1, :]
    assert abs(_ip(cbar, o.from_grid(g)) - _ip(ADJ.from_grid_adjoint(o, cbar), g)) < 1e-12


def test_nonlinear_adjoint_exact(orc):
    # N is bilinear: N'(X) d = (N(X + d) - N(X - d)) / 2 exactly
    o = orc
    X = _rand_state(o, 3)
    d = _rand_state(o, 4)
    Fbar = si.complex_noise(o.nonlinear(X).shape, 5)
    lin = 0.5 * (o.nonlinear(X + d) - o.nonlinear(X - d))
    lhs = _ip(Fbar, lin)
    rhs = _ip(ADJ.nonlinear_adjoint(o, X, Fbar), d)
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_kinetic_energy_adjoint_exact(orc):
    o = orc
    X = _rand_state(o, 6)
    d = _rand_state(o, 7)
    fd = 0.5 * (o.kinetic_energy(X + d) - o.kinetic_energy(X - d))
    assert abs(fd - _ip(ADJ.kinetic_energy_adjoint(o, X), d)) < 1e-12 * max(1.0, abs(fd))


def test_initial_state_adjoint_dot_product(orc):
    o = orc
    shape = (o.Nx, o.Nz) if o.dim == 2 else (o.Nx, o.Ny, o.Nz)
    g = np.random.default_rng(8).standard_normal(shape)
    Xbar = _rand_state(o, 9)
    X = o.state_from_b_grid(g)
    assert abs(_ip(Xbar, X) - _ip(ADJ.initial_state_adjoint(o, Xbar), g)) < 1e-11 * abs(_ip(Xbar, X))


@pytest.mark.parametrize("dim", [2, 3])
def test_gradient_matches_central_differences(dim):
    if dim == 2:
        o = RBOracle(8, 8, 3.0, RBParams(5e3, 1.0))
        shape = (8, 8)
    else:
        o = RBOracle(6, 6, 3.0, RBParams(5e3, 1.0), dim=3, Ny=4, Ly=2.0)
        shape = (6, 4, 6)
    x, *_ = o.scale1_grids()
    z = o.scale1_grids()[-1]
    xi = si.noise(shape, 21)
    b0 = o.initial_b_grid(xi, amp=0.05)
    dt, steps = 5e-2, 6
    J, g = ADJ.gradient(o, b0, dt, steps)
    for r in range(3):
        d = si.direction(shape, r)
        fd = []
        for h in (1e-2, 5e-3):
            fd.append((ADJ.objective(o, b0 + h * d, dt, steps) - ADJ.objective(o, b0 - h * d, dt, steps)) / (2 * h))
        ad = float(np.sum(g * d))
        # Richardson-extrapolated central difference
        fdr = (4 * fd[1] - fd[0]) / 3
        assert abs(fdr - ad) <= 1e-7 * abs(ad) + 1e-14, (fd, ad)
