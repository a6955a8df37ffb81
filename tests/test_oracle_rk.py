"""Pins of the oracle's IMEX Runge-Kutta stepper (Sec. IX "Runge-Kutta IMEX
integrators") against what the mathematics fixes:

* the order conditions of the tableaus (both halves of the IMEX pair and the
  coupling conditions for third order);
* the closed-form solution of a linear problem (pure diffusion of a
  horizontally uniform b, for which the explicit term vanishes): observed
  orders 1, 2, 3;
* a nonlinear convecting state against a Richardson-extrapolated SBDF2
  reference (SBDF2 is pinned on its own): observed orders 2 and about 3 (the
  algebraic constraints of the first-order system cost the third-order scheme
  a little order at these step sizes);
* RK111 is backward/forward Euler, which is the SBDF1 step.
"""
import math

import numpy as np
import pytest

import seeded_inputs as si
from oracle import RBOracle, RBParams, rk_tableau

ORDERS = {"RK111": 1, "RK222": 2, "RK443": 3}


@pytest.mark.parametrize("scheme", list(ORDERS))
def test_tableau_order_conditions(scheme):
    H, A, c = rk_tableau(scheme)
    p = ORDERS[scheme]
    s = len(c) - 1
    # explicit half strictly lower triangular; implicit half zero first column
    assert np.all(np.triu(A) == 0)
    assert np.all(H[:, 0] == 0) and np.all(np.triu(H, 1) == 0)
    # both halves share the stage times (row sums)
    np.testing.assert_allclose(A.sum(axis=1), c, atol=1e-15)
    np.testing.assert_allclose(H.sum(axis=1), c, atol=1e-15)
    bE, bI = A[s], H[s]  # globally stiffly accurate: the last stage is the step
    assert c[s] == 1.0
    for b in (bE, bI):
        assert abs(b.sum() - 1.0) < 1e-15
        if p >= 2:
            assert abs(b @ c - 0.5) < 1e-15
        if p >= 3:
            assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-15
            for Q in (A, H):  # coupling conditions of the IMEX pair
                assert abs(b @ Q @ c - 1.0 / 6.0) < 1e-15


def _orders(errs):
    return [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]


@pytest.mark.parametrize("scheme", list(ORDERS))
def test_linear_diffusion_closed_form(scheme):
    """b = 1 - z + a sin(pi z), u = w = 0, no x dependence: the explicit term
    is zero and b evolves by the heat equation with kappa = 1 (Ra = Pr = 1):
    b(t) = 1 - z + a exp(-pi^2 t) sin(pi z)."""
    Nx, Nz, a, T = 8, 32, 0.3, 0.1
    o = RBOracle(Nx, Nz, 4.0, RBParams(1.0, 1.0))
    _, z = o.scale1_grids()

    def state(t):
        prof = 1.0 - z + a * math.exp(-math.pi ** 2 * t) * np.sin(math.pi * z)
        return o.state_from_b_grid(np.broadcast_to(prof[None, :], (Nx, Nz)).copy())

    X0, Xe = state(0.0), state(T)
    ib = o.vi["b"]
    errs = []
    for n in (4, 8, 16, 32):
        X = X0
        for _ in range(n):
            X = o.step_rk(X, T / n, scheme)
        errs.append(np.linalg.norm(X[:, ib] - Xe[:, ib]) / np.linalg.norm(Xe[:, ib]))
        assert np.abs(X[:, o.vi["u"]]).max() < 1e-15 and np.abs(X[:, o.vi["w"]]).max() < 1e-15
    p = ORDERS[scheme]
    assert min(_orders(errs)) > p - 0.1, (scheme, errs)
    assert errs[-1] < {1: 2e-3, 2: 5e-6, 3: 1e-7}[p], errs


@pytest.fixture(scope="module")
def convecting():
    """A 16x16 convecting state (Ra = 1e4, above onset) reached by 150 SBDF2
    steps from a perturbed conduction profile, and the Richardson-extrapolated
    SBDF2 solution at T = 0.2 (800 and 1600 steps)."""
    Nx, Nz = 16, 16
    o = RBOracle(Nx, Nz, 2.0, RBParams(1e4, 1.0))
    X = o.initial_state(si.workload_noise((Nx, Nz), 3), amp=1.0)
    X = o.run(X, 2e-2, 150)
    T = 0.2

    def sbdf2(n):
        o.reset()
        Y = X
        for _ in range(n):
            Y = o.step(Y, T / n)
        return Y

    r1, r2 = sbdf2(800), sbdf2(1600)
    ref = (4.0 * r2 - r1) / 3.0
    assert np.linalg.norm(r2 - ref) / np.linalg.norm(ref) < 2e-9
    return o, X, T, ref


@pytest.mark.parametrize("scheme,min_order,max_err", [("RK222", 1.9, 5e-7), ("RK443", 2.5, 5e-8)])
def test_nonlinear_convergence_against_sbdf2(convecting, scheme, min_order, max_err):
    o, X, T, ref = convecting
    sel = [o.vi[v] for v in ("b", "u", "w")]
    assert np.linalg.norm(X[:, o.vi["u"]]) > 1e-2  # the explicit term matters
    errs = []
    for n in (4, 8, 16):
        Y = X
        for _ in range(n):
            Y = o.step_rk(Y, T / n, scheme)
        errs.append(np.linalg.norm(Y[:, sel] - ref[:, sel]) / np.linalg.norm(ref[:, sel]))
    assert min(_orders(errs)) > min_order, (scheme, errs)
    assert errs[0] < max_err, errs


def test_rk111_is_sbdf1():
    Nx, Nz, dt = 16, 16, 1e-2
    o = RBOracle(Nx, Nz, 2.0, RBParams(1e4, 1.0))
    X = o.initial_state(si.workload_noise((Nx, Nz), 4), amp=1.0)
    X = o.run(X, 2e-2, 20)
    o.reset()
    Xs = o.step(X, dt)            # first step of a run: SBDF1
    Xr = o.step_rk(X, dt, "RK111")
    assert np.linalg.norm(Xr - Xs) <= 1e-12 * np.linalg.norm(Xs)
