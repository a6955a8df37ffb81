"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
library routines it does not call (numpy.polynomial.chebyshev, numpy.fft),
closed forms, classical results, or brute force on tiny inputs.
"""
import math

import numpy as np
import numpy.polynomial.chebyshev as npc
import pytest

from oracle import RBOracle, RBParams, sbdf_coefficients, spectral as S, tau_poisson_bvp


# ---------------------------------------------------------------- transforms

@pytest.mark.parametrize("Nc,Ng", [(8, 8), (8, 12), (32, 48), (256, 384), (64, 96)])
def test_chebyshev_forward_of_Tm_is_unit_vector(Nc, Ng):
    # discrete orthogonality of T_n on the Gauss grid (Chebyshev basis, Sec. IV)
    x = S.cheb_grid(Ng)
    F = S.cheb_forward_matrix(Nc, Ng)
    for m in range(0, Nc, max(1, Nc // 7)):
        vals = npc.chebval(x, np.eye(Nc)[m])          # Clenshaw, library routine
        np.testing.assert_allclose(F @ vals, np.eye(Nc)[m], atol=1e-13 * max(1, Nc / 32))


@pytest.mark.parametrize("Nc,Ng", [(8, 12), (32, 48), (128, 192)])
def test_chebyshev_backward_matches_clenshaw(Nc, Ng):
    rng = np.random.default_rng(1)
    c = rng.standard_normal(Nc)
    x = S.cheb_grid(Ng)
    np.testing.assert_allclose(S.cheb_backward_matrix(Nc, Ng) @ c, npc.chebval(x, c),
                               atol=1e-13 * np.abs(c).sum())
    assert np.all(np.diff(x) > 0)            # ascending grid
    assert abs(x[0] + math.cos(math.pi * 0.5 / Ng)) < 1e-15


@pytest.mark.parametrize("Nc,Ng", [(8, 12), (64, 96), (1024, 1536)])
def test_fourier_real_transforms_match_numpy_fft(Nc, Ng):
    rng = np.random.default_rng(2)
    g = rng.standard_normal(Ng)
    c = S.fourier_real_forward_matrix(Nc, Ng) @ g
    ref = np.fft.rfft(g)[: Nc // 2] / Ng
    np.testing.assert_allclose(c, ref, atol=1e-14 * np.abs(ref).max() * math.log2(Ng))
    # backward of a half spectrum (k < Nc/2, k = 0 real) against irfft of the padded spectrum
    h = rng.standard_normal(Nc // 2) + 1j * rng.standard_normal(Nc // 2)
    h[0] = h[0].real
    full = np.zeros(Ng // 2 + 1, dtype=complex)
    full[: Nc // 2] = h
    ref_g = np.fft.irfft(full, n=Ng) * Ng
    np.testing.assert_allclose(np.real(S.fourier_real_backward_matrix(Nc, Ng) @ h), ref_g,
                               atol=1e-13 * np.abs(h).sum())


def test_fourier_mode_is_unit_coefficient():
    Nc, Ng = 16, 24
    x = 2 * np.pi * np.arange(Ng) / Ng
    F = S.fourier_real_forward_matrix(Nc, Ng)
    for k in range(Nc // 2):
        c = F @ np.cos(k * x)
        exp = np.zeros(Nc // 2)
        exp[k] = 1.0 if k == 0 else 0.5
        np.testing.assert_allclose(c, exp, atol=1e-15)
    # the Nyquist mode of the scale-1 grid is dropped
    F1 = S.fourier_real_forward_matrix(Nc, Nc)
    x1 = 2 * np.pi * np.arange(Nc) / Nc
    assert np.abs(F1 @ np.cos(Nc // 2 * x1)).max() < 1e-14


def test_fourier_complex_transforms_match_numpy_fft():
    Nc, Ng = 12, 18
    rng = np.random.default_rng(3)
    g = rng.standard_normal(Ng) + 1j * rng.standard_normal(Ng)
    c = S.fourier_complex_forward_matrix(Nc, Ng) @ g
    ref = np.fft.fft(g) / Ng
    k = S.fourier_signed_wavenumbers(Nc)
    act = S.fourier_complex_active(Nc)
    np.testing.assert_allclose(c[act], ref[k[act] % Ng], atol=1e-14)
    assert c[~act].tolist() == [0.0]


# ------------------------------------------------------- operator identities

@pytest.mark.parametrize("N", [4, 9, 32])
def test_conversion_and_derivative_by_evaluation(N):
    # <U_i|T_j> and <U_i|dT_j> checked by evaluating U_n(x) = sin((n+1)t)/sin(t)
    rng = np.random.default_rng(4)
    a = rng.standard_normal(N)
    th = rng.uniform(0.1, 3.0, 17)
    x = np.cos(th)
    U = np.sin(np.outer(th, np.arange(1, N + 1))) / np.sin(th)[:, None]
    np.testing.assert_allclose(U @ (S.cheb_conversion_TU(N) @ a), npc.chebval(x, a), atol=1e-11)
    np.testing.assert_allclose(U @ (S.cheb_diff_TU(N) @ a), npc.chebval(x, npc.chebder(a)),
                               atol=1e-10 * N * N)


@pytest.mark.parametrize("N", [5, 16, 33])
def test_identity_PL_DTT_equals_DTU(N):
    DTT = S.cheb_diff_TT(N)
    for j in range(N):      # T-to-T derivative against numpy's chebder
        np.testing.assert_allclose(DTT[:, j], np.r_[npc.chebder(np.eye(N)[j]), np.zeros(1)][:N],
                                   atol=1e-12)
    np.testing.assert_allclose(S.cheb_conversion_TU(N) @ DTT, S.cheb_diff_TU(N), atol=1e-12)
    D = S.cheb_diff_TU(N)
    assert all(D[n - 1, n] == n for n in range(1, N))


def test_dirichlet_recombination_and_interpolation():
    N = 12
    PR = S.cheb_dirichlet_PR(N)
    for side, x in (("left", -1.0), ("right", 1.0)):
        row = S.cheb_interp_row(N, side)
        np.testing.assert_allclose(row, npc.chebval(x, np.eye(N)))
        vals = row @ PR                                      # D_n(+-1)
        np.testing.assert_allclose(vals[2:], 0.0, atol=0)
        np.testing.assert_allclose(vals[:2], [1.0, x])


def test_integration_vector():
    N = 10
    w = S.cheb_integ_row(N)
    for n in range(N):
        ref = npc.chebval(1.0, npc.chebint(np.eye(N)[n])) - npc.chebval(-1.0, npc.chebint(np.eye(N)[n]))
        assert abs(w[n] - ref) < 1e-14


# --------------------------------------------------------------- dealiasing

def _brute_product_2d(cf, cg, Nx, N):
    """Exact product of two real fields given by half spectra (kx>=0, n<N):
    full Fourier convolution and numpy's chebmul, truncated to kx<Nx/2, n<N."""
    K = cf.shape[0]

    def full(c):
        d = {}
        for k in range(K):
            d[k] = c[k]
            if k:
                d[-k] = np.conj(c[k])
        return d

    F, G = full(cf), full(cg)
    out = np.zeros((Nx // 2, N), dtype=complex)
    for k1, a in F.items():
        for k2, b in G.items():
            k = k1 + k2
            if 0 <= k < Nx // 2:
                pr = npc.chebmul(a.real, b.real) - npc.chebmul(a.imag, b.imag) \
                    + 1j * (npc.chebmul(a.real, b.imag) + npc.chebmul(a.imag, b.real))
                out[k] += pr[:N] if pr.size >= N else np.r_[pr, np.zeros(N - pr.size)]
    return out


def test_dealiased_product_is_exact_truncated_product():
    Nx, N = 8, 6
    o = RBOracle(Nx, N, 2 * np.pi, RBParams(1e4, 1.0))
    rng = np.random.default_rng(5)
    a = rng.standard_normal((Nx // 2, N)) + 1j * rng.standard_normal((Nx // 2, N))
    b = rng.standard_normal((Nx // 2, N)) + 1j * rng.standard_normal((Nx // 2, N))
    a[0] = a[0].real
    b[0] = b[0].real
    A = np.zeros((o.Px, N), complex)
    B = np.zeros((o.Px, N), complex)
    A[: Nx // 2], B[: Nx // 2] = a, b
    got = o.from_grid(o.to_grid(A) * o.to_grid(B))
    ref = _brute_product_2d(a, b, Nx, N)
    np.testing.assert_allclose(got[: Nx // 2], ref, atol=1e-12)
    assert np.all(got[Nx // 2] == 0)
    # without padding the same product aliases
    o1 = RBOracle(Nx, N, 2 * np.pi, RBParams(1e4, 1.0), dealias=1.0)
    bad = o1.from_grid(o1.to_grid(A) * o1.to_grid(B))
    assert np.abs(bad[: Nx // 2] - ref).max() > 1e-3


def test_nonlinear_term_against_brute_force_2d():
    Nx, N, Lx = 8, 6, 3.0
    o = RBOracle(Nx, N, Lx, RBParams(1e4, 1.0))
    rng = np.random.default_rng(6)
    X = rng.standard_normal(o.state_shape) + 1j * rng.standard_normal(o.state_shape)
    X[0] = X[0].real
    X[Nx // 2] = 0
    vi = o.vi
    kx = 2 * np.pi * np.arange(o.Px) / Lx
    h = lambda v: X[: Nx // 2, vi[v]]
    dx = lambda v: (1j * kx[: Nx // 2, None]) * h(v)
    got = o.nonlinear(X)
    for e, q in enumerate(("b", "u", "w")):
        ref = -(_brute_product_2d(h("u"), dx(q), Nx, N) + _brute_product_2d(h("w"), h(q + "z"), Nx, N))
        np.testing.assert_allclose(got[: Nx // 2, e], ref, atol=1e-11)


def test_nonlinear_term_3d_against_2d_embedding():
    # a 3-D state independent of y reproduces the 2-D nonlinear term
    Nx, Ny, N = 8, 6, 6
    o3 = RBOracle(Nx, N, 3.0, RBParams(1e4, 1.0), dim=3, Ny=Ny, Ly=2.0)
    o2 = RBOracle(Nx, N, 3.0, RBParams(1e4, 1.0))
    rng = np.random.default_rng(7)
    X2 = rng.standard_normal(o2.state_shape) + 1j * rng.standard_normal(o2.state_shape)
    X2[0] = X2[0].real
    X2[Nx // 2] = 0
    X3 = np.zeros(o3.state_shape, complex)
    for v in o2.vars:
        X3[0, :, o3.vi[v]] = X2[:, o2.vi[v]]
    got3 = o3.nonlinear(X3)
    got2 = o2.nonlinear(X2)
    m3 = {q: e for e, q in enumerate(o3.evolved)}
    for e, q in enumerate(o2.evolved):
        np.testing.assert_allclose(got3[0, :, m3[q]], got2[:, e], atol=1e-12)
    assert np.abs(got3[1:]).max() < 1e-13


def test_nonlinear_term_3d_y_derivative():
    # u = 0, w = 0, v = cos(y) only, q = sin(2y): N_q = -v dq/dy exactly
    Nx, Ny, N, Ly = 4, 8, 4, 2 * np.pi
    o = RBOracle(Nx, N, 2 * np.pi, RBParams(1e4, 1.0), dim=3, Ny=Ny, Ly=Ly)
    X = np.zeros(o.state_shape, complex)
    ky = S.fourier_signed_wavenumbers(Ny)
    iy = {int(k): i for i, k in enumerate(ky)}
    X[iy[1], 0, o.vi["v"], 0] = 0.5
    X[iy[-1], 0, o.vi["v"], 0] = 0.5
    X[iy[2], 0, o.vi["b"], 0] = -0.5j
    X[iy[-2], 0, o.vi["b"], 0] = 0.5j
    # -cos(y) * 2 cos(2y) = -(cos(3y) + cos(y))
    got = o.nonlinear(X)[:, 0, 0, 0]
    exp = np.zeros(Ny, complex)
    for k in (1, -1, 3, -3):
        exp[iy[k]] = -0.5
    np.testing.assert_allclose(got, exp, atol=1e-14)


# ------------------------------------------------------------ tau BVP pins

def test_poisson_tau_polynomial_exact():
    # u = x^2 - 2x - 3 satisfies u'' = 2, u(-1) = 0, u'(1) = 0 exactly
    for N in (3, 4, 8, 16):
        f = np.zeros(N)
        f[0] = 2.0
        u = tau_poisson_bvp(N, f)
        exp = np.zeros(N)
        exp[:3] = npc.poly2cheb([-3.0, -2.0, 1.0])
        np.testing.assert_allclose(u, exp, atol=1e-13)


def test_poisson_tau_spectral_convergence():
    # u = sin(pi (x+1)/4): u(-1)=0, u'(1)=0, u'' = -(pi/4)^2 u
    errs = []
    xs = np.linspace(-1, 1, 101)
    for N in (8, 16, 24):
        f = npc.chebinterpolate(lambda x: -(np.pi / 4) ** 2 * np.sin(np.pi * (x + 1) / 4), N - 1)
        u = tau_poisson_bvp(N, f)
        errs.append(np.abs(npc.chebval(xs, u) - np.sin(np.pi * (xs + 1) / 4)).max())
    assert errs[0] < 1e-5 and errs[1] < 1e-12 and errs[2] < 1e-13
    assert errs[1] < errs[0] * 1e-5


# ----------------------------------------------------------- time stepping

def test_sbdf_coefficients_consistency():
    for w in (1.0, 0.5, 2.0):
        a0, a1, a2, b0, c1, c2 = sbdf_coefficients(1, 1e-2 * w, 1e-2)
        dt = 1e-2 * w
        # exact for polynomials of degree <= 2 in t: sum a_j y(t_{n-j}) = y'(t_n)
        t = np.array([0.0, -dt, -dt - 1e-2])
        for p in (0, 1, 2):
            lhs = a0 * t[0] ** p + a1 * t[1] ** p + a2 * t[2] ** p
            rhs = 0.0 if p != 1 else 1.0
            assert abs(lhs - rhs) < 1e-10 * max(1, abs(a0))
        assert abs(c1 + c2 - 1) < 1e-15 and b0 == 1.0
    a0, a1, a2, b0, c1, c2 = sbdf_coefficients(1, 0.1, 0.1)
    assert np.allclose([a0 * 0.1, a1 * 0.1, a2 * 0.1, c1, c2], [1.5, -2.0, 0.5, 2.0, -1.0])


def _diffusion_setup(dim=2):
    par = RBParams(1e4, 1.0, buoyancy=0.0)
    if dim == 2:
        o = RBOracle(16, 24, 4.0, par)
    else:
        o = RBOracle(8, 24, 4.0, par, dim=3, Ny=8, Ly=3.0)
    N = o.Nz
    s = npc.chebinterpolate(lambda x: np.sin(np.pi * (x + 1) / 2), 60)[:N]
    cz = npc.chebinterpolate(lambda x: np.pi * np.cos(np.pi * (x + 1) / 2), 60)[:N]
    return o, s, cz


@pytest.mark.parametrize("dim", [2, 3])
def test_diffusion_mode_decays_by_sbdf_recurrence(dim):
    o, s, cz = _diffusion_setup(dim)
    eps, m, dt = 1e-2, 2, 2e-2
    X = np.zeros(o.state_shape, complex)
    mean = (0,) if dim == 2 else (0, 0)
    if dim == 2:
        key = (m,)
        k2 = (2 * np.pi * m / o.Lx) ** 2
    else:
        ky = S.fourier_signed_wavenumbers(o.Ny)
        iy = int(np.where(ky == -1)[0][0])
        key = (iy, m)
        k2 = (2 * np.pi * m / o.Lx) ** 2 + (2 * np.pi / o.Ly) ** 2
    X[mean + (o.vi["b"], 0)] = 0.5
    X[mean + (o.vi["b"], 1)] = -0.5
    X[mean + (o.vi["bz"], 0)] = -1.0
    X[key + (o.vi["b"],)] = 0.5 * eps * s
    X[key + (o.vi["bz"],)] = 0.5 * eps * cz
    lam = -o.par.kappa * (k2 + np.pi ** 2)
    y = [1.0]
    for n in range(12):
        X = o.step(X, dt)
        if n == 0:
            y.append(y[0] / (1 - lam * dt))
        else:
            y.append((2 * y[-1] - 0.5 * y[-2]) / (1.5 - lam * dt))
        np.testing.assert_allclose(X[key + (o.vi["b"],)], 0.5 * eps * y[-1] * s, atol=1e-14)
        np.testing.assert_allclose(X[key + (o.vi["bz"],)], 0.5 * eps * y[-1] * cz, atol=1e-13)
    np.testing.assert_allclose(X[mean + (o.vi["b"],)][:2], [0.5, -0.5], atol=1e-14)
    assert np.abs(X[..., [o.vi["u"], o.vi["w"], o.vi["p"]], :]).max() < 1e-14


def test_rb_onset_critical_rayleigh():
    # no-slip, fixed-temperature onset: Ra_c = 1707.76 at k_c = 3.117 (classical)
    def growth(Ra, k=3.117):
        o = RBOracle(8, 32, 4.0, RBParams(Ra, 1.0))
        return o.linear_growth_rate(k)
    assert growth(1650.0) < 0 < growth(1770.0)
    lo, hi = 1650.0, 1770.0
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        if growth(mid) > 0:
            hi = mid
        else:
            lo = mid
    assert abs(0.5 * (lo + hi) - 1707.76) / 1707.76 < 1e-3


def test_rb_onset_3d_depends_on_horizontal_wavenumber_magnitude():
    o = RBOracle(8, 24, 4.0, RBParams(1800.0, 1.0), dim=3, Ny=8, Ly=4.0)
    g1 = o.linear_growth_rate(3.117, 0.0)
    g2 = o.linear_growth_rate(3.117 / math.sqrt(2), 3.117 / math.sqrt(2))
    assert g1 > 0 and abs(g1 - g2) < 1e-9


def test_linear_ivp_growth_matches_eigenvalue():
    # Ra above onset, k = pi (Lx = 2): the SBDF2 IVP amplitude grows at the EVP rate
    Ra = 2500.0
    o = RBOracle(4, 24, 2.0, RBParams(Ra, 1.0))
    sigma = o.linear_growth_rate(np.pi)
    M, L = o.linearized_matrices(np.pi, 0.0)
    import scipy.linalg as sla
    w, V = sla.eig(L.toarray(), -M.toarray())
    i = int(np.nanargmax(np.where(np.isfinite(w) & (np.abs(w) < 1e8), w.real, -np.inf)))
    v = V[:, i] / np.abs(V[:, i]).max() * 1e-8
    X = np.zeros(o.state_shape, complex)
    X[1] = v.reshape(o.S, o.Nz)
    X[0, o.vi["b"], :2] = [0.5, -0.5]
    X[0, o.vi["bz"], 0] = -1.0
    dt, steps = 2e-3, 200
    bi = o.vi["b"]
    amp0 = np.abs(X[1, bi]).max()
    X = o.run(X, dt, steps)
    rate = math.log(np.abs(X[1, bi]).max() / amp0) / (dt * steps)
    assert sigma > 0
    assert abs(rate - sigma) / sigma < 2e-3


def test_sbdf2_second_order_in_time():
    o_ref = None
    par = RBParams(2e4, 1.0)

    def run(dt, steps):
        o = RBOracle(16, 16, 2.0, par)
        x, z = o.scale1_grids()
        b = (1 - z)[None, :] + 0.05 * np.cos(np.pi * x)[:, None] * np.sin(np.pi * z)[None, :]
        X = o.state_from_b_grid(b)
        return o.run(X, dt, steps)

    T, base = 0.8, 0.05
    ref = run(base / 16, 16 * 16)
    errs = [np.abs(run(base / m, int(T / (base / m) + 0.5)) - ref).max() for m in (1, 2, 4)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.3 < r2 < 4.7, (errs, r1, r2)


def test_superlu_and_dense_pencil_solves_agree():
    par = RBParams(1e5, 1.0)
    Xs = []
    for solver in ("dense", "superlu"):
        o = RBOracle(8, 16, 4.0, par, solver=solver)
        rng = np.random.default_rng(9)
        X = o.initial_state(rng.standard_normal((8, 16)), amp=1e-2)
        Xs.append(o.run(X, 1e-2, 3))
    np.testing.assert_allclose(Xs[0], Xs[1], atol=1e-13)


def test_step_solution_satisfies_bcs_and_constraints():
    o = RBOracle(16, 16, 4.0, RBParams(1e5, 1.0))
    rng = np.random.default_rng(10)
    X = o.run(o.initial_state(rng.standard_normal((16, 16)), amp=1e-1), 1e-2, 3)
    vi = o.vi
    left, right = S.cheb_interp_row(16, "left"), S.cheb_interp_row(16, "right")
    b = X[:, vi["b"]]
    assert abs(b[0] @ left - 1.0) < 1e-13 and abs(b[0] @ right) < 1e-13
    assert np.abs(b[1:] @ left).max() < 1e-13 and np.abs(b[1:] @ right).max() < 1e-13
    for q in ("u", "w"):
        assert np.abs(X[:, vi[q]] @ left).max() < 1e-13
    assert np.abs(X[1:, vi["w"]] @ right).max() < 1e-13
    assert abs(X[0, vi["p"]] @ right) < 1e-13            # gauge
    kx = 2 * np.pi * np.arange(o.Px) / o.Lx
    div = 1j * kx[:, None] * X[:, vi["u"]] + X[:, vi["wz"]]
    assert np.abs(div).max() < 1e-12
    assert np.abs(X[o.Px - 1]).max() == 0.0              # Nyquist slot


# ----------------------------------------------------- initial condition, J

def test_initial_state_consistency():
    o = RBOracle(16, 16, 4.0, RBParams(1e4, 1.0))
    rng = np.random.default_rng(11)
    xi = rng.standard_normal((16, 16))
    X = o.initial_state(xi)
    bz_ref = np.array([2.0 * np.r_[npc.chebder(c.real) + 1j * npc.chebder(c.imag), 0] for c in X[:, o.vi["b"]]])
    np.testing.assert_allclose(X[:, o.vi["bz"]], bz_ref, atol=1e-12)
    # grid round trip at scale 1 reproduces the grid up to the dropped Nyquist column
    g = o.initial_b_grid(xi)
    back = o.coeff_to_grid_scale1(X[:, o.vi["b"]])
    nyq = np.fft.rfft(g, axis=0)[8] / 16
    x = o.Lx * np.arange(16) / 16
    resid = g - back - np.real(nyq[None, :] * np.exp(1j * 2 * np.pi * 8 * x / o.Lx)[:, None])
    assert np.abs(resid).max() < 1e-13


def test_kinetic_energy_closed_forms():
    o = RBOracle(16, 8, 4.0, RBParams(1e4, 1.0))
    X = np.zeros(o.state_shape, complex)
    X[0, o.vi["u"], 1] = 1.0                      # u = 2z - 1: J = 1/6
    assert abs(o.kinetic_energy(X) - 1.0 / 6.0) < 1e-15
    X[:] = 0
    X[3, o.vi["w"], 0] = 0.5 * 0.3                # w = 0.3 cos(k x): J = 0.3^2 / 4
    assert abs(o.kinetic_energy(X) - 0.09 / 4) < 1e-15
