"""Non-constant coefficient Gamma(z) w in the b equation (Sec. II, NCCs)
through every call that assembles the pencil operator: SBDF steps, the
Runge-Kutta step, the mixed-precision residual, the linear boundary value
solve, the linear-stability eigenvalues and the adjoint, against the oracle
(whose product matrix comes from numpy's Chebyshev multiplication).

Bars: those of the calls without the NCC (1e-10 FP64, 1e-5 mixed, 1e-9 for
eigenvalues and the 12-step gradient).  At 1024x256 in the benchmark's launch
configuration: one SBDF1 step on sampled pencils with a one-term Gamma
(two-block solve) and a three-term Gamma (whole-band solve, wider band)."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import RBOracle, RBParams
from oracle import adjoint as ADJ
from gpu_helpers import field_errors, oracle_solve_from_ev, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1905_10388_amd import RBSolver  # noqa: E402

GAMMAS = [(0.5,), (0.3, -0.2), (0.2, 0.15, -0.1)]
IDS = ["1-term", "2-term", "3-term"]


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _pair(cfg, gamma, **kw):
    Nx, Nz, Lx, Ra, Pr = cfg[:5]
    return (RBSolver(Nx, Nz, Lx, Ra, Pr, gamma=gamma, **kw),
            RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr, gamma=gamma)))


@pytest.mark.parametrize("gamma", GAMMAS, ids=IDS)
def test_ncc_sbdf_and_rk_trajectories(gamma):
    cfg = (64, 32, 4.0, 1e4, 1.0)
    dt = 2e-3
    g, o = _pair(cfg, gamma)
    X = o.initial_state(si.workload_noise(cfg[:2], 7), amp=0.5)
    g.set_state(torch.from_numpy(X).cuda())
    Xo = X
    for _ in range(8):
        Xo = o.step(Xo, dt)
        g.step(dt)
    e1 = field_errors(o, _np(g.X), Xo)
    for _ in range(3):
        Xo = o.step_rk(Xo, dt, "RK443")
        g.step_rk(dt, "RK443")
    e2 = field_errors(o, _np(g.X), Xo)
    print("ncc", gamma, max(e1.values()), max(e2.values()))
    assert max(e1.values()) < 1e-10 and max(e2.values()) < 1e-10, (e1, e2)


def test_ncc_mixed_within_bound():
    cfg = (128, 64, 4.0, 1e6, 1.0)
    g, o = _pair(cfg, GAMMAS[1], precision="mixed")
    X = o.initial_state(si.workload_noise(cfg[:2], 8), amp=0.2)
    g.set_state(torch.from_numpy(X).cuda())
    Xo = X
    for _ in range(10):
        Xo = o.step(Xo, 1e-4)
        g.step(1e-4)
    errs = field_errors(o, _np(g.X), Xo)
    assert 1e-15 < max(errs.values()) < 1e-5, errs


@pytest.mark.parametrize("gamma", GAMMAS, ids=IDS)
def test_ncc_lbvp_and_evp(gamma):
    cfg = (16, 32, 2.0, 1e4, 1.0)
    g, o = _pair(cfg, gamma)
    F = si.complex_noise(g.ev_shape, 25) * np.exp(-np.arange(32) / 4.0)
    F[0] = F[0].real
    errs = field_errors(o, _np(g.lbvp(torch.from_numpy(F))), o.lbvp(F))
    assert max(errs.values()) < 1e-10, errs
    sig, res, nconv, _, _ = g.evp(0.5, nev=3, tol=1e-10)
    sig, nconv = _np(sig), _np(nconv)
    for ix in range(8):
        assert nconv[ix] == 3, ix
        ref = o.stability_eigenvalues(2 * np.pi * ix / cfg[2], 0.0, 0.5, nev=3, is_mean=ix == 0)
        for x, y in zip(sorted(sig[ix], key=lambda z: z.real), sorted(ref, key=lambda z: z.real)):
            assert abs(x - y) < 1e-9 * max(1.0, abs(y)), (ix, sig[ix], ref)


def test_ncc_3d_step():
    Nx, Ny, Nz, Lx, Ly, Ra, Pr, dt = 16, 8, 16, 4.0, 4.0, 1e5, 1.0, 5e-4
    gamma = (0.3, -0.2)
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, dim=3, Ny=Ny, Ly=Ly, gamma=gamma)
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr, gamma=gamma), dim=3, Ny=Ny, Ly=Ly)
    X = o.initial_state(si.workload_noise((Nx, Ny, Nz), 2), amp=0.5)
    g.set_state(torch.from_numpy(X).cuda())
    Xo = X
    for _ in range(5):
        Xo = o.step(Xo, dt)
        g.step(dt)
    errs = field_errors(o, _np(g.X), Xo)
    assert max(errs.values()) < 1e-10, errs


def test_ncc_adjoint_gradient():
    Nx, Nz, Lx, Ra, Pr, dt, steps = 32, 16, 4.0, 2e4, 1.0, 5e-3, 12
    from paper_1905_10388_amd.adjoint import kinetic_energy_and_gradient
    gamma = (0.3, -0.2)
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, gamma=gamma)
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr, gamma=gamma))
    b0 = o.initial_b_grid(si.workload_noise((Nx, Nz), 3), amp=0.05)
    Jo, go = ADJ.gradient(o, b0, dt, steps)
    Jg, gg = kinetic_energy_and_gradient(g, torch.from_numpy(b0).cuda(), dt, steps, checkpoint=5)
    assert abs(Jg - Jo) <= 1e-10 * abs(Jo)
    assert rel_err(_np(gg), go) < 1e-9


def test_ncc_limits():
    from paper_1905_10388_amd._lib import StauError
    with pytest.raises(StauError, match="band too wide"):
        RBSolver(16, 16, 2.0, 1e4, 1.0, gamma=(0.1, 0.1, 0.1, 0.1))
    g = RBSolver(16, 16, 2.0, 1e4, 1.0, gamma=GAMMAS[2])  # forward fits, transposed does not
    Xb = torch.zeros(g.state_shape, dtype=torch.complex128, device="cuda")
    hb = torch.zeros((g.info["P"], 2, g.info["ne"], 16), dtype=torch.complex128, device="cuda")
    with pytest.raises(StauError, match="adjoint"):
        g.adjoint_step(g.X, 0, 1e-3, 1e-3, Xb, hb)
    with pytest.raises(ValueError):
        RBSolver(16, 16, 2.0, 1e4, 1.0, gamma=(0.1,) * 5)


@pytest.mark.parametrize("gamma", [GAMMAS[0], GAMMAS[2]], ids=["1-term-two-block", "3-term-whole-band"])
def test_ncc_full_size_one_step_sampled_pencils(gamma):
    Nx, Nz, Lx, Ra, Pr, dt = 1024, 256, 4.0, 1e8, 1.0, 1e-5
    g, o = _pair((Nx, Nz, Lx, Ra, Pr), gamma)
    X0 = o.initial_state(si.workload_noise((Nx, Nz), 1), amp=0.1)
    g.set_state(torch.from_numpy(X0).cuda())
    g.step(dt)
    Xg = _np(g.X)
    F = o.nonlinear(X0)
    sample = [(0,), (1,), (77,), (510,), (511,)]
    Bev = np.zeros((o.Px, o.ne, Nz), complex)
    for key in sample:
        M, L = o.pencil_matrices(2 * np.pi * key[0] / Lx, 0.0, key[0] == 0)
        B = o.precondition_rhs(F[key], key[0] == 0) + (M @ X0[key].reshape(-1)) / dt
        for e in range(o.ne):
            Bev[key][e, : Nz - 1] = B[e * Nz: e * Nz + Nz - 1]
    Xo = oracle_solve_from_ev(o, Bev, 1.0 / dt, 1.0, pencils=set(sample))
    for key in sample:
        assert rel_err(Xg[key], Xo[key]) < 1e-10, key
