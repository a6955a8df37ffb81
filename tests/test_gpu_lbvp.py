"""Linear boundary value solve (stau_lbvp) against the oracle's lbvp.

Bar: 1e-10 relative per field (the FP64 bar of the step).  At 1024x256 in the
launch configuration of the benchmark (two-block solve): sampled pencils of a
random right-hand side against the oracle's per-pencil solve, and the
conduction state (F = 0) against the oracle's mean pencil at Nx = 4 (a
horizontally uniform solution does not depend on Nx) with every other pencil
exactly zero.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import RBOracle, RBParams
from gpu_helpers import field_errors, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1905_10388_amd import RBSolver  # noqa: E402

BAR = 1e-10


def _to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _forcing(shape, N, seed):
    F = si.complex_noise(shape, seed) * np.exp(-np.arange(N) / (N / 8.0))
    return F


@pytest.mark.parametrize("cfg", [(64, 32, 4.0, 1e4, 1.0, "fp64"), (32, 128, 2.0, 1e7, 7.0, "fp64"),
                                 (64, 32, 4.0, 1e4, 1.0, "mixed")],
                         ids=["64x32", "32x128", "64x32-mixed-domain"])
def test_lbvp_matches_oracle(cfg):
    Nx, Nz, Lx, Ra, Pr, prec = cfg
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, precision=prec)
    F = _forcing(g.ev_shape, Nz, 21)
    F[0] = F[0].real  # the mean pencil of a real field
    Xg = _to_np(g.lbvp(torch.from_numpy(F)))
    Xo = o.lbvp(F)
    errs = field_errors(o, Xg, Xo)
    print("lbvp", cfg, {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) < BAR, errs


def test_lbvp_3d_matches_oracle():
    Nx, Ny, Nz, Lx, Ly, Ra, Pr = 16, 8, 16, 4.0, 4.0, 1e5, 1.0
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr), dim=3, Ny=Ny, Ly=Ly)
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, dim=3, Ny=Ny, Ly=Ly)
    F = _forcing(g.ev_shape, Nz, 22)
    F[0, 0] = F[0, 0].real
    Xg = _to_np(g.lbvp(torch.from_numpy(F)))
    Xo = o.lbvp(F)
    errs = field_errors(o, Xg, Xo)
    assert max(errs.values()) < BAR, errs


def test_lbvp_and_step_share_the_factor_cache():
    """lbvp, then SBDF steps (two other operators), then lbvp again: the same
    solution, and the steps unaffected by the solve in between."""
    Nx, Nz, Lx, Ra, Pr, dt = 64, 32, 4.0, 1e4, 1.0, 1e-3
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    g = RBSolver(Nx, Nz, Lx, Ra, Pr)
    F = _forcing(g.ev_shape, Nz, 23)
    F[0] = F[0].real
    X1 = _to_np(g.lbvp(torch.from_numpy(F)))
    xi = si.workload_noise((Nx, Nz), 0)
    Xo = o.initial_state(xi)
    g.initial_state(torch.from_numpy(o.initial_b_grid(xi)))
    for k in range(4):
        Xo = o.step(Xo, dt)
        g.step(dt)
        if k == 1:
            X2 = _to_np(g.lbvp(torch.from_numpy(F)))
    assert max(field_errors(o, _to_np(g.X), Xo).values()) < BAR
    assert np.array_equal(X1, X2)


FULL = (1024, 256, 4.0, 1e8, 1.0)


def test_full_size_lbvp_sampled_pencils():
    Nx, Nz, Lx, Ra, Pr = FULL
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    g = RBSolver(Nx, Nz, Lx, Ra, Pr)
    F = _forcing(g.ev_shape, Nz, 24)
    F[0] = F[0].real
    Xg = _to_np(g.lbvp(torch.from_numpy(F)))
    for ix in (0, 1, 77, 465, 511):
        kx = 2 * np.pi * ix / Lx
        solve = o.solver_for((ix,), kx, 0.0, ix == 0, 0.0, 1.0)
        Xo = solve(o.precondition_rhs(F[ix], ix == 0)).reshape(o.S, Nz)
        for i, v in enumerate(o.vars):
            if np.linalg.norm(Xo[i]) > 0:
                assert rel_err(Xg[ix, i], Xo[i]) < BAR, (ix, v)
    assert np.abs(Xg[Nx // 2]).max() == 0.0  # Nyquist slot


def test_full_size_conduction_state():
    Nx, Nz, Lx, Ra, Pr = FULL
    o = RBOracle(4, Nz, Lx, RBParams(Ra, Pr))
    g = RBSolver(Nx, Nz, Lx, Ra, Pr)
    Xg = _to_np(g.lbvp(torch.zeros(g.ev_shape, dtype=torch.complex128)))
    Xo = o.lbvp(np.zeros((3, o.ne, Nz), complex))
    assert np.abs(Xg[1:]).max() == 0.0
    scale = np.linalg.norm(Xo[0])
    for i, v in enumerate(o.vars):
        assert np.linalg.norm(Xg[0, i] - Xo[0, i]) < 1e-12 * scale, v
