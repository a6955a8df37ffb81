"""3-D (Fourier x, y x Chebyshev z) HIP path against the FP64 oracle.

Same bars as the 2-D parity tests: explicit term and pencil solve within the
transform / LU rounding, 1e-10 relative per field for a stepped trajectory,
and the mixed-precision step within its stated bound of 1e-5.
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import RBOracle, RBParams
from gpu_helpers import field_errors, oracle_solve_from_ev, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1905_10388_amd import RBSolver  # noqa: E402

# (Nx, Ny, Nz, Lx, Ly, Ra, Pr, dt)
SMALL3 = [(8, 8, 8, 4.0, 3.0, 1e4, 1.0, 1e-3), (16, 8, 16, 4.0, 4.0, 1e5, 1.0, 5e-4),
          (8, 16, 32, 2.0, 5.0, 1e6, 7.0, 1e-4)]


def _pair(cfg, **kw):
    Nx, Ny, Nz, Lx, Ly, Ra, Pr, dt = cfg
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, dim=3, Ny=Ny, Ly=Ly, **kw)
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr), dim=3, Ny=Ny, Ly=Ly)
    return g, o


def _random_state(o, seed):
    X = si.complex_noise(o.state_shape, seed)
    decay = np.exp(-np.arange(o.Nz) / (o.Nz / 6.0))
    return X * decay


def _to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _ids(c):
    return f"{c[0]}x{c[1]}x{c[2]}"


@pytest.mark.parametrize("cfg", SMALL3, ids=_ids)
def test_nonlinear_term_3d_matches_oracle(cfg):
    g, o = _pair(cfg)
    X = _random_state(o, 21)
    Fg = _to_np(g.nonlinear(torch.from_numpy(X).cuda()))
    Fo = o.nonlinear(X)
    assert Fg.shape == Fo.shape
    assert rel_err(Fg, Fo) < 1e-13
    assert np.all(Fg[:, o.Px - 1] == 0)
    assert np.all(Fg[o.Ny // 2] == 0)


@pytest.mark.parametrize("cfg", SMALL3, ids=_ids)
def test_pencil_solve_3d_matches_oracle(cfg):
    g, o = _pair(cfg)
    dt = cfg[-1]
    a0 = 1.5 / dt
    g.factor(a0, 1.0)
    Bev = si.complex_noise(g.ev_shape, 22)
    Xg = _to_np(g.solve(torch.from_numpy(Bev).cuda()))
    Xo = oracle_solve_from_ev(o, Bev, a0, 1.0)
    errs = field_errors(o, Xg, Xo)
    assert max(errs.values()) < 1e-11, errs
    assert np.all(Xg[:, o.Px - 1] == 0) and np.all(Xg[o.Ny // 2] == 0)


def test_initial_state_and_kinetic_energy_3d():
    cfg = SMALL3[1]
    Nx, Ny, Nz = cfg[:3]
    g, o = _pair(cfg)
    xi = si.workload_noise((Nx, Ny, Nz), 0)
    bgrid = o.initial_b_grid(xi)
    Xg = _to_np(g.initial_state(torch.from_numpy(bgrid)))
    Xo = o.initial_state(xi)
    eps = np.finfo(float).eps
    assert rel_err(Xg[..., o.vi["b"], :], Xo[..., o.vi["b"], :]) < 1e-14
    assert rel_err(Xg[..., o.vi["bz"], :], Xo[..., o.vi["bz"], :]) < 20 * Nz ** 2 * eps
    X = _random_state(o, 23)
    J = g.kinetic_energy(torch.from_numpy(X).cuda())
    Jo = o.kinetic_energy(X)
    assert abs(J - Jo) < 1e-13 * abs(Jo)


@pytest.mark.parametrize("cfg", SMALL3[:2], ids=_ids)
def test_step_trajectory_3d_matches_oracle(cfg):
    Nx, Ny, Nz, Lx, Ly, Ra, Pr, dt = cfg
    g, o = _pair(cfg)
    xi = si.workload_noise((Nx, Ny, Nz), 1)
    Xo = o.initial_state(xi, amp=1e-2)
    g.initial_state(torch.from_numpy(o.initial_b_grid(xi, amp=1e-2)))
    for _ in range(20):
        Xo = o.step(Xo, dt)
        g.step(dt)
    errs = field_errors(o, _to_np(g.X), Xo)
    assert max(errs.values()) < 1e-10, errs


def test_mixed_trajectory_3d_within_bound():
    cfg = SMALL3[1]
    Nx, Ny, Nz, Lx, Ly, Ra, Pr, dt = cfg
    g, o = _pair(cfg, precision="mixed")
    xi = si.workload_noise((Nx, Ny, Nz), 1)
    Xo = o.initial_state(xi, amp=1e-2)
    g.initial_state(torch.from_numpy(o.initial_b_grid(xi, amp=1e-2)))
    for _ in range(20):
        Xo = o.step(Xo, dt)
        g.step(dt)
    errs = field_errors(o, _to_np(g.X), Xo)
    print("mixed 3-D per-field error", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) < 1e-5, errs


def test_adjoint_rejects_3d():
    from paper_1905_10388_amd import StauError

    g, o = _pair(SMALL3[0])
    with pytest.raises(StauError):
        g.kinetic_energy_adjoint()


# --------------------------------------------------------------- full size
C3 = (256, 256, 128, 4.0, 4.0, 1e7, 1.0, 5e-5)


def test_full_size_3d_solve_sampled_pencils():
    """Nx=Ny=256, Nz=128 (33,024 pencil slots in one launch): the batched
    solve against the oracle's dense solve on sampled pencils."""
    g, o = _pair(C3)
    a0 = 1.5 / C3[-1]
    g.factor(a0, 1.0)
    Bev = si.complex_noise(g.ev_shape, 31)
    Xg = _to_np(g.solve(torch.from_numpy(Bev).cuda()))
    sample = {(0, 0), (0, 1), (1, 0), (5, 77), (255, 127), (129, 3), (127, 126)}
    Xo = oracle_solve_from_ev(o, Bev, a0, 1.0, pencils=sample)
    for key in sample:
        assert rel_err(Xg[key], Xo[key]) < 1e-11, key
    assert np.all(Xg[:, o.Px - 1] == 0) and np.all(Xg[o.Ny // 2] == 0)
    g.close()


def _swap_xy(o, R):
    """Coefficients of the x <-> y mirrored state (u <-> v, uz <-> vz) for
    Nx = Ny, Lx = Ly: c'(kx=b, ky=a) = c(kx=a, ky=b), using c(-k) = conj(c(k))."""
    Ny, Px = o.Ny, o.Px
    ky = o.ky_int
    iy_of = {int(k): i for i, k in enumerate(ky) if o.ky_act[i]}
    perm = [o.vi[v] for v in ("p", "b", "v", "u", "w", "bz", "vz", "uz", "wz")]
    out = np.zeros_like(R)
    for iy in range(Ny):
        if not o.ky_act[iy]:
            continue
        a = int(ky[iy])
        for b in range(o.kx_active):
            if a >= 0:
                src = R[iy_of[b], a] if b in iy_of else None
            else:
                src = np.conj(R[iy_of[-b], -a]) if -b in iy_of else None
            if src is not None:
                out[iy, b] = src[perm]
    return out


def test_full_size_3d_step_xy_mirror_symmetry():
    """Nx=Ny=256, Lx=Ly: one SBDF1 step from a seeded b grid and one from its
    x <-> y mirror give mirrored states (u <-> v) to rounding.  Exercises the
    y pass, the 15-field x pass and the 33,024-pencil solve at full size."""
    Nx, Ny, Nz, Lx, Ly, Ra, Pr, dt = C3
    g, o = _pair(C3)
    xi = si.workload_noise((Nx, Ny, Nz), 2)
    bgrid = o.initial_b_grid(xi, amp=1e-1)
    g.initial_state(torch.from_numpy(bgrid))
    Xu = si.complex_noise(g.state_shape, 32) * 1e-3 * np.exp(-np.arange(Nz) / 12.0)
    # a velocity field that is mirror-consistent: add (u, v) and its mirror
    X0 = _to_np(g.X)
    X0[..., o.vi["u"], :] += Xu[..., o.vi["u"], :]
    X0[..., o.vi["v"], :] += Xu[..., o.vi["v"], :]
    X0[:, 0] = 0.5 * (X0[:, 0] + np.conj(X0[[(-i) % Ny for i in range(Ny)], 0]))  # real on kx = 0
    X0[Ny // 2] = 0
    X0[:, o.Px - 1] = 0
    X0m = _swap_xy(o, X0)
    g.set_state(torch.from_numpy(X0).cuda())
    g.step(dt)
    R1 = _to_np(g.X)
    g.set_state(torch.from_numpy(X0m).cuda())
    g.step(dt)
    R2 = _to_np(g.X)
    g.close()
    errs = field_errors(o, R2, _swap_xy(o, R1))
    assert max(errs.values()) < 1e-11, errs
    assert rel_err(R1, X0) > 1e-8          # the step did change the state
