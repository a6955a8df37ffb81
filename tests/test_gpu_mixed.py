"""Mixed-precision step (FP32 transforms and products; FP64 factorisation,
pencil solve and boundary rows) against the
FP64 oracle, per field.  The Chebyshev transforms run either as FP32 FFTs or
as split-BF16 matrix-core products with FP32 accumulation; both are checked.

Stated bound: relative L2 error per field at most 1e-5 after the trajectories
below.  The FP64 component calls (stau_nonlinear, stau_solve) are unaffected by
the precision mode; that is checked too.
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

MIXED_BOUND = 1e-5
C1 = (64, 32, 4.0, 1e4, 1.0, 1e-3)


def _to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("cfg,steps,dct", [(C1, 100, "fft"), ((128, 64, 4.0, 1e6, 1.0, 1e-4), 20, "fft"),
                                           ((128, 64, 4.0, 1e6, 1.0, 1e-4), 20, "matmul"),
                                           ((32, 128, 2.0, 1e7, 7.0, 2e-5), 10, "fft"),
                                           ((32, 128, 2.0, 1e7, 7.0, 2e-5), 10, "matmul"),
                                           ((16, 256, 2.0, 1e8, 1.0, 1e-5), 5, "matmul")],
                         ids=["C1-fft", "128x64-fft", "128x64-bf16", "32x128-fft", "32x128-bf16",
                              "16x256-bf16"])
def test_mixed_trajectory_within_bound(cfg, steps, dct):
    Nx, Nz, Lx, Ra, Pr, dt = cfg
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, precision="mixed", dct=dct)
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    xi = si.workload_noise((Nx, Nz), 0)
    Xo = o.initial_state(xi)
    g.initial_state(torch.from_numpy(o.initial_b_grid(xi)))
    for _ in range(steps):
        Xo = o.step(Xo, dt)
        g.step(dt)
    errs = field_errors(o, _to_np(g.X), Xo)
    print("mixed per-field error", cfg, {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) < MIXED_BOUND, errs
    # the reduced precision is visible: not the FP64 result bit for bit
    assert max(errs.values()) > 1e-15


@pytest.mark.parametrize("dct", ["fft", "matmul"])
def test_mixed_full_size_one_step_sampled_pencils(dct):
    """Nx=1024, Nz=256, Ra=1e8, dt=1e-5: one SBDF1 step of the mixed path from
    the oracle's seeded state, compared on sampled pencils."""
    Nx, Nz, Lx, Ra, Pr, dt = 1024, 256, 4.0, 1e8, 1.0, 1e-5
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, precision="mixed", dct=dct)
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    xi = si.workload_noise((Nx, Nz), 1)
    X0 = o.initial_state(xi)
    g.set_state(torch.from_numpy(X0).cuda())
    g.step(dt)
    Xg = _to_np(g.X)
    F = o.nonlinear(X0)
    a0, a1 = 1.0 / dt, -1.0 / dt
    sample = [(0,), (1,), (77,), (510,), (511,)]
    Bev = np.zeros((o.Px, o.ne, Nz), complex)
    for key in sample:
        M, L = o.pencil_matrices(2 * np.pi * key[0] / Lx, 0.0, key[0] == 0)
        Ft = o.precondition_rhs(F[key], key[0] == 0)
        B = Ft - a1 * (M @ X0[key].reshape(-1))
        for e in range(o.ne):
            Bev[key][e, : Nz - 1] = B[e * Nz: e * Nz + Nz - 1]
    Xo = oracle_solve_from_ev(o, Bev, a0, 1.0, pencils=set(sample))
    for key in sample:
        errs = {v: rel_err(Xg[key][i], Xo[key][i]) for i, v in enumerate(o.vars)
                if np.linalg.norm(Xo[key][i]) > 0}
        print("mixed full-size pencil", key, {k: f"{v:.2e}" for k, v in errs.items()})
        assert rel_err(Xg[key], Xo[key]) < MIXED_BOUND, key


def test_mixed_mode_leaves_fp64_components_exact():
    Nx, Nz, Lx, Ra, Pr, dt = C1
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, precision="mixed")
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    g.factor(1.0 / dt, 1.0)
    Bev = si.complex_noise(g.ev_shape, 12)
    Bev[0] = Bev[0].real
    Xg = _to_np(g.solve(torch.from_numpy(Bev).cuda()))
    Xo = oracle_solve_from_ev(o, Bev, 1.0 / dt, 1.0)
    assert max(field_errors(o, Xg, Xo).values()) < 1e-11


def test_mixed_matmul_rejects_unsupported_nz():
    """The split-BF16 products cover Nz = 64, 128, 256; Nz = 32 is refused
    for the mixed step (the FP64 products accept it)."""
    with pytest.raises(RuntimeError, match="Nz = 64, 128 or 256"):
        RBSolver(64, 32, 4.0, 1e4, 1.0, precision="mixed", dct="matmul")
    RBSolver(64, 32, 4.0, 1e4, 1.0, precision="fp64", dct="matmul")


@pytest.mark.parametrize("cfg,steps,dct", [(C1, 100, "fft"), ((128, 64, 4.0, 1e6, 1.0, 1e-4), 20, "matmul"),
                                           ((32, 128, 2.0, 1e7, 7.0, 2e-5), 10, "fft")],
                         ids=["C1-fft", "128x64-bf16", "32x128-fft"])
def test_refined_solve_trajectory_within_bound(cfg, steps, dct):
    """Mixed steps whose pencil solve is FP32 sweeps with one FP64 refinement
    (mixed_solve='refined'), against the FP64 oracle; the FP64 residual makes
    the solve's own error negligible next to the FP32 transforms'."""
    Nx, Nz, Lx, Ra, Pr, dt = cfg
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, precision="mixed", dct=dct, mixed_solve="refined")
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr))
    xi = si.workload_noise((Nx, Nz), 0)
    Xo = o.initial_state(xi)
    g.initial_state(torch.from_numpy(o.initial_b_grid(xi)))
    for _ in range(steps):
        Xo = o.step(Xo, dt)
        g.step(dt)
    errs = field_errors(o, _to_np(g.X), Xo)
    print("refined mixed per-field error", cfg, {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) < MIXED_BOUND, errs


def test_refined_solve_3d_and_rk():
    """3-D mixed steps and a mixed RK443 step with the refined solve."""
    Nx, Ny, Nz, Lx, Ly, Ra, Pr, dt = 16, 8, 16, 4.0, 4.0, 1e5, 1.0, 5e-4
    o = RBOracle(Nx, Nz, Lx, RBParams(Ra, Pr), dim=3, Ny=Ny, Ly=Ly)
    g = RBSolver(Nx, Nz, Lx, Ra, Pr, dim=3, Ny=Ny, Ly=Ly, precision="mixed", mixed_solve="refined")
    xi = si.workload_noise((Nx, Ny, Nz), 0)
    Xo = o.initial_state(xi, amp=1e-2)
    g.initial_state(torch.from_numpy(o.initial_b_grid(xi, amp=1e-2)))
    for _ in range(10):
        Xo = o.step(Xo, dt)
        g.step(dt)
    errs = field_errors(o, _to_np(g.X), Xo)
    assert max(errs.values()) < MIXED_BOUND, errs
    Xr = o.step_rk(Xo, dt, "RK443")
    g.set_state(torch.from_numpy(Xo).cuda())
    g.step_rk(dt, "RK443")
    errs = field_errors(o, _to_np(g.X), Xr)
    assert max(errs.values()) < MIXED_BOUND, errs


@pytest.mark.parametrize("shape", [(16, 8, 16), (2048, 1, 16)], ids=["3d-16x8x16", "2d-2048x16"])
def test_refined_solve_is_taken_in_the_single_block_layout(shape):
    """The refined solve must run where the pencils use the single-block
    layout (3-D, and 2-D domains with more pencils than two per compute
    unit): one step differs from the FP64-solve mixed step in the last bits
    and agrees with it to the refinement's accuracy."""
    Nx, Ny, Nz = shape
    dim = 3 if Ny > 1 else 2
    kw = dict(dim=3, Ny=Ny, Ly=4.0) if dim == 3 else {}
    ga = RBSolver(Nx, Nz, 4.0, 1e5, 1.0, precision="mixed", mixed_solve="fp64", **kw)
    gr = RBSolver(Nx, Nz, 4.0, 1e5, 1.0, precision="mixed", mixed_solve="refined", **kw)
    xi = si.workload_noise((Nx, Ny, Nz) if dim == 3 else (Nx, Nz), 0)
    o = RBOracle(Nx, Nz, 4.0, RBParams(1e5, 1.0), **({"dim": 3, "Ny": Ny, "Ly": 4.0} if dim == 3 else {}))
    X0 = torch.from_numpy(o.initial_state(xi, amp=1e-2)).cuda()
    ga.set_state(X0)
    gr.set_state(X0)
    ga.step(1e-4)
    gr.step(1e-4)
    a, r = _to_np(ga.X), _to_np(gr.X)
    d = np.abs(a - r).max() / np.abs(a).max()
    assert 0.0 < d < 1e-9, d


def test_mixed_solve_option_is_checked():
    from paper_1905_10388_amd import StauError, _lib
    import ctypes as C

    desc = _lib.DomainDesc(dim=2, precision=_lib.STAU_MIXED, Nx=64, Ny=1, Nz=32, Lx=4.0, Ly=1.0,
                           dealias=1.5, device=0, dct_method=0, mixed_solve=7)
    dom = C.c_void_p()
    lib = _lib.load()
    with pytest.raises(StauError, match="EINVAL"):
        _lib.check(lib.stau_create_domain(C.byref(desc), C.byref(dom)))
