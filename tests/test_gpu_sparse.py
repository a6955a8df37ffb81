"""Sparse factor records (factor_layout "auto"): where the pencil solve streams
its vectors through device memory (single-block layout with more than 32
pencils per compute unit: 3-D domains of at least 8192 pencil slots) the
nonzero entries of the factors are packed into records after each
factorisation and the solve reads those instead of the whole band.

* The same values as the whole-band solve (factor_layout "band") over three
  steps (the SBDF1 and SBDF2 factor slots), in the component solve and the
  linear boundary value solve: a missing entry is a zero of the band, which
  only adds a zero product.  Shapes: 128 x 128 x 8 (72-row pencils, 9 record
  units), 64 x 256 x 32, 256 x 256 x 16 and the 3-D headline size
  256 x 256 x 128 (1152-row pencils, 144 units).
* The component solve on sampled pencils at 128 x 128 x 8 and 256 x 256 x 16
  against the oracle's matrices (backward error) and its dense solve, as the
  headline-size check in test_gpu_3d.py does at 256 x 256 x 128.
* The records are built only where they apply (the workspace grows by their
  size on the first factorisation).
"""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import RBOracle, RBParams
from gpu_helpers import oracle_solve_from_ev, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1905_10388_amd import RBSolver  # noqa: E402

RA, PR, DT = 1e7, 1.0, 5e-5


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _solver(Nx, Ny, Nz, layout):
    return RBSolver(Nx, Nz, 4.0, RA, PR, dim=3, Ny=Ny, Ly=4.0, factor_layout=layout)


@pytest.mark.parametrize("shape", [(128, 128, 8), (64, 256, 32), (256, 256, 16), (256, 256, 128)],
                         ids=lambda s: "x".join(map(str, s)))
def test_records_give_the_band_solve_values(shape):
    Nx, Ny, Nz = shape
    X0 = si.complex_noise((Ny, Nx // 2 + 1, 9, Nz), 80) * np.exp(-np.arange(Nz) / 4.0)
    X0[:, Nx // 2] = 0
    X0[Ny // 2] = 0
    X0[0, 0] = X0[0, 0].real
    B = si.complex_noise((Ny, Nx // 2 + 1, 4, Nz), 81)
    out = {}
    for layout in ("band", "auto"):
        g = _solver(Nx, Ny, Nz, layout)
        g.set_state(torch.from_numpy(X0).cuda())
        traj = []
        for _ in range(3):
            g.step(DT)
            traj.append(_np(g.X))
        g.factor(1.0 / DT)
        xs = _np(g.solve(torch.from_numpy(B).cuda()))
        xl = _np(g.lbvp(torch.from_numpy(B).cuda()))
        out[layout] = (traj, xs, xl)
        g.close()
        del g
        torch.cuda.empty_cache()
    for n in range(3):
        assert np.array_equal(out["auto"][0][n], out["band"][0][n]), (shape, n)
    assert np.array_equal(out["auto"][1], out["band"][1])
    assert np.array_equal(out["auto"][2], out["band"][2])
    assert np.isfinite(out["auto"][0][2]).all()


@pytest.mark.parametrize("shape", [(128, 128, 8), (256, 256, 16)], ids=lambda s: "x".join(map(str, s)))
def test_records_solve_matches_oracle_sampled_pencils(shape):
    """The component solve with the SBDF2 operator (records built by the
    factorisation) on sampled pencils against the oracle's matrices: the
    normwise backward error |A x - b| / (|A| |x| + |b|) below 1e-15, and the
    oracle's dense solve within 2e-11 relative, scaled up by cond(A) / 1e10
    where the pencil is worse conditioned (the short 8-mode pencils at the
    largest wavenumbers reach cond 9e11).  The headline size runs the same
    comparison in test_gpu_3d.py."""
    Nx, Ny, Nz = shape
    o = RBOracle(Nx, Nz, 4.0, RBParams(RA, PR), dim=3, Ny=Ny, Ly=4.0)
    g = _solver(Nx, Ny, Nz, "auto")
    a0 = 1.5 / DT
    g.factor(a0, 1.0)
    Bev = si.complex_noise(g.ev_shape, 33)
    Xg = _np(g.solve(torch.from_numpy(Bev).cuda()))
    g.close()
    sample = {(0, 0), (0, 1), (1, 0), (3, 17), (Ny - 1, Nx // 2 - 1), (Ny // 2 + 1, 5), (Ny // 2 - 1, Nx // 2 - 2)}
    Xo = oracle_solve_from_ev(o, Bev, a0, 1.0, pencils=sample)
    N = o.Nz
    for (iy, ix), kx, ky, is_mean, act in o.pencils():
        if (iy, ix) not in sample:
            continue
        M, L = o.pencil_matrices(kx, ky, is_mean)
        A = (a0 * M + L).toarray()
        b = np.zeros(o.S * N, dtype=np.complex128)
        for e in range(o.ne):
            b[e * N:e * N + N - 1] = Bev[iy, ix][e, :N - 1]
        for r, val in o.bc_values(is_mean).items():
            b[r] = val
        x = Xg[iy, ix].reshape(-1)
        berr = np.linalg.norm(A @ x - b) / (np.linalg.norm(A, 2) * np.linalg.norm(x) + np.linalg.norm(b))
        assert berr < 1e-15, ((iy, ix), berr)
        bar = 2e-11 * max(1.0, np.linalg.cond(A) / 1e10)
        assert rel_err(Xg[iy, ix], Xo[iy, ix]) < bar, ((iy, ix), rel_err(Xg[iy, ix], Xo[iy, ix]), bar)
    assert np.all(Xg[:, o.Px - 1] == 0) and np.all(Xg[Ny // 2] == 0)


def test_records_built_only_where_they_apply():
    """Workspace after a factorisation: 3-D at 8320 pencil slots holds the
    records, 3-D at 4160 slots does not, and the band layout never does."""
    def workspace(Nx, Ny, Nz, layout):
        g = _solver(Nx, Ny, Nz, layout)
        g.factor(1.0 / DT)
        ws = g.query()["workspace_bytes"]
        g.close()
        return ws

    many = (workspace(128, 128, 8, "auto"), workspace(128, 128, 8, "band"))
    few = (workspace(128, 64, 8, "auto"), workspace(128, 64, 8, "band"))
    # forward and backward records of 9 units per pencil, plus the lengths
    assert many[0] - many[1] >= 8320 * 9 * (32 + 64)
    assert few[0] == few[1]


def test_factor_layout_rejects_unknown_values():
    with pytest.raises(KeyError):
        _solver(8, 8, 8, "csr")
