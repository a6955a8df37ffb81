"""The entry point that allocates nothing (stau_kinetic_energy_noalloc)
against the kinetic energy of stau_kinetic_energy, through the C ABI: two
calls in a row on one GPU, the second on a smaller domain, and a 3-D domain;
a domain too large for the fixed scratch array is refused."""
import ctypes as C

import numpy as np
import pytest

import seeded_inputs as si

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("no GPU", allow_module_level=True)

from paper_1905_10388_amd import RBSolver, StauError, _lib  # noqa: E402


def _state(g, seed):
    X = si.complex_noise(g.state_shape, seed) * np.exp(-np.arange(g.info["Nz"]) / 8.0)
    return torch.from_numpy(X).cuda()


def _both(g, X):
    """(stau_kinetic_energy on the host, stau_kinetic_energy_noalloc read back)."""
    ref = C.c_double()
    _lib.check(g.lib.stau_kinetic_energy(g._pen, C.c_void_p(X.data_ptr()), C.byref(ref), None))
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    _lib.check(g.lib.stau_kinetic_energy_noalloc(g._pen, C.c_void_p(X.data_ptr()),
                                                 C.c_void_p(out.data_ptr()), None))
    torch.cuda.synchronize()
    return ref.value, float(out.cpu()[0])


def test_noalloc_kinetic_energy_matches_and_reuses_its_scratch():
    big = RBSolver(1024, 256, 4.0, 1e8, 1.0)
    small = RBSolver(64, 32, 4.0, 1e4, 1.0)
    for g, seed in ((big, 61), (small, 62), (big, 63)):
        ref, got = _both(g, _state(g, seed))
        assert ref != 0.0
        assert abs(got - ref) <= 1e-15 * abs(ref), (g.info["Nx"], got, ref)
    g3 = RBSolver(16, 16, 4.0, 1e5, 1.0, dim=3, Ny=8, Ly=3.0)
    ref, got = _both(g3, _state(g3, 64))
    assert abs(got - ref) <= 1e-15 * abs(ref)


def test_noalloc_kinetic_energy_refuses_domains_beyond_its_scratch():
    g = RBSolver(128, 64, 4.0, 1e6, 1.0, dim=3, Ny=128, Ly=4.0)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(StauError, match="EUNSUPPORTED"):
        _lib.check(g.lib.stau_kinetic_energy_noalloc(g._pen, C.c_void_p(g.X.data_ptr()),
                                                     C.c_void_p(out.data_ptr()), None))
