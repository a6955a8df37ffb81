"""The runtime's per-pencil operator, checked on the host (no GPU).

* `tests/host/templates_check.cpp` (compiled with the runtime's own headers):
  the structured row application of the stability iteration against the
  entry-by-entry matrix, the band templates the factorisation combines per
  pencil against the same entries, and the band widths against a full scan.
* The operator itself against the oracle's dense pencil matrices (Sec. IX
  "Matrix construction"): the runtime's a0 M~ + b0 L~ is the oracle's
  a0 M + b0 L (Kronecker order, no recombination, complex) after three
  changes of form that do not change the solution, restated here from their
  definitions:
    - interleaved order: column (mode m, variable), rows the kb boundary
      conditions first, then (mode n, equation) with only continuity at the
      last mode;
    - Dirichlet recombination (Sec. II "Banded boundary conditions"): the
      T-coefficients of a variable are x_T[k] = x~[k] - x~[k + 2];
    - real scaling: the horizontal velocities and their z derivatives are
      stored times i (u = -i u~), and their equations and boundary rows are
      multiplied by i, so that every entry is real.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import RBOracle, RBParams

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)

pytestmark = pytest.mark.skipif(HIPCC is None, reason="hipcc not available")

# interleaved variable and equation order of one mode (the runtime's layout)
COLS = {2: ("w", "b", "u", "p", "bz", "uz", "wz"), 3: ("w", "b", "u", "v", "p", "bz", "uz", "vz", "wz")}
ROWS = {2: ("w", "b", "u", "c", "uz", "bz", "wz"), 3: ("w", "b", "u", "v", "c", "uz", "vz", "bz", "wz")}
SCALED = ("u", "v", "uz", "vz")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = tmp_path_factory.mktemp("tc") / "templates_check"
    src = os.path.join(ROOT, "tests", "host", "templates_check.cpp")
    inc = os.path.join(ROOT, "paper_1905_10388_amd", "csrc")
    r = subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", inc,
                        src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return str(exe)


def test_structured_rows_templates_and_band_widths(checker):
    out = subprocess.run([checker], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr


def test_host_code_under_sanitizers(tmp_path):
    """The host build of the system description, band widths and templates
    with AddressSanitizer and UndefinedBehaviorSanitizer (host code only:
    -fno-gpu-sanitize); any report aborts the program."""
    exe = tmp_path / "templates_check_san"
    src = os.path.join(ROOT, "tests", "host", "templates_check.cpp")
    inc = os.path.join(ROOT, "paper_1905_10388_amd", "csrc")
    r = subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-fsanitize=address", "-fsanitize=undefined", "-fno-gpu-sanitize",
                        "-fno-sanitize-recover=all", "-I", inc, src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    assert out.returncode == 0, out.stdout + out.stderr[-4000:]
    out = subprocess.run([str(exe), "dump", "3", "9", "1", "2.0", "1.0", "0.1", "0.2", "1.0", "0", "0", "-1",
                          "2", "0.5", "0.25", "0", "0"], capture_output=True, text=True, env=env)
    assert out.returncode == 0, out.stderr[-4000:]


def _runtime_matrix(checker, dim, N, mean, a0, b0, par, kx, ky, lin):
    g = list(par.gamma) + [0.0] * (4 - len(par.gamma))
    args = [checker, "dump", dim, N, int(mean), a0, b0, par.kappa, par.nu, par.buoyancy, kx, ky, lin,
            len(par.gamma), *g]
    out = subprocess.run([str(a) if isinstance(a, (int, str)) else repr(float(a)) for a in args],
                         capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    lines = out.stdout.strip().split("\n")
    n, kl, ku = (int(v) for v in lines[0].split())
    A = np.array([[float(v) for v in ln.split()] for ln in lines[1:]])
    assert A.shape == (n, n)
    return A, kl, ku


def _maps(o, dim, N):
    """(R, Q): runtime operator = R (a0 M + b0 L) Q for the oracle's (M, L)."""
    S = len(COLS[dim])
    n = S * N
    vi = o.vi
    ev = list(o.evolved)
    ne = len(ev)
    Q = np.zeros((n, n), dtype=complex)
    for m in range(N):
        for pos, var in enumerate(COLS[dim]):
            s = -1j if var in SCALED else 1.0
            c = m * S + pos
            Q[vi[var] * N + m, c] += s          # T_m
            if m >= 2:
                Q[vi[var] * N + m - 2, c] -= s  # - T_{m-2}
    R = np.zeros((n, n), dtype=complex)
    r = 0
    for side in (0, 1):                  # boundary rows: z = 0, then z = 1
        for e, q in enumerate(ev):
            blk = e if side == 0 else ne + e
            R[r, blk * N + N - 1] = 1j if q in SCALED else 1.0
            r += 1
    for nm in range(N):
        for eq in ROWS[dim]:
            if nm == N - 1 and eq != "c":
                continue
            if eq == "c":
                blk = 2 * ne
            elif eq.endswith("z"):
                blk = ne + ev.index(eq[0])
            else:
                blk = ev.index(eq)
            R[r, blk * N + nm] = 1j if eq in SCALED else 1.0
            r += 1
    assert r == n
    return R, Q


CASES = [
    # dim, N, mean, kx, ky, lin, Ra, Pr, gamma
    (2, 8, False, 3.3, 0.0, False, 1e5, 1.0, ()),
    (2, 12, True, 0.0, 0.0, False, 1e4, 0.5, ()),
    (2, 10, False, 1.7, 0.0, True, 2e3, 7.0, ()),
    (2, 9, False, 2.5, 0.0, False, 1e6, 1.0, (0.3, -0.2, 0.1)),
    (2, 8, True, 0.0, 0.0, True, 1e6, 1.0, (0.5, 0.25)),
    (3, 8, False, 3.1, -2.2, False, 1e5, 1.0, ()),
    (3, 7, True, 0.0, 0.0, False, 1e5, 2.0, ()),
    (3, 8, False, 0.0, 1.4, True, 1e4, 1.0, ()),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}d-N{c[1]}{'-mean' if c[2] else ''}"
                                             f"{'-lin' if c[5] else ''}{'-ncc' if c[8] else ''}"
                                             for c in CASES])
def test_operator_matches_oracle_pencil_matrices(checker, case):
    dim, N, mean, kx, ky, lin, Ra, Pr, gamma = case
    par = RBParams(Ra, Pr, gamma=gamma)
    kw = dict(dim=3, Ny=8, Ly=2.0) if dim == 3 else {}
    o = RBOracle(8, N, 2.0, par, **kw)
    rng = np.random.default_rng(N + 10 * dim)
    a0, b0 = rng.uniform(0.5, 300.0), rng.uniform(0.2, 2.0)
    if lin:
        M, L = o.linearized_matrices(kx, ky, mean)
    else:
        M, L = o.pencil_matrices(kx, ky, mean)
    Ao = (a0 * M + b0 * L).toarray()
    A, kl, ku = _runtime_matrix(checker, dim, N, mean, a0, b0, par, kx, ky,
                                (par.b_top - par.b_bottom) if lin else 0.0)
    R, Q = _maps(o, dim, N)
    B = R @ Ao @ Q
    scale = np.abs(B).max()
    assert np.abs(B.imag).max() <= 1e-14 * scale
    assert np.abs(A - B.real).max() <= 1e-13 * scale, np.unravel_index(np.argmax(np.abs(A - B.real)), A.shape)
    # the band the runtime stores holds every nonzero entry
    rr, cc = np.nonzero(A)
    assert (rr - cc).max() <= kl and (cc - rr).max() <= ku
