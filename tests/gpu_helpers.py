"""Helpers shared by the GPU parity tests (oracle side and comparisons)."""
import numpy as np

from oracle import RBOracle, RBParams


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def field_errors(o: RBOracle, Xg, Xo):
    """Relative L2 error per variable over all coefficients."""
    return {v: rel_err(Xg[..., i, :], Xo[..., i, :]) for i, v in enumerate(o.vars)}


def oracle_solve_from_ev(o: RBOracle, Bev, a0, b0, pencils=None):
    """Solve (a0 M + b0 L) X = B per pencil, where B carries Bev on the evolved
    U-rows, the Dirichlet values on the boundary rows and zero elsewhere."""
    N = o.Nz
    X = np.zeros(o.state_shape, dtype=np.complex128)
    for key, kx, ky, is_mean, act in o.pencils():
        if not act:
            continue
        if pencils is not None and key not in pencils:
            continue
        M, L = o.pencil_matrices(kx, ky, is_mean)
        B = np.zeros(o.S * N, dtype=np.complex128)
        for e in range(o.ne):
            B[e * N:e * N + N - 1] = Bev[key][e, :N - 1]
        for r, val in o.bc_values(is_mean).items():
            B[r] = val
        f = o._factor(None, (a0 * M + b0 * L).tocsc())
        X[key] = f(B).reshape(o.S, N)
    return X
