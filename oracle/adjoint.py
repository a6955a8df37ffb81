"""Oracle: discrete adjoint of the FP64 SBDF stepper (gradient of the kinetic
energy after K steps with respect to the scale-1 grid values of b).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file;
only tests, the smoke check and the CPU-baseline leg of the benchmark do.

The paper defines no adjoint; this is the exact reverse-mode derivative of the
oracle's own discrete forward map (`oracle.rb`), written with the transposes
(Hermitian transposes for complex-linear maps) of the same dense matrices.
Complex coefficients are pairs of independent reals; the adjoint of a complex
number z is  dJ/dRe z + i dJ/dIm z, so a complex-linear map y = A x has the
adjoint x_bar = A^H y_bar, and y = Re(A x) has x_bar = A^H y_bar for real y_bar.

Forward step n (SBDF coefficients of that step):
    F~^{n-1} = P^L N(X^{n-1}),   MX^{n-1} = M X^{n-1}
    B = c1 F~^{n-1} + c2 F~^{n-2} - a1 MX^{n-1} - a2 MX^{n-2}  (BC rows = g)
    X^n = A^{-1} B,  A = a0 M + b0 L
Reverse of step n, given X_bar^n and the pending history adjoints
(Ft_bar, MX_bar) that step n+1 handed back for F~^{n-1}, MX^{n-1}:
    B_bar = A^{-H} X_bar^n            (BC rows of B are constants: dropped)
    Ft_bar^{n-1} = c1 B_bar + pending_F,   MX_bar^{n-1} = -a1 B_bar + pending_M
    pending for step n-1:  c2 B_bar,  -a2 B_bar
    X_bar^{n-1} = M^H MX_bar^{n-1} + N'(X^{n-1})^H (P^L)^H Ft_bar^{n-1}
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import spectral as S
from .rb import RBOracle, sbdf_coefficients


# ----------------------------------------------------------------------------
# adjoints of the grid transforms (transposes of the oracle's dense matrices)
# ----------------------------------------------------------------------------

def to_grid_adjoint(o: RBOracle, gbar: np.ndarray) -> np.ndarray:
    """Adjoint of RBOracle.to_grid: real grid adjoint -> coefficient adjoint."""
    if o.dim == 2:
        Gbar = np.zeros((o.Px, o.Ngz), dtype=np.complex128)
        Gbar[: o.kx_active] = o.Ex.conj().T @ gbar        # g = Re(Ex G)
        return Gbar @ o.Bz                                 # G = c Bz^T, Bz real
    Gy = np.matmul(o.Ex.conj().T, gbar)                    # (Ngy, kx_active, Ngz)
    Gfull = np.zeros((o.Ngy, o.Px, o.Ngz), dtype=np.complex128)
    Gfull[:, : o.kx_active] = Gy
    G = np.tensordot(o.Ey.conj().T, Gfull, axes=(1, 0))    # y backward adjoint
    return G @ o.Bz


def from_grid_adjoint(o: RBOracle, cbar: np.ndarray) -> np.ndarray:
    """Adjoint of RBOracle.from_grid: coefficient adjoint -> real grid adjoint."""
    if o.dim == 2:
        Hbar = cbar[: o.kx_active] @ o.Fz                 # F = H Fz^T, Fz real
        return np.real(o.Fx.conj().T @ Hbar)               # H = Fx g
    Hbar = cbar[:, : o.kx_active] @ o.Fz                   # (Ny, kx_active, Ngz)
    Hy = np.tensordot(o.Fy.conj().T, Hbar, axes=(1, 0))    # (Ngy, kx_active, Ngz)
    return np.real(np.matmul(o.Fx.conj().T, Hy))


def nonlinear_adjoint(o: RBOracle, X: np.ndarray, Fbar: np.ndarray) -> np.ndarray:
    """N'(X)^H Fbar for the explicit term N_q = -(u.grad) q (Sec. IV products
    on the dealiased grid).  Fbar has the layout of RBOracle.nonlinear."""
    vi = o.vi
    kx, ky = o._wavenumber_arrays()
    comps = ("u", "w") if o.dim == 2 else ("u", "v", "w")
    vel = {c: o.to_grid(X[..., vi[c], :]) for c in comps}
    velbar = {c: np.zeros_like(vel[c]) for c in comps}
    Xbar = np.zeros_like(X)
    for e, q in enumerate(o.evolved):
        nbar = from_grid_adjoint(o, Fbar[..., e, :])      # grid adjoint of N_q
        cq = X[..., vi[q], :]
        qx = o.to_grid(1j * kx * cq)
        qz = o.to_grid(X[..., vi[q + "z"], :])
        velbar["u"] -= nbar * qx
        velbar["w"] -= nbar * qz
        Xbar[..., vi[q], :] += np.conj(1j * kx) * to_grid_adjoint(o, -nbar * vel["u"])
        Xbar[..., vi[q + "z"], :] += to_grid_adjoint(o, -nbar * vel["w"])
        if o.dim == 3:
            qy = o.to_grid(1j * ky * cq)
            velbar["v"] -= nbar * qy
            Xbar[..., vi[q], :] += np.conj(1j * ky) * to_grid_adjoint(o, -nbar * vel["v"])
    for c in comps:
        Xbar[..., vi[c], :] += to_grid_adjoint(o, velbar[c])
    return Xbar


def kinetic_energy_adjoint(o: RBOracle, X: np.ndarray) -> np.ndarray:
    """dJ/dX (complex adjoint) of RBOracle.kinetic_energy."""
    comps = ("u", "w") if o.dim == 2 else ("u", "v", "w")
    w = S.cheb_integ_row(o.Nz) * 0.5
    cbar = np.zeros(o.state_shape[:-2] + (o.Nz,), dtype=np.complex128)
    if o.dim == 2:
        cbar[0] = w
    else:
        cbar[0, 0] = w
    ebar = from_grid_adjoint(o, cbar)                      # J = Re(w . mean)
    Xbar = np.zeros(o.state_shape, dtype=np.complex128)
    for c in comps:
        ug = o.to_grid(X[..., o.vi[c], :])
        Xbar[..., o.vi[c], :] = to_grid_adjoint(o, ebar * ug)   # d(u^2/2) = u du
    return Xbar


def initial_state_adjoint(o: RBOracle, Xbar: np.ndarray) -> np.ndarray:
    """Adjoint of RBOracle.state_from_b_grid: state adjoint -> real grid adjoint
    of b on the scale-1 grid (b coefficients and bz = d_z b depend on it)."""
    DTT = 2.0 * S.cheb_diff_TT(o.Nz)
    cbar = Xbar[..., o.vi["b"], :] + Xbar[..., o.vi["bz"], :] @ DTT   # bz = b DTT^T
    Fz1 = S.cheb_forward_matrix(o.Nz, o.Nz)
    Fx1 = S.fourier_real_forward_matrix(o.Nx, o.Nx)
    if o.dim == 2:
        H = cbar[: o.kx_active] @ Fz1                      # c = (Fx1 g) Fz1^T
        return np.real(Fx1.conj().T @ H)
    Fy1 = S.fourier_complex_forward_matrix(o.Ny, o.Ny)
    H = cbar[:, : o.kx_active] @ Fz1                       # (Ny, kx, Nz)
    H = np.tensordot(Fy1.conj().T, H, axes=(1, 0))         # (Ny grid, kx, Nz)
    return np.real(np.matmul(Fx1.conj().T, H)).transpose(1, 0, 2)


# ----------------------------------------------------------------------------
# step adjoint and the checkpointed gradient
# ----------------------------------------------------------------------------

class StepRecord:
    """What the reverse of one step needs: X^{n-1}, the step's coefficients."""

    def __init__(self, X_prev, coeffs):
        self.X_prev = X_prev
        self.coeffs = coeffs


def step_adjoint(o: RBOracle, rec: StepRecord, Xbar: np.ndarray, pend_F: dict, pend_M: dict):
    """Reverse one step.  Returns (Xbar^{n-1}, new pending dicts)."""
    a0, a1, a2, b0, c1, c2 = rec.coeffs
    N = o.Nz
    Fbar = np.zeros(o.state_shape[:-2] + (o.ne, N), dtype=np.complex128)
    Xbar_prev = np.zeros_like(Xbar)
    new_F, new_M = {}, {}
    for key, kx, ky, is_mean, act in o.pencils():
        if not act:
            continue
        M, L = o._ML_cached(key, kx, ky, is_mean)
        A = (a0 * M + b0 * L).tocsc()
        if A.shape[0] <= 1200:
            Bbar = sla.solve(A.toarray().conj().T, Xbar[key].reshape(-1))
        else:
            Bbar = spla.splu(sp.csc_matrix(A.conj().T)).solve(Xbar[key].reshape(-1))
        for r in o.bc_values(is_mean):          # constant rows
            Bbar[r] = 0.0
        ev = np.zeros_like(Bbar)                # only evolved U-rows carry F~, MX
        for e in range(o.ne):
            ev[e * N:e * N + N - 1] = Bbar[e * N:e * N + N - 1]
        Ftbar = c1 * ev + pend_F.get(key, 0.0)
        MXbar = -a1 * ev + pend_M.get(key, 0.0)
        new_F[key] = c2 * ev
        new_M[key] = -a2 * ev
        # MX = M X  ->  X_bar += M^H MX_bar
        Xbar_prev[key] += (M.conj().T @ MXbar).reshape(o.S, N)
        # F~ = P^L F on evolved U-rows  ->  F_bar = (P^L)^H F~_bar
        for e in range(o.ne):
            ft = np.zeros(N, dtype=np.complex128)
            ft[: N - 1] = Ftbar[e * N:e * N + N - 1]
            Fbar[key][e] = o.C.conj().T @ ft
    Xbar_prev += nonlinear_adjoint(o, rec.X_prev, Fbar)
    return Xbar_prev, new_F, new_M


def forward_with_records(o: RBOracle, X0: np.ndarray, dt: float, steps: int):
    o.reset()
    X = X0
    recs = []
    for _ in range(steps):
        coeffs = sbdf_coefficients(o.iteration, dt, o.dt_prev)
        recs.append(StepRecord(X, coeffs))
        X = o.step(X, dt)
    return X, recs


def gradient(o: RBOracle, bgrid: np.ndarray, dt: float, steps: int):
    """J(b grid) after `steps` steps and dJ/d(b grid), by the discrete adjoint
    (all states kept; the oracle needs no checkpointing)."""
    X0 = o.state_from_b_grid(bgrid)
    XK, recs = forward_with_records(o, X0, dt, steps)
    J = o.kinetic_energy(XK)
    Xbar = kinetic_energy_adjoint(o, XK)
    pF, pM = {}, {}
    for rec in reversed(recs):
        Xbar, pF, pM = step_adjoint(o, rec, Xbar, pF, pM)
    return J, initial_state_adjoint(o, Xbar)


def objective(o: RBOracle, bgrid: np.ndarray, dt: float, steps: int) -> float:
    o.reset()
    X = o.state_from_b_grid(bgrid)
    X = o.run(X, dt, steps)
    return o.kinetic_energy(X)
