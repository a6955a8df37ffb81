"""Oracle: FP64 CPU Rayleigh-Benard IMEX (SBDF1 -> SBDF2) stepper.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file;
only tests, the smoke check and the CPU-baseline leg of the benchmark do.

The oracle follows the paper's algorithm step by step with no blocking,
fusion or fast transforms:

* bases and transforms are the dense matrices of `oracle.spectral` (Sec. IV);
* per-pencil matrices are assembled from the Chebyshev templates of
  Appendix A following the row/column processing of Sec. IX "Matrix
  construction": T-to-U left preconditioning of every equation with a z
  derivative, the last row of each such equation replaced by a boundary
  condition, no Dirichlet recombination (it does not change the solution),
  variable-major (Kronecker block) ordering;
* the multistep IMEX update of Sec. IX "Multistep IMEX integrators" with the
  semi-implicit BDF coefficients (first order on the first step);
* an optional non-constant coefficient Gamma(z) w in the b equation
  (Sec. II, non-constant coefficients: the product matrix of numpy's
  Chebyshev multiplication, truncated to N modes);
* the linear boundary value solve of Sec. IX "Linear boundary value
  solver" (`lbvp`);
* the IMEX Runge-Kutta stages of Sec. IX "Runge-Kutta IMEX integrators"
  (`step_rk`, stage right-hand sides with L~X applied directly);
* each pencil is solved by a direct LU factorisation (dense LAPACK getrf for
  small pencils, SuperLU for large ones) reused while (a0, b0) are unchanged.

Readings of points the paper leaves open (equations, units, BC placement,
gauge, SBDF2 coefficients, initial condition, functional) are listed in the
design document; each is marked `reading:` below.

Layouts: 2-D state X[kx_slot][var][n] with kx_slot = 0..Nx/2 (the last slot is
the Nyquist mode, held at zero).  3-D state X[ky_slot][kx_slot][var][n] with
ky in FFT order (0..Ny/2-1, Nyquist slot, -Ny/2+1..-1).  Variables are
(p, b, u, w, bz, uz, wz) in 2-D and (p, b, u, v, w, bz, uz, vz, wz) in 3-D.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import numpy.polynomial.chebyshev as npc
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import spectral as S

VARS_2D = ("p", "b", "u", "w", "bz", "uz", "wz")
VARS_3D = ("p", "b", "u", "v", "w", "bz", "uz", "vz", "wz")


def sbdf_coefficients(iteration: int, dt: float, dt_prev: float | None):
    """Semi-implicit BDF coefficients (a0, a1, a2, b0, c1, c2) for
    sum_j a_j M X^{n-j} + b0 L X^n = c1 F^{n-1} + c2 F^{n-2}.

    reading: the paper cites the SBDF family without coefficients; this is the
    standard variable-step SBDF2 with w = dt_n / dt_{n-1}, and SBDF1
    (backward/forward Euler) for the first step (Sec. IX: multistep schemes
    start at lower order)."""
    if iteration == 0:
        return 1.0 / dt, -1.0 / dt, 0.0, 1.0, 1.0, 0.0
    w = dt / dt_prev
    a0 = (1.0 + 2.0 * w) / ((1.0 + w) * dt)
    a1 = -(1.0 + w) / dt
    a2 = w * w / ((1.0 + w) * dt)
    return a0, a1, a2, 1.0, 1.0 + w, -w


def ncc_matrix(coeffs, N: int) -> np.ndarray:
    """Multiplication by g = sum_k coeffs_k T_k as an N x N matrix on T
    coefficients, the product truncated to the first N modes (Sec. II
    "non-constant coefficients"): column j holds the T expansion of g T_j,
    formed with numpy's Chebyshev product."""
    G = np.zeros((N, N))
    for j in range(N):
        ej = np.zeros(j + 1)
        ej[j] = 1.0
        prod = npc.chebmul(np.asarray(coeffs, dtype=np.float64), ej)
        m = min(N, prod.size)
        G[:m, j] = prod[:m]
    return G


def rk_tableau(scheme: str):
    """(H, A, c) of an IMEX Runge-Kutta scheme with stages 0..s (Sec. IX
    "Runge-Kutta IMEX integrators"): H implicit (first row and column zero),
    A explicit (strictly lower triangular), c the stage times; the last stage
    is the new state.

    reading: the paper names the family (Ascher, Ruuth & Spiteri 1997) but
    prints no tableau; RK111, RK222 and RK443 are that reference's (1,1,1),
    (2,2,2) and (4,4,3) schemes, orders 1, 2 and 3."""
    if scheme == "RK111":
        c = [0.0, 1.0]
        A = [[0.0, 0.0], [1.0, 0.0]]
        H = [[0.0, 0.0], [0.0, 1.0]]
    elif scheme == "RK222":
        g = (2.0 - math.sqrt(2.0)) / 2.0
        d = 1.0 - 1.0 / (2.0 * g)
        c = [0.0, g, 1.0]
        A = [[0.0, 0.0, 0.0], [g, 0.0, 0.0], [d, 1.0 - d, 0.0]]
        H = [[0.0, 0.0, 0.0], [0.0, g, 0.0], [0.0, 1.0 - g, g]]
    elif scheme == "RK443":
        c = [0.0, 1 / 2, 2 / 3, 1 / 2, 1.0]
        A = [[0.0] * 5,
             [1 / 2, 0.0, 0.0, 0.0, 0.0],
             [11 / 18, 1 / 18, 0.0, 0.0, 0.0],
             [5 / 6, -5 / 6, 1 / 2, 0.0, 0.0],
             [1 / 4, 7 / 4, 3 / 4, -7 / 4, 0.0]]
        H = [[0.0] * 5,
             [0.0, 1 / 2, 0.0, 0.0, 0.0],
             [0.0, 1 / 6, 1 / 2, 0.0, 0.0],
             [0.0, -1 / 2, 1 / 2, 1 / 2, 0.0],
             [0.0, 3 / 2, -3 / 2, 1 / 2, 1 / 2]]
    else:
        raise ValueError(f"unknown scheme {scheme!r}")
    return np.array(H), np.array(A), np.array(c)


@dataclass
class RBParams:
    Ra: float
    Pr: float
    buoyancy: float = 1.0   # coefficient of the -b term in the w equation
    b_bottom: float = 1.0   # b(z=0)
    b_top: float = 0.0      # b(z=1)
    # non-constant coefficient Gamma(z) = sum_k gamma_k T_k(2 z - 1) multiplying
    # w in the b equation (a background stratification: d_t b + Gamma w - ...);
    # empty: none
    gamma: tuple = ()

    @property
    def kappa(self) -> float:
        # reading: free-fall units, kappa = (Ra Pr)^(-1/2)
        return (self.Ra * self.Pr) ** -0.5

    @property
    def nu(self) -> float:
        # reading: free-fall units, nu = (Ra / Pr)^(-1/2)
        return (self.Ra / self.Pr) ** -0.5


class RBOracle:
    """Boussinesq Rayleigh-Benard convection, Fourier (x[, y]) x Chebyshev (z).

    reading (equations):  d_t b - kappa lap b = -u.grad b,
    d_t u - nu lap u + grad p - b e_z = -u.grad u,  div u = 0, written first
    order in z with bz, uz, (vz), wz; every linear term on the left.
    z in [0, 1] maps to the native [-1, 1] by z = (zeta + 1) / 2, so d_z = 2 d_zeta.
    """

    def __init__(self, Nx: int, Nz: int, Lx: float, params: RBParams,
                 dim: int = 2, Ny: int | None = None, Ly: float | None = None,
                 dealias: float = 1.5, solver: str = "auto"):
        if dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        self.dim = dim
        self.Nx, self.Nz, self.Lx = int(Nx), int(Nz), float(Lx)
        self.Ny = int(Ny) if dim == 3 else 1
        self.Ly = float(Ly) if dim == 3 else 1.0
        self.par = params
        self.vars = VARS_2D if dim == 2 else VARS_3D
        self.S = len(self.vars)
        self.evolved = ("b", "u", "w") if dim == 2 else ("b", "u", "v", "w")
        self.ne = len(self.evolved)
        self.vi = {v: i for i, v in enumerate(self.vars)}
        self.dealias = dealias
        self.Ngx = int(round(dealias * self.Nx))
        self.Ngy = int(round(dealias * self.Ny)) if dim == 3 else 1
        self.Ngz = int(round(dealias * self.Nz))
        self.Px = self.Nx // 2 + 1
        self.solver = solver
        N = self.Nz
        # z transforms (dealias grid and scale-1 grid)
        self.Bz = S.cheb_backward_matrix(N, self.Ngz)
        self.Fz = S.cheb_forward_matrix(N, self.Ngz)
        # x transforms (real data: half spectrum, k < Nx/2)
        self.Ex = S.fourier_real_backward_matrix(self.Nx, self.Ngx)
        self.Fx = S.fourier_real_forward_matrix(self.Nx, self.Ngx)
        self.kx_active = S.fourier_kmax(self.Nx) + 1          # = Nx/2
        if dim == 3:
            self.Ey = S.fourier_complex_backward_matrix(self.Ny, self.Ngy)
            self.Fy = S.fourier_complex_forward_matrix(self.Ny, self.Ngy)
            self.ky_int = S.fourier_signed_wavenumbers(self.Ny)
            self.ky_act = S.fourier_complex_active(self.Ny)
        # Chebyshev templates on [0, 1]
        self.C = sp.csr_matrix(S.cheb_conversion_TU(N))
        self.D = sp.csr_matrix(2.0 * S.cheb_diff_TU(N))
        self.I = sp.identity(N, format="csr")
        self.left = S.cheb_interp_row(N, "left")    # z = 0
        self.right = S.cheb_interp_row(N, "right")  # z = 1
        self._factor_cache: dict = {}
        self.reset()

    # ------------------------------------------------------------------
    # pencils
    # ------------------------------------------------------------------
    @property
    def state_shape(self):
        if self.dim == 2:
            return (self.Px, self.S, self.Nz)
        return (self.Ny, self.Px, self.S, self.Nz)

    def pencils(self):
        """Yield (index tuple, kx, ky, is_mean, active) for every pencil slot."""
        if self.dim == 2:
            for ix in range(self.Px):
                kx = 2.0 * math.pi * ix / self.Lx
                yield (ix,), kx, 0.0, ix == 0, ix < self.kx_active
        else:
            for iy in range(self.Ny):
                ky = 2.0 * math.pi * float(self.ky_int[iy]) / self.Ly
                for ix in range(self.Px):
                    kx = 2.0 * math.pi * ix / self.Lx
                    yield ((iy, ix), kx, ky, ix == 0 and iy == 0,
                           ix < self.kx_active and bool(self.ky_act[iy]))

    def pencil_matrices(self, kx: float, ky: float, is_mean: bool):
        """Return (M, L) as sparse complex matrices of size S*N, rows grouped by
        equation block and columns by variable block (Kronecker order).

        Row blocks: for each evolved q, the q equation (N-1 U-rows, then the
        z=0 boundary condition on q); for each evolved q, the qz equation (N-1
        U-rows, then the z=1 condition on q); then continuity (N T-rows, no
        preconditioning since it holds no z derivative).
        reading: which dropped row carries which BC only permutes rows.
        reading: at the mean pencil the w(z=1) condition is replaced by the
        gauge p(z=1) = 0 (the paper's per-mode `condition` mechanism).
        """
        N, Sv = self.Nz, self.S
        C, D, I = self.C, self.D, self.I
        kap, nu = self.par.kappa, self.par.nu
        k2 = kx * kx + ky * ky
        vi = self.vi
        Mb = [[None] * Sv for _ in range(Sv)]
        Lb = [[None] * Sv for _ in range(Sv)]

        def add(blocks, r, v, mat):
            blocks[r][vi[v]] = mat if blocks[r][vi[v]] is None else blocks[r][vi[v]] + mat

        def bc_row(vec):
            m = sp.lil_matrix((N, N))
            m[N - 1, :] = vec
            return m.tocsr()

        trunc = sp.diags(np.r_[np.ones(N - 1), 0.0])   # keep U-rows 0..N-2
        for e, q in enumerate(self.evolved):
            r = e
            diff = kap if q == "b" else nu
            add(Mb, r, q, trunc @ C)
            add(Lb, r, q, trunc @ (diff * k2 * C))
            add(Lb, r, q + "z", trunc @ (-diff * D))
            if q == "b" and len(self.par.gamma):
                add(Lb, r, "w", trunc @ (C @ sp.csr_matrix(ncc_matrix(self.par.gamma, N))))
            if q == "u":
                add(Lb, r, "p", trunc @ (1j * kx * C))
            elif q == "v":
                add(Lb, r, "p", trunc @ (1j * ky * C))
            elif q == "w":
                add(Lb, r, "p", trunc @ D)
                if self.par.buoyancy != 0.0:
                    add(Lb, r, "b", trunc @ (-self.par.buoyancy * C))
            add(Lb, r, q, bc_row(self.left))                     # q(z=0)
            rz = self.ne + e
            add(Lb, rz, q + "z", trunc @ C)
            add(Lb, rz, q, trunc @ (-D))
            if q == "w" and is_mean:
                add(Lb, rz, "p", bc_row(self.right))             # gauge p(z=1)
            else:
                add(Lb, rz, q, bc_row(self.right))               # q(z=1)
        rc = 2 * self.ne
        add(Lb, rc, "u", 1j * kx * I)
        if self.dim == 3:
            add(Lb, rc, "v", 1j * ky * I)
        add(Lb, rc, "wz", I)
        Z = sp.csr_matrix((N, N))
        for blocks in (Mb, Lb):
            for r in range(Sv):
                for c in range(Sv):
                    if blocks[r][c] is None:
                        blocks[r][c] = Z
        M = sp.bmat(Mb, format="csr").astype(np.complex128)
        L = sp.bmat(Lb, format="csr").astype(np.complex128)
        return M, L

    def bc_values(self, is_mean: bool):
        """Values of the boundary rows, keyed by row index in the system."""
        N = self.Nz
        g = {}
        if is_mean:
            g[0 * N + N - 1] = self.par.b_bottom                 # b(z=0)
            g[(self.ne + 0) * N + N - 1] = self.par.b_top        # b(z=1)
        return g

    def precondition_rhs(self, Fp: np.ndarray, is_mean: bool) -> np.ndarray:
        """F~ = P^L F on the evolved-equation U-rows; BC rows carry their values;
        the qz and continuity rows are zero.  Fp has shape (ne, N)."""
        N = self.Nz
        out = np.zeros(self.S * N, dtype=np.complex128)
        for e in range(self.ne):
            out[e * N:e * N + N - 1] = (self.C @ Fp[e])[:N - 1]
        for r, val in self.bc_values(is_mean).items():
            out[r] = val
        return out

    def apply_M(self, M, Xp: np.ndarray) -> np.ndarray:
        return M @ Xp.reshape(-1)

    # ------------------------------------------------------------------
    # grid-space nonlinear term (Sec. IV "Scaled transforms & dealiasing")
    # ------------------------------------------------------------------
    def _wavenumber_arrays(self):
        kx = 2.0 * math.pi * np.arange(self.Px) / self.Lx
        if self.dim == 2:
            return kx[:, None], None
        ky = 2.0 * math.pi * self.ky_int.astype(np.float64) / self.Ly
        return kx[None, :, None], ky[:, None, None]

    def to_grid(self, c: np.ndarray) -> np.ndarray:
        """Coefficients (state layout without the var axis) -> real values on
        the dealiased grid.  2-D: (Px, N) -> (Ngx, Ngz); 3-D: (Ny, Px, N) ->
        (Ngy, Ngx, Ngz).  Direct sums: z, then y (complex), then x (real)."""
        G = c @ self.Bz.T                                   # z backward
        if self.dim == 2:
            return np.real(self.Ex @ G[: self.kx_active])    # x backward
        G = np.tensordot(self.Ey, G, axes=(1, 0))           # y backward
        G = G[:, : self.kx_active, :]
        return np.real(np.matmul(self.Ex, G))               # x backward, per y level

    def from_grid(self, g: np.ndarray) -> np.ndarray:
        """Real values on the dealiased grid -> truncated coefficients."""
        if self.dim == 2:
            H = self.Fx @ g                                  # x forward (Nx/2, Ngz)
            out = np.zeros((self.Px, self.Nz), dtype=np.complex128)
            out[: self.kx_active] = H @ self.Fz.T            # z forward
            return out
        H = np.matmul(self.Fx, g)                            # x forward, per y level
        H = np.tensordot(self.Fy, H, axes=(1, 0))            # y forward
        out = np.zeros((self.Ny, self.Px, self.Nz), dtype=np.complex128)
        out[:, : self.kx_active] = H @ self.Fz.T             # z forward
        return out

    def nonlinear(self, X: np.ndarray) -> np.ndarray:
        """Coefficients of N_q = -(u . grad) q for q in the evolved fields.

        Returns an array of the state layout with an evolved-field axis of size
        ne in place of the variable axis."""
        vi = self.vi
        kx, ky = self._wavenumber_arrays()
        comps = ("u", "w") if self.dim == 2 else ("u", "v", "w")
        vel = {c: self.to_grid(X[..., vi[c], :]) for c in comps}
        out = np.zeros(X.shape[:-2] + (self.ne, self.Nz), dtype=np.complex128)
        for e, q in enumerate(self.evolved):
            cq = X[..., vi[q], :]
            acc = -vel["u"] * self.to_grid(1j * kx * cq)
            if self.dim == 3:
                acc -= vel["v"] * self.to_grid(1j * ky * cq)
            acc -= vel["w"] * self.to_grid(X[..., vi[q + "z"], :])
            out[..., e, :] = self.from_grid(acc)
        return out

    # ------------------------------------------------------------------
    # time stepping (Sec. IX "Multistep IMEX integrators")
    # ------------------------------------------------------------------
    def reset(self):
        self.iteration = 0
        self.dt_prev = None
        self.Ft_hist: list = []     # [F~^{n-1}, F~^{n-2}] per pencil (dicts)
        self.MX_hist: list = []
        self.last_coeffs = None

    def _factor(self, key, A):
        n = A.shape[0]
        use_dense = self.solver == "dense" or (self.solver == "auto" and n <= 1200)
        if use_dense:
            lu = sla.lu_factor(A.toarray(), check_finite=False)
            return lambda b: sla.lu_solve(lu, b, check_finite=False)
        slu = spla.splu(sp.csc_matrix(A), permc_spec="COLAMD")
        return slu.solve

    def solver_for(self, key, kx, ky, is_mean, a0, b0):
        ck = (key, a0, b0)
        f = self._factor_cache.get(ck)
        if f is None:
            M, L = self.pencil_matrices(kx, ky, is_mean)
            f = self._factor(ck, (a0 * M + b0 * L).tocsc())
            # keep only the factorisations for the current (a0, b0)
            for old in [k for k in self._factor_cache if k[1:] != (a0, b0)]:
                del self._factor_cache[old]
            self._factor_cache[ck] = f
        return f

    def step(self, X: np.ndarray, dt: float) -> np.ndarray:
        """One IMEX step X^{n-1} -> X^n (returns a new array)."""
        a0, a1, a2, b0, c1, c2 = sbdf_coefficients(self.iteration, dt, self.dt_prev)
        self.last_coeffs = (a0, a1, a2, b0, c1, c2)
        Fnl = self.nonlinear(X)
        Xn = np.zeros_like(X)
        Ft_now, MX_now = {}, {}
        for key, kx, ky, is_mean, active in self.pencils():
            if not active:
                continue
            M, L = self._ML_cached(key, kx, ky, is_mean)
            Ft = self.precondition_rhs(Fnl[key], is_mean)
            MX = M @ X[key].reshape(-1)
            B = c1 * Ft - a1 * MX
            if self.iteration > 0:
                B += c2 * self.Ft_hist[0][key] - a2 * self.MX_hist[0][key]
            # reading: BC rows carry g directly (M has zero BC rows, c1 + c2 = 1)
            for r, val in self.bc_values(is_mean).items():
                B[r] = val
            Ft_now[key], MX_now[key] = Ft, MX
            solve = self.solver_for(key, kx, ky, is_mean, a0, b0)
            Xn[key] = solve(B).reshape(self.S, self.Nz)
        self.Ft_hist = [Ft_now] + self.Ft_hist[:1]
        self.MX_hist = [MX_now] + self.MX_hist[:1]
        self.dt_prev = dt
        self.iteration += 1
        return Xn

    _ML_store: dict

    def _ML_cached(self, key, kx, ky, is_mean):
        if not hasattr(self, "_ML_store"):
            self._ML_store = {}
        v = self._ML_store.get(key)
        if v is None:
            v = self.pencil_matrices(kx, ky, is_mean)
            if len(self._ML_store) < 4096:
                self._ML_store[key] = v
        return v

    def run(self, X: np.ndarray, dt: float, steps: int) -> np.ndarray:
        for _ in range(steps):
            X = self.step(X, dt)
        return X

    # ------------------------------------------------------------------
    # linear boundary value problem (Sec. IX "Linear boundary value solver")
    # ------------------------------------------------------------------
    def lbvp(self, F: np.ndarray) -> np.ndarray:
        """Solve L X = F per pencil: the left-preconditioned system
        P^L L P^R (P^R)^{-1} X = P^L F (here without P^R, which does not change
        X), with F given as T coefficients of the right side of each evolved
        equation (evolved-field axis of size ne in place of the variable
        axis), the boundary rows carrying their Dirichlet values and the
        first-order and continuity rows zero.  Returns X in the state layout."""
        X = np.zeros(self.state_shape, dtype=np.complex128)
        for key, kx, ky, is_mean, active in self.pencils():
            if not active:
                continue
            M, L = self._ML_cached(key, kx, ky, is_mean)
            solve = self.solver_for(key, kx, ky, is_mean, 0.0, 1.0)
            X[key] = solve(self.precondition_rhs(F[key], is_mean)).reshape(self.S, self.Nz)
        return X

    # ------------------------------------------------------------------
    # time stepping (Sec. IX "Runge-Kutta IMEX integrators")
    # ------------------------------------------------------------------
    def step_rk(self, X: np.ndarray, dt: float, scheme: str = "RK222") -> np.ndarray:
        """One IMEX Runge-Kutta step X^n -> X^{n+1} (returns a new array).

        Stages i = 1..s solve, per pencil,
          (M~ + dt H_ii L~) X^{n,i} = M~ X^{n,0} + dt sum_{j<i} A_ij F~^{n,j}
                                     - dt sum_{j<i} H_ij L~ X^{n,j},
        with F~^{n,j} = P^L F(X^{n,j}) (boundary rows carrying their values)
        and L~ X^{n,j} applied directly; the last stage is X^{n+1} (globally
        stiffly accurate).  The multistep history is not touched."""
        H, A, c = rk_tableau(scheme)
        s = len(c) - 1
        Xs = [X]
        MX0: dict = {}
        Ft: list = []   # Ft[j][key] = F~^{n,j}
        LX: list = []   # LX[j][key] = L~ X^{n,j}
        for i in range(1, s + 1):
            Fnl = self.nonlinear(Xs[i - 1])
            Ft_j, LX_j = {}, {}
            for key, kx, ky, is_mean, active in self.pencils():
                if not active:
                    continue
                M, L = self._ML_cached(key, kx, ky, is_mean)
                xv = Xs[i - 1][key].reshape(-1)
                if i == 1:
                    MX0[key] = M @ xv
                Ft_j[key] = self.precondition_rhs(Fnl[key], is_mean)
                LX_j[key] = L @ xv
            Ft.append(Ft_j)
            LX.append(LX_j)
            Xn = np.zeros_like(X)
            for key, kx, ky, is_mean, active in self.pencils():
                if not active:
                    continue
                B = MX0[key].copy()
                for j in range(i):
                    B += dt * A[i][j] * Ft[j][key] - dt * H[i][j] * LX[j][key]
                solve = self.solver_for(key, kx, ky, is_mean, 1.0, dt * H[i][i])
                Xn[key] = solve(B).reshape(self.S, self.Nz)
            Xs.append(Xn)
        return Xs[s]

    # ------------------------------------------------------------------
    # initial condition and functionals
    # ------------------------------------------------------------------
    def scale1_grids(self):
        """Scale-1 grids: x_i = Lx i / Nx, (y_l = Ly l / Ny), z_j on [0, 1]."""
        x = self.Lx * np.arange(self.Nx) / self.Nx
        z = 0.5 * (S.cheb_grid(self.Nz) + 1.0)
        if self.dim == 2:
            return x, z
        y = self.Ly * np.arange(self.Ny) / self.Ny
        return x, y, z

    def grid_to_coeff_scale1(self, g: np.ndarray) -> np.ndarray:
        """Real scale-1 grid values -> coefficients in the state layout (one
        field).  2-D g[i_x, j_z]; 3-D g[i_x, l_y, j_z]."""
        Fz1 = S.cheb_forward_matrix(self.Nz, self.Nz)
        Fx1 = S.fourier_real_forward_matrix(self.Nx, self.Nx)
        if self.dim == 2:
            out = np.zeros((self.Px, self.Nz), dtype=np.complex128)
            out[: self.kx_active] = (Fx1 @ g) @ Fz1.T
            return out
        Fy1 = S.fourier_complex_forward_matrix(self.Ny, self.Ny)
        H = np.matmul(Fx1, g.transpose(1, 0, 2))             # (Ny, Nx/2, Nz)
        H = np.tensordot(Fy1, H, axes=(1, 0))
        out = np.zeros((self.Ny, self.Px, self.Nz), dtype=np.complex128)
        out[:, : self.kx_active] = H @ Fz1.T
        return out

    def coeff_to_grid_scale1(self, c: np.ndarray) -> np.ndarray:
        Bz1 = S.cheb_backward_matrix(self.Nz, self.Nz)
        Ex1 = S.fourier_real_backward_matrix(self.Nx, self.Nx)
        G = c @ Bz1.T
        if self.dim == 2:
            return np.real(Ex1 @ G[: self.kx_active])
        Ey1 = S.fourier_complex_backward_matrix(self.Ny, self.Ny)
        G = np.tensordot(Ey1, G, axes=(1, 0))[:, : self.kx_active, :]
        return np.real(np.matmul(Ex1, G)).transpose(1, 0, 2)

    def initial_b_grid(self, xi: np.ndarray, amp: float = 1e-3) -> np.ndarray:
        """reading: b = 1 - z + amp z (1 - z) xi on the scale-1 grid."""
        grids = self.scale1_grids()
        z = grids[-1]
        prof = z * (1.0 - z)
        if self.dim == 2:
            return (1.0 - z)[None, :] + amp * prof[None, :] * xi
        return (1.0 - z)[None, None, :] + amp * prof[None, None, :] * xi

    def state_from_b_grid(self, bgrid: np.ndarray) -> np.ndarray:
        """Consistent initial state: b from the grid, bz = d_z b through the
        T-to-T derivative, every other variable zero."""
        X = np.zeros(self.state_shape, dtype=np.complex128)
        bc = self.grid_to_coeff_scale1(bgrid)
        X[..., self.vi["b"], :] = bc
        DTT = 2.0 * S.cheb_diff_TT(self.Nz)
        X[..., self.vi["bz"], :] = bc @ DTT.T
        return X

    def initial_state(self, xi: np.ndarray, amp: float = 1e-3) -> np.ndarray:
        return self.state_from_b_grid(self.initial_b_grid(xi, amp))

    def kinetic_energy(self, X: np.ndarray) -> float:
        """J = (1 / volume) * integral of (|u|^2) / 2, evaluated the method's way:
        product on the dealiased grid, truncated forward transform, then the
        integration functionals (the mean Fourier coefficient, and the
        Chebyshev integration vector rescaled by the affine map dz = dzeta/2).
        reading: the functional of the adjoint workload."""
        comps = ("u", "w") if self.dim == 2 else ("u", "v", "w")
        e = sum(self.to_grid(X[..., self.vi[c], :]) ** 2 for c in comps) * 0.5
        ce = self.from_grid(e)
        mean = ce[0] if self.dim == 2 else ce[0, 0]
        w = S.cheb_integ_row(self.Nz) * 0.5            # integral over z in [0,1]
        return float(np.real(w @ mean))                # Lz = 1

    # ------------------------------------------------------------------
    # linear eigenproblem sigma M X + L X = 0 (Sec. IX "Eigenvalue solver")
    # ------------------------------------------------------------------
    def linearized_matrices(self, kx: float, ky: float = 0.0, is_mean: bool = False):
        """(M, L + L') for the problem linearised about the conduction state
        b0 = b_bottom + (b_top - b_bottom) z.  L' is the linearisation of the
        explicit term -(u.grad) b about b0, i.e. -w d_z b0 in the b equation,
        moved to the left-hand side as (b_top - b_bottom) P^L w on its U-rows."""
        M, L = self.pencil_matrices(kx, ky, is_mean)
        N = self.Nz
        Lp = sp.lil_matrix(L.shape, dtype=np.complex128)
        w0 = self.vi["w"] * N
        Lp[0:N - 1, w0:w0 + N] = (self.par.b_top - self.par.b_bottom) * self.C.toarray()[:N - 1]
        return M, (L + Lp.tocsr())

    def linear_growth_rate(self, kx: float, ky: float = 0.0) -> float:
        """Largest real part of the finite eigenvalues sigma of
        sigma M X + (L + L') X = 0 (linearised about conduction) at (kx, ky),
        solved densely (Sec. IX "Eigenvalue solver")."""
        M, A = self.linearized_matrices(kx, ky)
        w = sla.eigvals(A.toarray(), -M.toarray())
        w = w[np.isfinite(w)]
        w = w[np.abs(w) < 1e8]
        return float(np.max(w.real))


    def stability_eigenvalue(self, kx: float, ky: float = 0.0, tau: float = 0.0,
                             is_mean: bool = False, method: str = "auto") -> float:
        """The eigenvalue sigma of sigma M X + (L + L') X = 0 (linearised about
        conduction, Sec. IX "Eigenvalue solver") nearest the real shift tau:
        the dense generalized eigenvalues for small pencils, else ARPACK on the
        shift-inverted operator (L + L' + tau M)^{-1} M, whose dominant
        eigenvalue is 1 / (tau - sigma) (the paper's sparse shift-invert
        route).  The spectrum of this problem is real; the real part is
        returned.  is_mean selects the mean pencil's rows (gauge p(1) = 0);
        method "dense" or "arpack" forces a route."""
        M, A = self.linearized_matrices(kx, ky, is_mean)
        n = M.shape[0]
        if method == "dense" or (method == "auto" and n <= 1200):
            w = sla.eigvals(A.toarray(), -M.toarray())
            w = w[np.isfinite(w)]
            w = w[np.abs(w) < 1e8]
            return float(np.real(w[np.argmin(np.abs(w - tau))]))
        lu = spla.splu((A + tau * M).tocsc())
        T = spla.LinearOperator(A.shape, matvec=lambda x: lu.solve(M @ x), dtype=np.complex128)
        mu = spla.eigs(T, k=1, which="LM", return_eigenvectors=False, tol=1e-14)[0]
        return float(np.real(tau - 1.0 / mu))


    def stability_eigenvalues(self, kx: float, ky: float = 0.0, tau: float = 0.0, nev: int = 1,
                              is_mean: bool = False, method: str = "auto") -> np.ndarray:
        """The nev eigenvalues sigma of sigma M X + (L + L') X = 0 (linearised
        about conduction, Sec. IX "Eigenvalue solver") nearest the real shift
        tau, nearest first, as complex numbers: all finite generalized
        eigenvalues (dense, small pencils) or ARPACK's nev dominant
        eigenvalues mu of the shift-inverted operator (L + L' + tau M)^{-1} M,
        sigma = tau - 1 / mu (the paper's sparse route); method "dense" or
        "arpack" forces a route."""
        M, A = self.linearized_matrices(kx, ky, is_mean)
        n = M.shape[0]
        if method == "dense" or (method == "auto" and n <= 1200):
            w = sla.eigvals(A.toarray(), -M.toarray())
            w = w[np.isfinite(w)]
            w = w[np.abs(w) < 1e8]
        else:
            lu = spla.splu((A + tau * M).tocsc())
            T = spla.LinearOperator(A.shape, matvec=lambda x: lu.solve(M @ x), dtype=np.complex128)
            mu = spla.eigs(T, k=nev, ncv=max(2 * nev + 1, 20), which="LM", return_eigenvectors=False,
                           tol=1e-14)
            w = tau - 1.0 / mu
        return w[np.argsort(np.abs(w - tau), kind="stable")][:nev]

def tau_poisson_bvp(N: int, f_coeffs: np.ndarray) -> np.ndarray:
    """Worked example of Sec. II "Summary & example": u'' = f on [-1, 1],
    u(-1) = 0, u'(1) = 0, as the first-order system d_x ux = f,
    d_x u - ux = 0 (T-to-U, last rows replaced by the two conditions).
    Returns the T coefficients of u."""
    C = S.cheb_conversion_TU(N)
    D = S.cheb_diff_TU(N)
    A = np.zeros((2 * N, 2 * N))
    rhs = np.zeros(2 * N)
    # block 0: d_x ux = f  (variables: u -> cols 0..N-1, ux -> cols N..2N-1)
    A[0:N - 1, N:2 * N] = D[:N - 1]
    rhs[0:N - 1] = (C @ f_coeffs)[:N - 1]
    A[N - 1, 0:N] = S.cheb_interp_row(N, "left")          # u(-1) = 0
    # block 1: d_x u - ux = 0
    A[N:2 * N - 1, 0:N] = D[:N - 1]
    A[N:2 * N - 1, N:2 * N] = -C[:N - 1]
    A[2 * N - 1, N:2 * N] = S.cheb_interp_row(N, "right")  # ux(1) = 0
    sol = np.linalg.solve(A, rhs)
    return sol[:N]
