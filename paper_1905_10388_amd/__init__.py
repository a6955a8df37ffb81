"""MI355X (gfx950) sparse-tau SBDF2 stepper for Fourier x Chebyshev
Rayleigh-Benard convection.

Every step of the path runs in the HIP kernels of libstau.so; this module only
marshals torch device tensors and the current HIP stream into the C ABI of
include/stau.h.  Importing it does not load the library; constructing an
`RBSolver` does, and fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C

from . import _lib

__all__ = ["RBSolver", "StauError"]

StauError = _lib.StauError


def _stream_ptr(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class RBSolver:
    """One domain + pencil system + caller-owned state tensors.

    Attributes after construction: `X` (complex128 state, layout of the C ABI),
    `hist` (complex128 history), `info` (sizes), `iteration`, `dt_prev`.
    """

    def __init__(self, Nx: int, Nz: int, Lx: float, Ra: float, Pr: float, *, dim: int = 2,
                 Ny: int = 1, Ly: float = 1.0, precision: str = "fp64", buoyancy: float = 1.0,
                 b_bottom: float = 1.0, b_top: float = 0.0, device: int = 0, dct: str = "auto",
                 gamma=(), mixed_solve: str = "auto", factor_layout: str = "auto",
                 library: str = "default"):
        import torch

        self._torch = torch
        # "check": the check build (the kernels' index checks, reported by check())
        lib = _lib.load({"default": _lib.LIB_PATH, "check": _lib.LIB_CHECK_PATH}[library])
        self.lib = lib
        desc = _lib.DomainDesc(dim=dim, precision={"fp64": _lib.STAU_FP64, "mixed": _lib.STAU_MIXED}[precision],
                               Nx=Nx, Ny=Ny, Nz=Nz, Lx=Lx, Ly=Ly, dealias=1.5, device=device,
                               dct_method={"auto": _lib.STAU_DCT_AUTO, "fft": _lib.STAU_DCT_FFT,
                                           "matmul": _lib.STAU_DCT_MATMUL}[dct],
                               mixed_solve={"auto": _lib.STAU_SOLVE_AUTO, "fp64": _lib.STAU_SOLVE_FP64,
                                            "refined": _lib.STAU_SOLVE_REFINED}[mixed_solve],
                               factor_layout={"auto": _lib.STAU_FACTORS_AUTO,
                                              "band": _lib.STAU_FACTORS_BAND}[factor_layout])
        gamma = tuple(float(g) for g in gamma)
        if len(gamma) > 4:
            raise ValueError("at most 4 Chebyshev terms of Gamma(z)")
        self._dom = C.c_void_p()
        self._ok(lib.stau_create_domain(C.byref(desc), C.byref(self._dom)))
        par = _lib.RBParamsC(Ra=Ra, Pr=Pr, buoyancy=buoyancy, b_bottom=b_bottom, b_top=b_top,
                             n_gamma=len(gamma), gamma=(C.c_double * 4)(*(gamma + (0.0,) * (4 - len(gamma)))))
        self._pen = C.c_void_p()
        rc = lib.stau_build_pencils(self._dom, C.byref(par), C.byref(self._pen))
        if rc:
            lib.stau_destroy_domain(self._dom)
            self._dom = None  # destroyed: close() must not free it again
            self._pen = None
            self._ok(rc)
        info = _lib.InfoC()
        self._ok(lib.stau_query(self._pen, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _lib.InfoC._fields_}
        self.dim = dim
        self.device = torch.device("cuda", device)
        i = self.info
        if dim == 2:
            self.state_shape = (i["Px"], i["S"], i["Nz"])
            self.ev_shape = (i["Px"], i["ne"], i["Nz"])
        else:
            self.state_shape = (i["Ny"], i["Px"], i["S"], i["Nz"])
            self.ev_shape = (i["Ny"], i["Px"], i["ne"], i["Nz"])
        self.X = torch.zeros(self.state_shape, dtype=torch.complex128, device=self.device)
        self.hist = torch.zeros((2, i["P"], 2, i["ne"], i["Nz"]), dtype=torch.complex128,
                                device=self.device)
        self._st = _lib.StateC(X=self.X.data_ptr(), hist=self.hist.data_ptr(), iteration=0,
                               dt_prev=0.0, head=0)

    # -- lifetime ---------------------------------------------------------
    def _ok(self, rc):
        _lib.check(rc, self.lib)

    def query(self):
        """Sizes of the domain as stau_query reports them now (the workspace
        grows when factor storage is allocated on first use)."""
        info = _lib.InfoC()
        self._ok(self.lib.stau_query(self._pen, C.byref(info)))
        return {f: getattr(info, f) for f, _ in _lib.InfoC._fields_}

    def close(self):
        if getattr(self, "_pen", None):
            self.lib.stau_destroy_pencils(self._pen)
            self._pen = None
        if getattr(self, "_dom", None):
            self.lib.stau_destroy_domain(self._dom)
            self._dom = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state ------------------------------------------------------------
    @property
    def iteration(self) -> int:
        return int(self._st.iteration)

    @property
    def dt_prev(self) -> float:
        return float(self._st.dt_prev)

    def reset(self):
        self._st.iteration = 0
        self._st.dt_prev = 0.0
        self._st.head = 0

    def set_state(self, X):
        """Copy a complex128 state (state layout) into the solver and restart at SBDF1."""
        self.X.copy_(X)
        self.reset()

    def initial_state(self, b_grid):
        """Initial state from scale-1 grid values of b (float64 device tensor)."""
        t = self._torch
        b = b_grid.to(device=self.device, dtype=t.float64).contiguous()
        self._ok(self.lib.stau_initial_state(self._pen, _ptr(b), _ptr(self.X), _stream_ptr()))
        self.reset()
        return self.X

    # -- the hot path -----------------------------------------------------
    def step(self, dt: float):
        self._st.X = self.X.data_ptr()
        self._st.hist = self.hist.data_ptr()
        self._ok(self.lib.stau_step(self._pen, C.byref(self._st), float(dt), _stream_ptr()))

    def step_rk(self, dt: float, scheme: str = "RK222"):
        """One IMEX Runge-Kutta step of the state in place (RK111, RK222 or
        RK443); independent of the multistep history."""
        code = _lib.RK_SCHEMES.get(scheme)
        if code is None:
            raise ValueError(f"unknown Runge-Kutta scheme {scheme!r}")
        self._ok(self.lib.stau_step_rk(self._pen, code, float(dt), _ptr(self.X), _stream_ptr()))

    def lbvp(self, F, out=None):
        """Linear boundary value solve L X = F per pencil (F: complex128 T
        coefficients [.., ne, Nz] of the evolved equations' right sides).
        Returns X in the state layout (a new tensor unless `out` is given)."""
        t = self._torch
        F = F.to(device=self.device, dtype=t.complex128).contiguous()
        if tuple(F.shape) != tuple(self.ev_shape):
            raise ValueError(f"F must have shape {self.ev_shape}")
        X = out if out is not None else t.empty(self.state_shape, dtype=t.complex128, device=self.device)
        self._ok(self.lib.stau_lbvp(self._pen, _ptr(F), _ptr(X), _stream_ptr()))
        return X

    def evp(self, tau: float, nev: int = 1, ncv: int = None, max_ops: int = 2000, tol: float = 1e-10,
            vectors: bool = False):
        """Linear-stability eigenvalues nearest tau for every pencil slot
        (shift-invert Krylov-Schur, stau_evp): (sigma complex [P, nev],
        resid [P, nev], nconv int32 [P], nops int32 [P], X [nev, *state] or
        None) as device tensors.  ncv defaults to max(2 nev + 8, 20), at
        most 32."""
        t = self._torch
        P = self.info["P"]
        if ncv is None:
            ncv = min(32, max(2 * nev + 8, 20))
        sigma = t.empty((P, nev), dtype=t.complex128, device=self.device)
        resid = t.empty((P, nev), dtype=t.float64, device=self.device)
        nconv = t.empty(P, dtype=t.int32, device=self.device)
        nops = t.empty(P, dtype=t.int32, device=self.device)
        X = t.empty((nev,) + tuple(self.state_shape), dtype=t.complex128, device=self.device) if vectors else None
        self._ok(self.lib.stau_evp(self._pen, float(tau), int(nev), int(ncv), int(max_ops), float(tol),
                                     _ptr(sigma), _ptr(resid), _ptr(nconv), _ptr(nops),
                                     _ptr(X) if X is not None else None, _stream_ptr()))
        return sigma, resid, nconv, nops, X

    def factor(self, a0: float, b0: float = 1.0):
        self._ok(self.lib.stau_factor(self._pen, float(a0), float(b0), _stream_ptr()))

    def last_singular_pencil(self) -> int:
        return int(self.lib.stau_last_singular_pencil(self._pen))

    # -- grid <-> coefficient transforms ------------------------------------
    def vars_mask(self, names) -> int:
        """Bit mask of state variables given by name ("b", "u", ...) or index."""
        order = ("p", "b", "u", "w", "bz", "uz", "wz") if self.dim == 2 else \
            ("p", "b", "u", "v", "w", "bz", "uz", "vz", "wz")
        m = 0
        for v in ([names] if isinstance(names, (str, int)) else names):
            m |= 1 << (order.index(v) if isinstance(v, str) else int(v))
        return m

    def grid_shape(self, nvars: int, scale: float):
        i = self.info
        Lg, Mg = int(round(scale * i["Nx"])), int(round(scale * i["Nz"]))
        if self.dim == 2:
            return (nvars, Lg, Mg)
        return (nvars, Lg, int(round(scale * i["Ny"])), Mg)

    def coeff_to_grid(self, names, scale: float = 1.0, X=None):
        """Grid values (float64 [nvars][x][(y)][z]) of the selected variables."""
        t = self._torch
        m = self.vars_mask(names)
        Xs = (self.X if X is None else X).contiguous()
        g = t.empty(self.grid_shape(bin(m).count("1"), scale), dtype=t.float64, device=self.device)
        self._ok(self.lib.stau_coeff_to_grid(self._pen, _ptr(Xs), m, float(scale), _ptr(g),
                                               _stream_ptr()))
        return g

    def grid_to_coeff(self, names, grid, scale: float = 1.0, X=None):
        """Coefficients of the selected variables from their grid values,
        written into X (default: the solver's state); other variables kept."""
        t = self._torch
        m = self.vars_mask(names)
        g = grid.to(device=self.device, dtype=t.float64).contiguous()
        if tuple(g.shape) != self.grid_shape(bin(m).count("1"), scale):
            raise ValueError(f"grid must have shape {self.grid_shape(bin(m).count('1'), scale)}")
        Xo = self.X if X is None else X
        self._ok(self.lib.stau_grid_to_coeff(self._pen, _ptr(g), m, float(scale), _ptr(Xo),
                                               _stream_ptr()))
        return Xo

    def coeff_to_grid_adjoint(self, names, grid_bar, scale: float = 1.0, X_bar=None):
        t = self._torch
        m = self.vars_mask(names)
        g = grid_bar.to(device=self.device, dtype=t.float64).contiguous()
        Xb = X_bar if X_bar is not None else t.zeros(self.state_shape, dtype=t.complex128,
                                                     device=self.device)
        self._ok(self.lib.stau_coeff_to_grid_adjoint(self._pen, _ptr(g), m, float(scale), _ptr(Xb),
                                                       _stream_ptr()))
        return Xb

    def grid_to_coeff_adjoint(self, names, X_bar, scale: float = 1.0):
        t = self._torch
        m = self.vars_mask(names)
        Xb = X_bar.to(device=self.device, dtype=t.complex128).contiguous()
        g = t.empty(self.grid_shape(bin(m).count("1"), scale), dtype=t.float64, device=self.device)
        self._ok(self.lib.stau_grid_to_coeff_adjoint(self._pen, _ptr(Xb), m, float(scale), _ptr(g),
                                                       _stream_ptr()))
        return g

    # -- components -------------------------------------------------------
    def nonlinear(self, X=None):
        t = self._torch
        Xs = (self.X if X is None else X).contiguous()
        F = t.empty(self.ev_shape, dtype=t.complex128, device=self.device)
        self._ok(self.lib.stau_nonlinear(self._pen, _ptr(Xs), _ptr(F), _stream_ptr()))
        return F

    def solve(self, Bev):
        t = self._torch
        B = Bev.to(device=self.device, dtype=t.complex128).contiguous()
        X = t.empty(self.state_shape, dtype=t.complex128, device=self.device)
        self._ok(self.lib.stau_solve(self._pen, _ptr(B), _ptr(X), _stream_ptr()))
        return X

    def set_kernel_timing(self, enable: bool):
        self._ok(self.lib.stau_set_kernel_timing(self._pen, 1 if enable else 0))

    def read_kernel_timing(self):
        """{kernel kind: (total ms, launches)} since timing was enabled (synchronises)."""
        n = len(_lib.KERNEL_KINDS)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self._ok(self.lib.stau_read_kernel_timing(self._pen, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_KINDS)}

    # -- adjoint ------------------------------------------------------------
    def snapshot(self):
        """Checkpoint of the multistep state (device copies + step counters)."""
        return (self.X.clone(), self.hist.clone(), int(self._st.iteration),
                float(self._st.dt_prev), int(self._st.head))

    def restore(self, snap):
        X, hist, it, dtp, head = snap
        self.X.copy_(X)
        self.hist.copy_(hist)
        self._st.iteration, self._st.dt_prev, self._st.head = it, dtp, head

    def new_adjoint_state(self):
        t = self._torch
        Xbar = t.zeros(self.state_shape, dtype=t.complex128, device=self.device)
        hbar = t.zeros((self.info["P"], 2, self.info["ne"], self.info["Nz"]),
                       dtype=t.complex128, device=self.device)
        return Xbar, hbar

    def adjoint_step(self, X_prev, iteration: int, dt: float, dt_prev: float, Xbar, hbar):
        """Reverse one forward step in place on (Xbar, hbar)."""
        adj = _lib.AdjStateC(Xbar=Xbar.data_ptr(), hbar=hbar.data_ptr())
        self._ok(self.lib.stau_adjoint_step(self._pen, _ptr(X_prev.contiguous()), int(iteration),
                                              float(dt), float(dt_prev), C.byref(adj),
                                              _stream_ptr()))

    def kinetic_energy_adjoint(self, X=None):
        t = self._torch
        Xs = (self.X if X is None else X).contiguous()
        Xbar = t.empty(self.state_shape, dtype=t.complex128, device=self.device)
        self._ok(self.lib.stau_kinetic_energy_adjoint(self._pen, _ptr(Xs), _ptr(Xbar),
                                                        _stream_ptr()))
        return Xbar

    def initial_state_adjoint(self, Xbar):
        t = self._torch
        i = self.info
        shape = (i["Nx"], i["Nz"]) if self.dim == 2 else (i["Nx"], i["Ny"], i["Nz"])
        g = t.empty(shape, dtype=t.float64, device=self.device)
        self._ok(self.lib.stau_initial_state_adjoint(self._pen, _ptr(Xbar.contiguous()), _ptr(g),
                                                       _stream_ptr()))
        return g

    def check(self, X=None):
        Xs = self.X if X is None else X
        self._ok(self.lib.stau_check(self._pen, _ptr(Xs), _stream_ptr()))

    def kinetic_energy_noalloc(self, X=None, out=None):
        """The kinetic energy into a device float64 tensor of one element,
        asynchronously, through the entry point that allocates nothing."""
        t = self._torch
        Xs = (self.X if X is None else X).contiguous()
        o = out if out is not None else t.empty(1, dtype=t.float64, device=self.device)
        self._ok(self.lib.stau_kinetic_energy_noalloc(self._pen, _ptr(Xs), _ptr(o), _stream_ptr()))
        return o

    def kinetic_energy(self, X=None) -> float:
        Xs = (self.X if X is None else X).contiguous()
        out = C.c_double()
        self._ok(self.lib.stau_kinetic_energy(self._pen, _ptr(Xs), C.byref(out), _stream_ptr()))
        return out.value
