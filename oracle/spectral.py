"""Oracle: one-dimensional spectral bases and operator matrices, plain FP64.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file;
only tests, the smoke check and the CPU-baseline leg of the benchmark do.

Every transform here is a dense matrix built straight from the definitions in
the paper (Sec. IV "Fourier basis", "Chebyshev basis", "Scaled transforms &
dealiasing") and every operator matrix straight from Appendix A.  Trig
arguments are reduced in exact integer arithmetic before calling libm, so the
matrices are accurate to a few ulp for any size used here.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# Chebyshev basis (Sec. IV, "Chebyshev basis")
# --------------------------------------------------------------------------

def cheb_grid(Ng: int) -> np.ndarray:
    """Gauss-Chebyshev nodes x_i = -cos(pi (i + 1/2) / Ng), ascending on [-1, 1]."""
    i = np.arange(Ng)
    return -np.cos(np.pi * (i + 0.5) / Ng)


def cheb_T_on_grid(Nc: int, Ng: int) -> np.ndarray:
    """Matrix T[j, n] = T_n(x_j) for the Ng-point Gauss grid, n < Nc.

    T_n(x) = cos(n arccos x) (Sec. II, Chebyshev polynomials).  On this grid
    arccos(x_j) = pi (2 Ng - 2 j - 1) / (2 Ng) exactly, so
    n arccos(x_j) = pi m / (2 Ng) with the integer m = n (2 Ng - 2 j - 1),
    reduced modulo 4 Ng before the cosine is taken.
    """
    j = np.arange(Ng, dtype=np.int64)[:, None]
    n = np.arange(Nc, dtype=np.int64)[None, :]
    m = (n * (2 * Ng - 2 * j - 1)) % (4 * Ng)
    return np.cos(np.pi * m.astype(np.float64) / (2 * Ng))


def cheb_backward_matrix(Nc: int, Ng: int) -> np.ndarray:
    """Coefficients -> grid values on the Ng grid (padding above Nc, Sec. IV
    "Scaled transforms"): g_j = sum_{n<Nc} c_n T_n(x_j).  Shape (Ng, Nc)."""
    return cheb_T_on_grid(Nc, Ng)


def cheb_forward_matrix(Nc: int, Ng: int) -> np.ndarray:
    """Grid values -> first Nc coefficients (truncation):
    c_n = (2 - delta_{n0}) / Ng * sum_j f(x_j) T_n(x_j).  Shape (Nc, Ng)."""
    T = cheb_T_on_grid(Nc, Ng)
    w = np.full(Nc, 2.0 / Ng)
    w[0] = 1.0 / Ng
    return w[:, None] * T.T


# --------------------------------------------------------------------------
# Fourier basis (Sec. IV, "Fourier basis")
# --------------------------------------------------------------------------

def _expi(num: np.ndarray, den: int, sign: int) -> np.ndarray:
    """exp(sign * 2 pi i num / den) with num reduced mod den in integers."""
    r = (num % den).astype(np.float64)
    ang = 2.0 * np.pi * r / den
    return np.cos(ang) + sign * 1j * np.sin(ang)


def fourier_kmax(Nc: int) -> int:
    """Largest kept wavenumber: floor((Nc-1)/2); the Nyquist mode is dropped."""
    return (Nc - 1) // 2


def fourier_real_backward_matrix(Nc: int, Ng: int) -> np.ndarray:
    """Half-spectrum -> real grid values (real data keeps k >= 0 only).

    f(x_i) = sum_{|k|<=km} f_k e^{i k x_i} with f_{-k} = conj(f_k), x_i = 2 pi i/Ng.
    Returned E has shape (Ng, km+1) and f = Re(E @ c): column k carries the
    weight 1 for k = 0 and 2 for k > 0 (the k and -k terms together).
    """
    km = fourier_kmax(Nc)
    i = np.arange(Ng, dtype=np.int64)[:, None]
    k = np.arange(km + 1, dtype=np.int64)[None, :]
    E = _expi(i * k, Ng, +1)
    w = np.full(km + 1, 2.0)
    w[0] = 1.0
    return E * w[None, :]


def fourier_real_forward_matrix(Nc: int, Ng: int) -> np.ndarray:
    """Real grid values -> coefficients f_k = (1/Ng) sum_i f(x_i) e^{-i k x_i},
    0 <= k <= km.  Shape (km+1, Ng)."""
    km = fourier_kmax(Nc)
    k = np.arange(km + 1, dtype=np.int64)[:, None]
    i = np.arange(Ng, dtype=np.int64)[None, :]
    return _expi(k * i, Ng, -1) / Ng


def fourier_signed_wavenumbers(Nc: int) -> np.ndarray:
    """Signed integer wavenumbers in storage order 0..km, (Nyquist slot), -km..-1.

    The Nyquist slot (Nc/2 for even Nc) is kept in storage and held at zero;
    its entry here is 0 and `fourier_complex_active(Nc)` marks it inactive.
    """
    k = np.fft.fftfreq(Nc, 1.0 / Nc).astype(np.int64)
    if Nc % 2 == 0:
        k[Nc // 2] = 0
    return k


def fourier_complex_active(Nc: int) -> np.ndarray:
    act = np.ones(Nc, dtype=bool)
    if Nc % 2 == 0:
        act[Nc // 2] = False
    return act


def fourier_complex_backward_matrix(Nc: int, Ng: int) -> np.ndarray:
    """Complex series on all stored slots -> grid: f(x_i) = sum_k f_k e^{i k x_i}.
    Shape (Ng, Nc); the Nyquist column is zero."""
    k = fourier_signed_wavenumbers(Nc)[None, :]
    i = np.arange(Ng, dtype=np.int64)[:, None]
    E = _expi(i * k, Ng, +1)
    E[:, ~fourier_complex_active(Nc)] = 0.0
    return E


def fourier_complex_forward_matrix(Nc: int, Ng: int) -> np.ndarray:
    """Grid -> complex series coefficients on all stored slots (Nyquist row zero)."""
    k = fourier_signed_wavenumbers(Nc)[:, None]
    i = np.arange(Ng, dtype=np.int64)[None, :]
    F = _expi(k * i, Ng, -1) / Ng
    F[~fourier_complex_active(Nc), :] = 0.0
    return F


# --------------------------------------------------------------------------
# Chebyshev operator matrices (Sec. II "Sparse differential operators",
# Appendix A "Differentiation and conversion matrices", "Dirichlet
# recombination matrices", "NCC multiplication matrices").  Native [-1, 1].
# --------------------------------------------------------------------------

def cheb_conversion_TU(N: int) -> np.ndarray:
    """P^L_{ij} = <U_i|T_j> = (delta_{ij} - delta_{i,j-2}) / (2 - delta_{j0})."""
    P = np.zeros((N, N))
    for j in range(N):
        s = 1.0 / (2.0 - (1.0 if j == 0 else 0.0))
        P[j, j] += s
        if j >= 2:
            P[j - 2, j] -= s
    return P


def cheb_diff_TU(N: int) -> np.ndarray:
    """<U_i| d/dx T_j> = j delta_{i,j-1}  (dT_n/dx = n U_{n-1})."""
    D = np.zeros((N, N))
    for j in range(1, N):
        D[j - 1, j] = j
    return D


def cheb_diff_TT(N: int) -> np.ndarray:
    """Dense T-to-T derivative D_{ij} = 2 j ((j - i) mod 2) / (1 + delta_{i0}) [i < j]."""
    D = np.zeros((N, N))
    for i in range(N):
        for j in range(i + 1, N):
            D[i, j] = 2.0 * j * ((j - i) % 2) / (1.0 + (1.0 if i == 0 else 0.0))
    return D


def cheb_dirichlet_PR(N: int) -> np.ndarray:
    """P^R_{ij} = <T_i|D_j> = delta_{ij} - delta_{i,j-2} [j > 1]."""
    P = np.eye(N)
    for j in range(2, N):
        P[j - 2, j] -= 1.0
    return P


def cheb_interp_row(N: int, side: str) -> np.ndarray:
    """Interpolation vector T_n(+-1) = (+-1)^n; 'left' is x=-1, 'right' is x=+1."""
    n = np.arange(N)
    if side == "left":
        return np.where(n % 2 == 0, 1.0, -1.0)
    if side == "right":
        return np.ones(N)
    raise ValueError(side)


def cheb_integ_row(N: int) -> np.ndarray:
    """Integration vector over [-1, 1]: int T_n = 2 / (1 - n^2) for even n, 0 for odd n."""
    n = np.arange(N, dtype=np.float64)
    out = np.zeros(N)
    ev = (np.arange(N) % 2) == 0
    out[ev] = 2.0 / (1.0 - n[ev] ** 2)
    return out
