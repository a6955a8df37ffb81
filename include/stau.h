/*
 * stau -- sparse generalized-tau IMEX stepper for Fourier x Chebyshev
 * Rayleigh-Benard convection on one gfx950 GPU.  C ABI.
 *
 * The operation is one implicit-explicit multistep step (SBDF1 on the first
 * step, SBDF2 afterwards) of the first-order sparse tau discretisation of
 * Burns et al., "Dedalus: A flexible framework for numerical simulations
 * with spectral methods" (2020):
 *   Sec. II   -- T-to-U differentiation/conversion, tau rows, Dirichlet
 *                recombination, interleaved (mode-major) banded systems;
 *   Sec. IV   -- Fourier / Chebyshev transforms, 3/2 dealiasing;
 *   Sec. IX   -- pencil matrix construction, IVP form M dX/dt + L X = F,
 *                multistep IMEX update (a0 M + b0 L) X^n = B^n, factor reuse.
 *
 * Conventions common to every call
 * --------------------------------
 * - Every function returns an int status (STAU_OK = 0, else an STAU_E* code);
 *   the message of the last failure on the calling thread is returned by
 *   stau_last_error().  No C++ exception crosses this boundary.
 * - Pointers documented as "device" are HIP device pointers on the domain's
 *   device; the caller owns them and must keep them alive for the call (and
 *   for the enqueued work, when the call is asynchronous).  The library never
 *   frees caller memory.  Handles (stau_domain, stau_pencils) are library
 *   owned and released by the matching destroy call.
 * - `stream` is a hipStream_t (NULL = the default stream).  All device work of
 *   a call is enqueued on it.  Only stau_factor, stau_check and the destroy
 *   calls synchronise the host with the device.
 * - Complex arrays are interleaved (re, im) float64 pairs (C99 double complex).
 *
 * State layout (the FieldSystem of Sec. VI, pencil-major, variable-major inside)
 * ---------------------------------------------------------------------------
 *   2-D: X[kx][var][n],  kx = 0..Nx/2 (slot Nx/2 is the Nyquist mode, kept 0),
 *        var in (p, b, u, w, bz, uz, wz), n = 0..Nz-1 Chebyshev T coefficients
 *        of z in [0, 1] (native [-1, 1] by z = (zeta + 1) / 2).
 *   3-D: X[ky][kx][var][n], ky in FFT order (0..Ny/2-1, Nyquist, -Ny/2+1..-1),
 *        var in (p, b, u, v, w, bz, uz, vz, wz).
 *   Fourier coefficients are mode amplitudes: f(x) = sum_k f_k e^{i k 2 pi x/Lx}.
 */
#ifndef STAU_H
#define STAU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STAU_OK 0
#define STAU_EINVAL 1        /* bad argument: null pointer, shape, dt <= 0 ... */
#define STAU_ENOMEM 2        /* device or host allocation failed */
#define STAU_EHIP 3          /* a HIP runtime call failed (message in last_error) */
#define STAU_ESINGULAR 4     /* zero or non-finite pivot in a pencil factorisation */
#define STAU_ESTATE 5        /* call not valid in the current state */
#define STAU_EUNSUPPORTED 6  /* size or option not supported */
#define STAU_ENONFINITE 7    /* non-finite value detected by stau_check */
#define STAU_EBOUNDS 8       /* index check failed (check builds only, reported by stau_check) */

#define STAU_FP64 0
#define STAU_MIXED 1

#define STAU_DCT_AUTO 0
#define STAU_DCT_FFT 1
#define STAU_DCT_MATMUL 2

#define STAU_SOLVE_AUTO 0
#define STAU_SOLVE_FP64 1
#define STAU_SOLVE_REFINED 2

#define STAU_FACTORS_AUTO 0
#define STAU_FACTORS_BAND 1

/* IMEX Runge-Kutta schemes of stau_step_rk: the (1,1,1), (2,2,2) and (4,4,3)
 * schemes of Ascher, Ruuth & Spiteri (1997), orders 1, 2, 3, with 1, 2, 4
 * implicit stages. */
#define STAU_RK111 1
#define STAU_RK222 2
#define STAU_RK443 3

typedef struct stau_domain stau_domain;
typedef struct stau_pencils stau_pencils;

/* Domain: direct product of Fourier (x[, y]) and Chebyshev (z) bases (Sec. V).
 * dim      2 or 3.
 * Nx, Ny   Fourier modes: powers of two in [4, 4096] (Ny ignored in 2-D); the
 *          dealiased grids have 3Nx/2 and 3Ny/2 points.
 * Nz       Chebyshev modes: a power of two in [4, 512] (3Nz/2 grid points).
 * Lx, Ly   periods of x, y (> 0).
 * dealias  transform scale; must be 1.5 (the 3/2 rule, Sec. IV).
 * precision STAU_FP64 (everything FP64) or STAU_MIXED (FP32 transforms and
 *          products in stau_step, stau_step_rk and stau_adjoint_step; the
 *          pencil factorisation, the adjoint's transposed solve, the state,
 *          history, right-hand side and their adjoints FP64; the step's
 *          solve as mixed_solve selects.)  The
 *          component calls (stau_nonlinear, stau_solve) and the
 *          kinetic-energy and initial-state adjoints run in FP64 in either
 *          mode.
 * device   HIP device ordinal.
 * dct_method  Chebyshev z transforms of the step: STAU_DCT_AUTO (matrix
 *          products for Nz <= 64, FFT otherwise), STAU_DCT_FFT (DCT through
 *          one complex FFT per column), STAU_DCT_MATMUL (dense products on the
 *          FP64 matrix cores; Nz a multiple of 32 in [32, 256], else
 *          STAU_EUNSUPPORTED).  In the mixed-precision step the products
 *          run as split-BF16 matrix-core products with FP32 accumulation
 *          (each operand split into three BF16 terms): STAU_DCT_MATMUL needs
 *          Nz = 64, 128 or 256 there (else STAU_EUNSUPPORTED) and
 *          STAU_DCT_AUTO takes them for Nz = 64; otherwise the mixed step
 *          uses the FP32 FFT.
 * mixed_solve  the pencil solve of the mixed-precision steps (ignored in
 *          FP64 domains): STAU_SOLVE_FP64 (FP64 sweeps on the FP64 factors),
 *          STAU_SOLVE_REFINED (FP32 sweeps on FP32 copies of the FP64
 *          factors, the residual of the first solution in FP64 from the
 *          operator templates, one FP32 correction sweep, the sum in FP64; in
 *          the single-block or the two-block sweep layout, as the FP64 solve
 *          uses), STAU_SOLVE_AUTO (FP64, the faster of the two at every size
 *          measured).  Else STAU_EINVAL.
 * factor_layout  storage of the factors the FP64 pencil solve reads (Sec. IX
 *          "Matrix solvers": the factors of the sparse banded pencil
 *          matrices are stored and reused while dt is fixed):
 *          STAU_FACTORS_AUTO (where the solve streams its vectors through
 *          device memory, i.e. single-block layouts with more than 32 pencils
 *          per compute unit, the nonzero entries are also packed into sparse
 *          records after each factorisation and the solve reads those;
 *          whole-band factors elsewhere), STAU_FACTORS_BAND (whole-band
 *          factors only).  Both give the same results.  Else STAU_EINVAL. */
typedef struct stau_domain_desc {
  int32_t dim;
  int32_t precision;
  int64_t Nx, Ny, Nz;
  double Lx, Ly;
  double dealias;
  int32_t device;
  int32_t dct_method;
  int32_t mixed_solve;
  int32_t factor_layout;
} stau_domain_desc;

/* Rayleigh-Benard parameters in free-fall units: kappa = (Ra Pr)^(-1/2),
 * nu = (Ra / Pr)^(-1/2).  buoyancy multiplies the -b term of the w equation
 * (1 for convection, 0 for pure diffusion checks).  b_bottom / b_top are the
 * Dirichlet values of b at z = 0 / z = 1; u = (v =) w = 0 on both walls.
 * n_gamma, gamma: an optional non-constant coefficient (Sec. II, NCCs)
 * Gamma(z) = sum_{k < n_gamma} gamma[k] T_k(2 z - 1) multiplying w in the b
 * equation (a background stratification: d_t b + Gamma w - kappa lap b = ...),
 * entered on the left-hand side as its truncated Chebyshev product matrix.
 * n_gamma in [0, 4] (0: none, else STAU_EINVAL); it widens the pencil band
 * by about S per term, and stau_build_pencils returns STAU_EUNSUPPORTED when
 * the band exceeds the sweep windows (kl < 32, kl + ku < 64: n_gamma <= 3 in
 * 2-D, <= 2 in 3-D).  The adjoint calls need the transposed band to fit too
 * (2-D: n_gamma <= 2), else they return STAU_EUNSUPPORTED. */
typedef struct stau_rb_params {
  double Ra, Pr, buoyancy, b_bottom, b_top;
  int32_t n_gamma;
  int32_t reserved;
  double gamma[4];
} stau_rb_params;

/* Multistep state, caller owned.
 * X     device, complex128, state layout above (read as X^{n-1}, overwritten
 *       with X^n by stau_step).
 * hist  device, complex128, [2][P][2][ne][Nz]: for the two latest steps, the
 *       left-preconditioned explicit term F~ = P^L F and M~X (evolved equation
 *       U-rows only; ne = 3 in 2-D, 4 in 3-D; P = number of pencil slots).
 * iteration  number of steps taken so far (0 selects SBDF1).
 * dt_prev    previous timestep (ignored when iteration == 0).
 * head       slot of hist holding step n-1 (updated by stau_step). */
typedef struct stau_state {
  void* X;
  void* hist;
  int64_t iteration;
  double dt_prev;
  int32_t head;
  int32_t reserved;
} stau_state;

/* Sizes derived from a domain (filled by stau_query). */
typedef struct stau_info {
  int64_t Nx, Ny, Nz, Ngx, Ngy, Ngz;
  int64_t Px;          /* Nx/2 + 1 rfft slots along x */
  int64_t P;           /* pencil slots: Px (2-D) or Ny*Px (3-D) */
  int64_t P_active;    /* pencils solved: Nx/2 (2-D) or (Nx/2)(Ny-1) (3-D) */
  int64_t S;           /* variables per pencil: 7 or 9 */
  int64_t ne;          /* evolved fields: 3 or 4 */
  int64_t n;           /* unknowns per pencil S*Nz */
  int64_t kl, ku;      /* band widths of the interleaved pencil matrix */
  int64_t state_elems; /* complex elements of X */
  int64_t hist_elems;  /* complex elements of hist */
  int64_t workspace_bytes; /* device bytes held by the pencils object */
} stau_info;

/* Create a domain (validates sizes, builds FP64 twiddle and Chebyshev tables
 * on the host and uploads them).  Sec. IV, V. */
int stau_create_domain(const stau_domain_desc* desc, stau_domain** out);
int stau_destroy_domain(stau_domain* dom);

/* Build the pencil system of the Rayleigh-Benard problem on a domain:
 * operator templates of Appendix A (T-to-U conversion P^L, derivative
 * dT_n = n U_{n-1}, boundary rows T_n(+-1) = (+-1)^n, Dirichlet recombination
 * P^R), row processing of Sec. IX "Matrix construction", interleaved mode-major
 * ordering, and the device workspaces.  The pencils object keeps a pointer to
 * the domain, which must outlive it. */
int stau_build_pencils(stau_domain* dom, const stau_rb_params* par, stau_pencils** out);
int stau_destroy_pencils(stau_pencils* pen);
int stau_query(const stau_pencils* pen, stau_info* info);

/* Assemble a0 M~ + b0 L~ for every pencil on the device and factor it by
 * banded LU with partial pivoting (Sec. IX: factorisations are stored and
 * reused while a0, b0 are unchanged).  Synchronises `stream`.  Returns
 * STAU_ESINGULAR if a pivot is zero or non-finite; the first such pencil index
 * is then returned by stau_last_singular_pencil(). */
int stau_factor(stau_pencils* pen, double a0, double b0, void* stream);
int64_t stau_last_singular_pencil(const stau_pencils* pen);

/* One IMEX step (Sec. IX "Multistep IMEX integrators"): SBDF1 when
 * st->iteration == 0, else variable-step SBDF2 with w = dt / st->dt_prev.
 * Evaluates the explicit term on the dealiased grid, forms
 * B = sum_j c_j F~^{n-j} - a_j M~X^{n-j}, solves (a0 M~ + b0 L~) X~ = B per
 * pencil and recovers X = P^R X~.  Refactors (synchronously) when (a0, b0)
 * differ from the stored factorisation.  Updates st->X, st->hist and the
 * host fields iteration, dt_prev, head.  Asynchronous otherwise. */
int stau_step(stau_pencils* pen, stau_state* st, double dt, void* stream);

/* One IMEX Runge-Kutta step X^n -> X^{n+1} (Sec. IX "Runge-Kutta IMEX
 * integrators"), in place on X (device, state layout).  For the stages
 * i = 1..s of `scheme` (STAU_RK111, STAU_RK222, STAU_RK443; else
 * STAU_EINVAL) it evaluates the explicit term of X^{n,i-1} on the dealiased
 * grid and solves, per pencil,
 *   (M~ + dt H_ii L~) X~^{n,i} = M~X^{n,0} + dt sum_{j<i} A_ij F~^{n,j}
 *                                 - dt sum_{j<i} H_ij L~X^{n,j},
 * recovering X^{n,i} = P^R X~^{n,i}; the last stage is X^{n+1}.  The stage
 * operator is factored as M~ / (dt H_ii) + L~ (one factorisation per dt, the
 * schemes' H_ii are equal; refactored synchronously when no stored
 * factorisation matches).  The stage values F~ and L~X live in a workspace of
 * the pencils object (allocated on the first call with a larger scheme:
 * max(1, 2s - 2) arrays of P ne Nz complex entries).  Needs no history: every step is full order, dt may change from
 * step to step.  In a STAU_MIXED domain the transforms and products run as in
 * stau_step (FP32; the solve FP64).  Asynchronous otherwise. */
int stau_step_rk(stau_pencils* pen, int scheme, double dt, void* X, void* stream);

/* Linear boundary value solve (Sec. IX "Linear boundary value solver"): per
 * pencil, L~ X~ = P^L F with the boundary rows taking the problem's Dirichlet
 * values and the z-derivative and continuity rows zero, then X = P^R X~.
 * F is device complex128 [P][ne][Nz] (2-D) / [Ny][Px][ne][Nz] (3-D): the T
 * coefficients of the right side of each evolved equation (b, u, [v], w;
 * -kappa lap b = F_b, -nu lap u + grad p - b e_z = F_u), read only for
 * active pencils.  X (device, state layout) is written entirely.  Factors
 * L~ (a0 = 0, b0 = 1) into the factorisation cache (synchronously when no
 * stored factorisation matches); the solve is FP64 in either precision
 * mode.  Asynchronous otherwise. */
int stau_lbvp(stau_pencils* pen, const void* F, void* X, void* stream);

/* Linear stability of the conduction state b0(z) = b_bottom + (b_top - b_bottom) z
 * (Sec. IX "Eigenvalue solver"): for every active pencil, the nev eigenvalues
 * sigma of  sigma M~ X + (L~ + L~') X = 0  nearest the real shift tau, where
 * L~' is the explicit term -w d_z b linearised about b0 and moved to the left
 * ((b_top - b_bottom) P^L w on the b rows).  Shift-invert Krylov-Schur
 * iteration: Arnoldi steps with T = A^{-1} M~ (the banded LU of
 * A = tau M~ + L~ + L~', factored by this call when tau changed,
 * synchronously; whole-band layout, kept apart from the step's factors) on a
 * basis of at most ncv vectors, Rayleigh-Ritz on the projected matrix, and
 * thick restarts that keep nev plus half of the remaining Ritz vectors, until
 * the nev Ritz values theta = 1 / (tau - sigma) of largest modulus have
 * converged or max_ops applications of T (exceeded by at most ncv) are spent.
 * sigma    device complex128 [P][nev] (float64 pairs): sigma = tau - 1 / theta,
 *          nearest tau first (0 for inactive slots; NaN for a value the
 *          iteration could not determine)
 * resid    device float64 [P][nev]: |T x - theta x| / |theta| of the Ritz
 *          pair (the Krylov estimate |beta y_last| / |theta|; for a complex
 *          pair that of its two-dimensional invariant subspace)
 * nconv    device int32 [P]: how many of the nev have resid <= tol
 * nops     device int32 [P] or NULL: applications of T spent
 * X        device complex128 [nev][P][state] or NULL: the eigenvectors
 *          (unit 2-norm of the real-scaled vector; X = P^R x with u-type
 *          variables scaled by -i; zero for inactive slots)
 * 1 <= nev <= 16, nev + 2 <= ncv <= min(32, pencil size), ncv <= max_ops <=
 * 1e6, 0 < tol < 1, else STAU_EINVAL; STAU_ESINGULAR when tau is an
 * eigenvalue of a pencil; STAU_ENOMEM when the bases (P (ncv + 1) n doubles,
 * kept for later calls) cannot be allocated.  Asynchronous after the
 * factorisation. */
int stau_evp(stau_pencils* pen, double tau, int nev, int ncv, int max_ops, double tol, double* sigma,
             double* resid, int32_t* nconv, int32_t* nops, void* X, void* stream);

/* Initial state from real scale-1 grid values of b (Sec. IX "Initial
 * conditions": the state is set in grid space and must satisfy the problem's
 * constraints; Sec. VI "Data manipulation").  b_grid is device float64,
 * 2-D b[ix][jz], 3-D b[ix][ly][jz], on the Chebyshev Gauss grid in z
 * (ascending) and x_i = Lx i / Nx, y_l = Ly l / Ny.  Forward transforms, then
 * bz = d_z b by the Chebyshev derivative recursion (so the first-order
 * constraint bz - d_z b = 0 holds), every other variable zero.  X (device,
 * state layout) is written entirely.  Asynchronous. */
int stau_initial_state(stau_pencils* pen, const double* b_grid, void* X, void* stream);

/* Grid <-> coefficient transforms of selected state variables (Sec. VI "Data
 * manipulation": the grid and coefficient data of a field; Sec. IV "Scaled
 * transforms & dealiasing": the transforms evaluated at a chosen scale).
 * vars     bit mask of the variables of the state layout (bit v: variable v in
 *          ABI order; non-empty, no bit at or above S, else STAU_EINVAL); the
 *          grid holds the selected variables in increasing order.
 * scale    1 (Nx x [Ny x] Nz grid points) or 1.5 (the dealiased 3/2 grid),
 *          else STAU_EINVAL.
 * grid     device float64 [nvars][Lg][Mg] (2-D) / [nvars][Lg][Lgy][Mg] (3-D),
 *          Lg = scale Nx, Lgy = scale Ny, Mg = scale Nz: x_i = Lx i / Lg,
 *          y_l = Ly l / Lgy, z_j = (1 - cos(pi (j + 1/2) / Mg)) / 2 ascending.
 * X        device complex128, state layout.
 * stau_coeff_to_grid: grid = sum over the stored modes (Nyquist modes
 *          excluded) of c e^{i k.x} T_n(2 z - 1), real.  X is only read.
 * stau_grid_to_coeff: the truncating forward transform (discrete
 *          orthogonality on the grid): coefficients of the selected variables
 *          for every pencil slot (Nyquist and unused slots zero); the other
 *          variables of X are left unchanged.  At scale 1 this inverts
 *          stau_coeff_to_grid on band-limited data.
 * The two adjoint calls are the exact transposes under the real inner
 * products (a complex coefficient is a pair of reals, so the adjoint of z is
 * dJ/dRe z + i dJ/dIm z):
 * stau_coeff_to_grid_adjoint: X_bar (selected variables overwritten, the
 *          others unchanged) = adjoint of stau_coeff_to_grid applied to grid_bar;
 * stau_grid_to_coeff_adjoint: grid_bar (written entirely) = adjoint of
 *          stau_grid_to_coeff applied to the selected variables of X_bar.
 * All four use the pencils object's transform workspaces (calls on one
 * pencils object are ordered on their streams) and are asynchronous. */
int stau_coeff_to_grid(stau_pencils* pen, const void* X, uint32_t vars, double scale, double* grid,
                       void* stream);
int stau_grid_to_coeff(stau_pencils* pen, const double* grid, uint32_t vars, double scale, void* X,
                       void* stream);
int stau_coeff_to_grid_adjoint(stau_pencils* pen, const double* grid_bar, uint32_t vars, double scale,
                               void* X_bar, void* stream);
int stau_grid_to_coeff_adjoint(stau_pencils* pen, const void* X_bar, uint32_t vars, double scale,
                               double* grid_bar, void* stream);

/* Explicit term alone: F = coefficients of -(u.grad) q for q in the evolved
 * fields, evaluated on the 3/2 grid (Sec. IV) from the state X.  F is device
 * complex128 [P][ne][Nz] (2-D) / [Ny][Px][ne][Nz] (3-D); inactive slots are
 * written as zero. */
int stau_nonlinear(stau_pencils* pen, const void* X, void* F, void* stream);

/* Pencil solve alone with the factors of the operator (a0, b0) of the last
 * successful stau_factor (refactored synchronously when later steps or
 * boundary value solves have evicted them from the two-slot cache; STAU_ESTATE
 * before any successful stau_factor).  B_ev is device complex128
 * [P][ne][Nz] holding the right-hand sides of the evolved-equation U-rows
 * n = 0..Nz-2 (entry Nz-1 ignored); the z-derivative and continuity rows are
 * zero and the boundary rows take the problem's Dirichlet values.  Writes X
 * (state layout).  Sec. IX "Linear boundary value solver". */
int stau_solve(stau_pencils* pen, const void* B_ev, void* X, void* stream);

/* Synchronise and check the device error flag and the state for non-finite
 * values.  Returns STAU_ENONFINITE if X holds a NaN/Inf.  In the check build
 * (libstau_check.so, compiled with STAU_CHECK_BOUNDS) the kernels also record
 * index checks (the factorisation's pivot offsets within the band, the
 * forward sweeps' window slots, the sparse factor records' sizes and ranks)
 * in a word per pencils object; stau_check then returns STAU_EBOUNDS if any
 * failed since stau_build_pencils.  A failed check never traps: the kernels
 * carry on, and the result of that call is not to be trusted. */
int stau_check(stau_pencils* pen, const void* X, void* stream);

/* Kinetic-energy functional J = (1/V) int |u|^2 / 2 evaluated on the 3/2 grid
 * with truncated forward transforms and the Chebyshev integration vector
 * (Sec. VII "Integration"); result written to *out (host) after a sync. */
int stau_kinetic_energy(stau_pencils* pen, const void* X, double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the kinetic-energy
 * functional of stau_kinetic_energy, with the same kernels and result, that
 * allocates nothing and does not synchronise.  `out` is a device double
 * written asynchronously on `stream`.  Every intermediate lives in a
 * library-owned device array of 64 MiB per GPU (held until the process
 * ends); domains whose intermediates exceed it (2-D: 2 fields x 3Nz/2 x
 * (Nx/2 + 1) complex entries, 3-D: 3 fields on the z and y grids) return
 * STAU_EUNSUPPORTED.  Calls on one GPU share that array: calls that overlap
 * in time on one GPU (concurrent streams, several host threads) race and
 * must be ordered by the caller. */
int stau_kinetic_energy_noalloc(stau_pencils* pen, const void* X, double* out, void* stream);

/* ------------------------------------------------------------------------
 * Discrete adjoint (2-D domains; the three calls below return
 * STAU_EUNSUPPORTED for dim = 3).  The adjoint of a complex coefficient z is
 * dJ/dRe z + i dJ/dIm z (coefficients are pairs of independent reals), so a
 * complex-linear map y = A x has x_bar = A^H y_bar.
 * ------------------------------------------------------------------------ */

/* Adjoint state, caller owned.
 * Xbar  device complex128, state layout: on entry the adjoint of X^n, on exit
 *       the adjoint of X^{n-1} (overwritten in place).
 * hbar  device complex128 [P][2][ne][Nz]: adjoints of the history entries
 *       (F~ and M~X of step n-1) pending from the step after; zero before the
 *       last step is reversed; on exit, those of step n-2. */
typedef struct stau_adjstate {
  void* Xbar;
  void* hbar;
} stau_adjstate;

/* Reverse of one stau_step (the exact derivative of the discrete forward
 * map): X_prev is the state X^{n-1} the forward step started from (device,
 * state layout), iteration the forward step's st->iteration (0: SBDF1), dt
 * and dt_prev its timesteps.  Computes, per pencil,
 *   B_bar = A^{-H} X_bar (transposed banded solve with the stored factors),
 *   F~_bar = c1 B_bar + pending, M~X_bar = -a1 B_bar + pending,
 *   X_bar^{n-1} = M^H M~X_bar + N'(X^{n-1})^H (P^L)^H F~_bar
 * where N' is the linearised explicit term (adjoint transforms and products on
 * the 3/2 grid).  Uses cached factors of (a0, b0), refactoring synchronously
 * if neither stored factorisation matches.  In a STAU_MIXED domain the
 * adjoint transforms and products run in FP32 (the transposed solve in FP64).
 * The forward grid fields at X_prev are transformed on an internal
 * non-blocking stream of the pencils object, forked from and joined back to
 * `stream` with events, so the call stays ordered on `stream` alone.  Sec. IX (IVP, multistep IMEX) is
 * the forward operation; the adjoint is not part of the paper. */
int stau_adjoint_step(stau_pencils* pen, const void* X_prev, int64_t iteration, double dt,
                      double dt_prev, stau_adjstate* adj, void* stream);

/* Xbar (device, state layout, written entirely) = dJ/dX of the kinetic-energy
 * functional of stau_kinetic_energy at the state X. */
int stau_kinetic_energy_adjoint(stau_pencils* pen, const void* X, void* Xbar, void* stream);

/* Adjoint of stau_initial_state: b_grid_bar (device float64, layout of the b
 * grid, written entirely) = dJ/d b_grid given Xbar = dJ/dX^0. */
int stau_initial_state_adjoint(stau_pencils* pen, const void* Xbar, double* b_grid_bar,
                               void* stream);

/* Measurement hook: when enabled, every kernel launched by stau_step and
 * stau_factor is bracketed by two HIP events recorded on the call's stream.
 * stau_read_kernel_timing synchronises on those events, writes the summed
 * elapsed milliseconds and launch counts per kernel kind (0 backward z
 * transform, 1 x pass with products, 2 forward z transform with right-hand
 * side assembly, 3 pencil solve, 4 pencil factorisation, 5 backward and
 * forward y transforms of 3-D domains) into ms[] and
 * launches[] (caller-owned host arrays of nkinds entries) and clears the
 * record. */
int stau_set_kernel_timing(stau_pencils* pen, int enable);
int stau_read_kernel_timing(stau_pencils* pen, double* ms, int64_t* launches, int nkinds);

const char* stau_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STAU_H */
