// Internal launcher interface between the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace stau {

constexpr int kMaxFields = 16;

struct PencilArgs {
  SysDesc desc;
  int n, kl, ku, FW, BW;
  int nst;    // factor columns stored per pencil (n rounded up to the sweep chunk; zero beyond n)
  int trans;  // 1: the factors are those of the transposed matrix
  // two-block solve: blk 0 = the whole system; 1 = the leading block (rows
  // and columns 0 .. n-1 of the whole system of size nfull); 2 = the trailing
  // block in reversed order (block index i <-> whole index nfull - 1 - i).
  // Q = kl + ku of the whole operator.
  int blk, nfull, Q;

  int P, Px, Ny;
  double kappa, nu, buoyancy, b_bottom, b_top;
  double lin;  // PencilCoef::lin of every pencil (0 for the step's operators)
  double refine_a0, refine_b0;  // operator of the refined mixed solve's residual
  double* ysp;  // solve workspace [P][2][nst] for the streamed solve (or null)
  // index-check word of builds with STAU_CHECK_BOUNDS (bits of the checks
  // that failed; null in other builds)
  unsigned int* check;
  // Band templates of the whole operator (row R, column C at R * tw + C - R + tkl):
  // a0 M~ + b0 L~ = a0 T0 + b0 (T1 + k^2 T2 + kx T3 + ky T4 + lin T5), with
  // T1 of the mean pencil (gauge row) in its own plane: planes T0, T1, T1 mean,
  // T2, T3, T4, T5, each tplane doubles
  const double* tpl;
  int tkl, tw;
  long long tplane;
  int nncc;    // non-constant coefficient Gamma(z): Chebyshev terms (0: none)
  double ncc[kMaxNcc];
  double two_pi_over_Lx, two_pi_over_Ly;
  int var_of_abi[9];
};

// Sparse records of one factor slot for the streamed solve (k_pencil.hip):
// per pencil, units of kSpU columns at fixed strides, record lengths in
// 16-byte words (kSpLen bytes per pencil and direction).
constexpr int kSpU = 8;
constexpr int kSpLen = 256;
struct SparseFactors {
  uint8_t* F;      // forward records [P][nst / kSpU][strideF]
  uint8_t* B;      // backward records [P][nst / kSpU][strideB]
  uint8_t* lenF;   // [P][kSpLen]
  uint8_t* lenB;   // [P][kSpLen]
  int strideF, strideB;
};

struct XformArgs {
  int dim;
  int N, M;          // Chebyshev modes, dealiased z grid
  int Nx, L;         // Fourier x modes, dealiased x grid
  int Pa, Px;        // active kx (Nx/2), kx slots (Nx/2 + 1)
  int Ny, Ngy;       // 3-D only
  int P;             // pencil slots = row length of the z-transform outputs
  int S, ne;
  double two_pi_over_Lx, two_pi_over_Ly;
  const double2* twz;   // e^{-2 pi i t / M}
  const double2* dctz;  // e^{+i pi n / (2 M)}
  const double2* twx;   // e^{-2 pi i t / L}
  const double2* twy;   // e^{-2 pi i t / Ngy}
  // FP32 copies (rounded from the FP64 tables) for the mixed-precision path
  const float2* twz32;
  const float2* dctz32;
  const float2* twx32;
  const float2* twy32;
};

// Field list for the backward z transform: source variable index and
// derivative flag (0: none, 1: multiply by i kx, 2: multiply by i ky).  The
// source array is [P][src_S][N]; wmode 1 multiplies coefficient n by the
// forward-transform weight (2 - delta_n0) / M first (adjoint of the forward z
// transform).
struct FieldList {
  int nf;
  int var[kMaxFields];
  int deriv[kMaxFields];
  int src_S;   // 0 means the state's S
  int wmode;
};

// Adjoint of the backward z transform: for each target variable, sum over its
// source fields of conj(i k)^deriv * T^T G_f, accumulated into Xbar[P][S][N].
struct AccList {
  int nt;
  int target[9];
  int nsrc[9];
  int src[9][2];
  int deriv[9][2];
};

// pencil kernels: factor arrays hold factor_stride(n) columns per pencil with
// factor_slack() columns of zero slack before the first and after the last
// pencil (the solve's look-ahead loads read into them)
int factor_stride(int n);
int factor_slack();
hipError_t launch_factor(const PencilArgs& a, double a0, double b0, double* Lf, uint8_t* sl,
                         double* Uf, int* sing, hipStream_t st, double* tailL = nullptr,
                         uint8_t* tailP = nullptr);
// Two-block solve (2-D): the whole operator A (band kl, ku) split at m into the
// leading block T and the trailing block B (factored in reversed order), each
// with its own banded LU; with A12 = A[0:m, m:m+ku] and A21 = A[m:n, m-kl:m],
//   E1 = L_T^{-1} P_T A12 (last Q rows),  E2 = L_B^{-1} P_B J A21 (last Q rows),
// and Rinv the inverse of the (kl + ku) x (kl + ku) interface system
//   [U_T(last kl)  E1 J; E2  U_B(last ku)].
// launch_coupling forms E1 [P][Q][ku], E2 [P][Q][kl] and Rinv [P][K][K] from
// the replayed last-Q elimination steps of both factorizations (tailL / tailP
// of launch_factor) and the stored U factors.  t / bt are the block
// descriptions (blk 1 / 2).
hipError_t launch_coupling(const PencilArgs& t, const PencilArgs& bt, double a0, double b0,
                           const double* tailLt, const uint8_t* tailPt, const double* tailLb,
                           const uint8_t* tailPb, const double* Uft, const double* Ufb,
                           double* Rinv, double* E1, double* E2, int* sing, hipStream_t st);
// Whole-system solve from the two blocks: forward sweeps of both blocks in
// parallel, the interface system, the corrections, backward sweeps.
hipError_t launch_solve2(const PencilArgs& t, const PencilArgs& bt, const void* Bev,
                         const double* Lft, const uint8_t* slt, const double* Uft,
                         const double* Lfb, const uint8_t* slb, const double* Ufb,
                         const double* Rinv, const double* E1, const double* E2, void* X,
                         hipStream_t st);
bool solve2_supported(const PencilArgs& t, const PencilArgs& bt);
// Linear-stability eigenvalues nearest tau by shift-invert Krylov-Schur
// iteration, one wavefront per pencil, on the whole-band factors of
// tau M~ + L~ + L~' (k_evp.hip).  V: device workspace of P (ncv + 1) n doubles.
struct EvpOut {
  double2* sigma;  // [P][nev]
  double* resid;   // [P][nev]
  int* nconv;      // [P]
  int* nops;       // [P]
  double2* X;      // [nev][P][S N] or null
};
hipError_t launch_evp(const PencilArgs& a, double tau, int nev, int ncv, int max_ops, double tol,
                      const double* Lf, const uint8_t* sl, const double* Uf, double* V,
                      const EvpOut& o, hipStream_t st);
hipError_t launch_solve(const PencilArgs& a, const void* Bev, const double* Lf, const uint8_t* sl,
                        const double* Uf, void* X, hipStream_t st);
// Sparse factor records (k_pencil.hip): whether the streamed solve runs for
// a (and then the record strides in geom), the packing of a slot's
// whole-band factors after its factorisation, and the solve over them
bool sparse_records_apply(const PencilArgs& a, SparseFactors* geom);
hipError_t launch_sparse_records(const PencilArgs& a, const double* Lf, const uint8_t* sl, const double* Uf,
                                 const SparseFactors& sf, hipStream_t st);
hipError_t launch_solve_sparse(const PencilArgs& a, const void* Bev, const SparseFactors& sf, void* X,
                               hipStream_t st);
// Mixed-precision solve with one FP64 refinement: FP32 sweeps on the FP32
// factor copies, the FP64 residual of (a.refine_a0 M~ + a.refine_b0 L~) from
// the templates, an FP32 correction sweep, the sum in FP64
hipError_t launch_solve_refined(const PencilArgs& a, const void* Bev, const float* Lf, const uint8_t* sl,
                                const float* Uf, void* X, hipStream_t st);
hipError_t launch_round_f32(const double* src, float* dst, size_t count, hipStream_t st);
// The same for the two-block layout: FP32 copies of both blocks' factors, the
// FP64 coupling data; t.refine_a0 / refine_b0 name the operator (2-D)
hipError_t launch_solve2_refined(const PencilArgs& t, const PencilArgs& bt, const void* Bev,
                                 const float* Lft, const uint8_t* slt, const float* Uft,
                                 const float* Lfb, const uint8_t* slb, const float* Ufb,
                                 const double* Rinv, const double* E1, const double* E2, void* X,
                                 hipStream_t st);

// transforms along y and the 3-D x pass
// ys: output scale in place of the default (0: 1 backward, 1 / Ngy forward)
// Output fields of the backward y pass from input fields: output f reads
// input src[f], times i ky where der[f] (n = 0: output f reads input f)
struct YMap {
  int n;
  int src[12];
  int der[12];
};
hipError_t launch_ypass(const XformArgs& a, int dir, int nf, const void* In, void* Out,
                        hipStream_t st, bool fp32 = false, double ys = 0.0, const YMap* map = nullptr);
hipError_t launch_xpass3(const XformArgs& a, const void* G2, void* H2, hipStream_t st,
                         bool fp32 = false);

// transforms (2-D)
// active_only (2-D): transform only the leading Pa pencils; G of the others
// is left unwritten (for consumers that read p < Pa only, as the x pass does)
hipError_t launch_zb(const XformArgs& a, const FieldList& fl, const void* X, void* G,
                     hipStream_t st, bool fp32 = false, bool active_only = false);
hipError_t launch_xpass(const XformArgs& a, const void* G, void* H, hipStream_t st,
                        bool fp32 = false);
// forward z; mode 0 writes F[P][ne][N]; mode 1 assembles the SBDF right-hand
// side and the history (see k_transform.hip); mode 2 the right-hand side of a
// Runge-Kutta stage (rk_rhs below)
constexpr int kMaxRkStages = 4;
struct RkArgs {
  int stage;      // i, 1 <= i <= s
  int last;       // i == s: F~^{n,i-1} and dt L~X^{n,i-1} are not needed later
  double dt;
  double scale;   // 1 / (dt H_ii): the stage system is factored as (M~ / (dt H_ii) + L~)
  double hprev;   // 1 / H_{i-1,i-1} (i >= 2)
  double A[kMaxRkStages], H[kMaxRkStages];  // A_ij, H_ij for j < i
  double2* F[kMaxRkStages];  // F~^{n,j} [P][ne][N], written by stage j + 1
  double2* K[kMaxRkStages];  // dt L~X^{n,j} (j >= 1) [P][ne][N], written by stage j + 1
  double2* MX0;              // M~X^{n,0} [P][ne][N], written by stage 1
  const double2* Bprev;      // the right-hand side of stage i - 1 (the buffer out is written to)
};
struct RhsArgs {
  int mode;
  double c1, c2, a1, a2;
  int has_hist;
  const double2* Xprev;  // state X^{n-1} (mode 2: the stage state X^{n,i-1})
  double2* hist_cur;     // [P][2][ne][N]
  const double2* hist_old;
  RkArgs rk;
};

// Right-hand side of Runge-Kutta stage i at one evolved-equation U-row
// (index o of the [P][ne][N] arrays) of an active pencil (Sec. IX
// "Runge-Kutta IMEX integrators"):
//   B~ = M~X^{n,0} + dt sum_{j<i} A_ij F~^{n,j} - dt sum_{j<i} H_ij L~X^{n,j},
// written to out as B~ / (dt H_ii).  H_i0 = 0 for the schemes built here.
// dt L~X^{n,i-1} is not applied from the operator: stage i - 1 solved
// (M~ / (dt H) + L~) X^{n,i-1} = out, so dt L~X^{n,i-1} = dt out - M~X^{n,i-1} / H
// row by row (H = H_{i-1,i-1}), read from out before it is overwritten.
// rk_load issues the row's loads (so that a caller can batch several rows),
// rk_finish takes Ft = F~^{n,i-1} and MX = M~X^{n,i-1} and stores.
struct RkRow {
  double2 bp, mx0;                  // out (stage i - 1), M~X^{n,0}
  double2 F[kMaxRkStages - 1];      // F~^{n,j}, j < i - 1
  double2 K[kMaxRkStages - 2];      // dt L~X^{n,j}, 1 <= j < i - 1 (slot j - 1)
};

__device__ __forceinline__ void rk_load(const RkArgs& k, size_t o, RkRow& v) {
  const int i = k.stage;
  if (i > 1) {
    v.bp = k.Bprev[o];
    v.mx0 = k.MX0[o];
  }
#pragma unroll
  for (int j = 0; j < kMaxRkStages - 1; ++j)
    if (j < i - 1) v.F[j] = k.F[j][o];
#pragma unroll
  for (int j = 1; j < kMaxRkStages - 1; ++j)
    if (j < i - 1) v.K[j - 1] = k.K[j][o];
}

__device__ __forceinline__ void rk_finish(const RkArgs& k, size_t o, const RkRow& v, double2 Ft,
                                          double2 MX, double2* __restrict__ out) {
  const int i = k.stage;
  double2 B;
  if (i == 1) {
    k.MX0[o] = MX;
    B = MX;
  } else {
    const double2 Kp = make_double2(k.dt * v.bp.x - k.hprev * MX.x, k.dt * v.bp.y - k.hprev * MX.y);
    if (!k.last) k.K[i - 1][o] = Kp;
    B = v.mx0;
    B.x -= k.H[i - 1] * Kp.x;
    B.y -= k.H[i - 1] * Kp.y;
#pragma unroll
    for (int j = 1; j < kMaxRkStages - 1; ++j)
      if (j < i - 1) {
        B.x -= k.H[j] * v.K[j - 1].x;
        B.y -= k.H[j] * v.K[j - 1].y;
      }
  }
#pragma unroll
  for (int j = 0; j < kMaxRkStages - 1; ++j)
    if (j < i - 1) {
      B.x += k.dt * k.A[j] * v.F[j].x;
      B.y += k.dt * k.A[j] * v.F[j].y;
    }
  B.x += k.dt * k.A[i - 1] * Ft.x;
  B.y += k.dt * k.A[i - 1] * Ft.y;
  if (!k.last) k.F[i - 1][o] = Ft;
  out[o] = make_double2(B.x * k.scale, B.y * k.scale);
}

__device__ __forceinline__ void rk_rhs(const RkArgs& k, size_t o, double2 Ft, double2 MX,
                                       double2* __restrict__ out) {
  RkRow v;
  rk_load(k, o, v);
  rk_finish(k, o, v, Ft, MX, out);
}
hipError_t launch_zf(const XformArgs& a, const void* H, void* out, const RhsArgs& r,
                     hipStream_t st, bool fp32 = false);

// z transforms as FP64 matrix-core products (k_dctmm.hip)
bool mm_supported(int N);
hipError_t launch_zb_mm(const XformArgs& a, const FieldList& fl, const void* X, void* G,
                        const double* Bfrag, hipStream_t st);
hipError_t launch_zf_mm(const XformArgs& a, const void* H, void* out, const RhsArgs& r,
                        const double* Ffrag, hipStream_t st);
// mixed path: split-BF16 products with FP32 accumulation; tables split into
// three BF16 terms in fragment order (N = 64, 128 or 256)
bool mm_bf16_supported(int N);
hipError_t launch_zb_bf16(const XformArgs& a, const FieldList& fl, const void* X, void* G,
                          const void* B3, hipStream_t st);
hipError_t launch_zf_bf16(const XformArgs& a, const void* H, void* out, const RhsArgs& r,
                          const void* F3, hipStream_t st);


// adjoint path
// fp32: Gbar (and in the x pass G, Hbar, Gbar) hold complex64, the
// transforms run in FP32; Xbar accumulates in FP64 either way
hipError_t launch_zadj(const XformArgs& a, const AccList& al, const void* Gbar, void* Xbar,
                       hipStream_t st, bool fp32 = false);
hipError_t launch_xpass_adj(const XformArgs& a, const void* G, const void* Hbar, void* Gbar,
                            hipStream_t st, bool fp32 = false);
struct AdjRhsArgs {
  double c1, c2, a1, a2;
  double2* hbar;  // [P][2][ne][N] pending adjoints (read, then overwritten)
  double2* Fbar;  // [P][ne][N] output: (P^L)^H F~bar
};
hipError_t launch_solveT(const PencilArgs& a, const void* Xbar_in, const double* Lf,
                         const uint8_t* sl, const double* Uf, void* Xbar_out,
                         const AdjRhsArgs& r, hipStream_t st);
// The same on the two-block factors of A~^T (t, bt: block descriptions with
// trans set; leading block FW 32, trailing block FW 8): the two-block solve's
// sweeps and interface system with the transposed solve's right-hand side and
// epilogue.
hipError_t launch_solve2T(const PencilArgs& t, const PencilArgs& bt, const void* Xbar_in,
                          const double* Lft, const uint8_t* slt, const double* Uft,
                          const double* Lfb, const uint8_t* slb, const double* Ufb,
                          const double* Rinv, const double* E1, const double* E2, void* Xbar_out,
                          const AdjRhsArgs& r, hipStream_t st);
hipError_t launch_ke_adjoint(const XformArgs& a, const void* X, void* G, void* Gbar,
                             const void* wvec, void* ebar, void* Xbar, hipStream_t st);
hipError_t launch_initial_state_adjoint(const XformArgs& a1, const void* Xbar, double* gbar,
                                        void* work, hipStream_t st);

// initial state from scale-1 grid values of b
// P^L F on the evolved U-rows for the linear boundary value solve
hipError_t launch_lbvp_rhs(const XformArgs& a, const void* F, void* Bev, hipStream_t st);
hipError_t launch_initial_state(const XformArgs& a1, const double* bgrid, void* X, void* work,
                                hipStream_t st);

// grid <-> coefficient transforms (k_grid.hip): the x stage between spectral
// rows s[f][jz][l][kx] and the grid g[f][ix][l][jz] (Lg x points, Ngy y levels,
// Mg z levels; tw the Lg-point FFT table), dir +1 synthesis
//   g = s0 Re c_0 + 2 s1 Re sum_{1 <= k < Pa} c_k e^{2 pi i k ix / Lg},
// dir -1 analysis c_0 = s0 sum g, c_k = s1 sum g e^{-2 pi i k ix / Lg} (k < Pa,
// zero up to Px); the variable gather / scatter of the state layout
bool xgrid_supported(int Lg, int Mg);
hipError_t launch_xgrid(const XformArgs& a, int dir, int nf, int Lg, int Ngy, int Mg,
                        const double2* tw, const void* in, void* out, double s0, double s1,
                        hipStream_t st);
hipError_t launch_put_vars(int P, int S, int N, const FieldList& fl, const void* F, void* X,
                           hipStream_t st);
hipError_t launch_zero_vars(int P, int S, int N, const FieldList& fl, void* X, hipStream_t st);

// kinetic energy: mean over x of |u|^2/2 per z row, then Chebyshev integral
hipError_t launch_ke(const XformArgs& a, const void* X, void* G, void* G2, double* rowmean, double* out,
                     hipStream_t st);

}  // namespace stau
