// Shared device helpers: complex arithmetic, the in-LDS mixed-radix FFT and
// the pencil-system description.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stau {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T x, T y) {
  cpx<T> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {  // a * conj(b)
  return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cpx<T> conj(cpx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by i (DIR=+1) or -i (DIR=-1)
template <int DIR, typename T>
__device__ __forceinline__ cpx<T> mul_pi(cpx<T> a) {
  return DIR > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Small DFTs.  DIR = -1: forward kernel e^{-2 pi i n k / R}; DIR = +1: inverse.
// ---------------------------------------------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft3(cpx<T>* v) {
  // w = e^{DIR 2 pi i / 3} = -1/2 + DIR i sqrt(3)/2
  const T c = T(-0.5);
  const T s = T(DIR) * T(0.86602540378443864676372317075294);
  cpx<T> sum = v[1] + v[2], dif = v[1] - v[2];
  cpx<T> m = mk(v[0].x + c * sum.x, v[0].y + c * sum.y);
  cpx<T> is = mk(-s * dif.y, s * dif.x);  // i s (v1 - v2)
  v[0] = v[0] + sum;
  v[1] = m + is;
  v[2] = m - is;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cpx<T>* v) {
  cpx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cpx<T> t2 = v[1] + v[3], t3 = v[1] - v[3];
  cpx<T> r3 = mul_pi<DIR>(t3);  // DIR i t3
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + r3;
  v[3] = t1 - r3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cpx<T>* v) {
  cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  const T h = T(0.70710678118654752440084436210485);
  // w^k = e^{DIR 2 pi i k / 8}
  cpx<T> w1o = cmul(o[1], mk(h, T(DIR) * h));
  cpx<T> w2o = mul_pi<DIR>(o[2]);
  cpx<T> w3o = cmul(o[3], mk(-h, T(DIR) * h));
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + w1o;
  v[5] = e[1] - w1o;
  v[2] = e[2] + w2o;
  v[6] = e[2] - w2o;
  v[3] = e[3] + w3o;
  v[7] = e[3] - w3o;
}

// 6 = 2 x 3: pairs (v[n], v[n + 3]) first (w^3 = -1), then a length-3 DFT of
// the sums for the even outputs and of the differences times w^n for the odd
// ones (w = e^{DIR 2 pi i / 6}, w^2 the length-3 root)
template <int DIR, typename T>
__device__ __forceinline__ void dft6(cpx<T>* v) {
  const T h = T(0.5);
  const T s = T(DIR) * T(0.86602540378443864676372317075294);
  cpx<T> a[3], b[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    a[n] = v[n] + v[n + 3];
    b[n] = v[n] - v[n + 3];
  }
  b[1] = cmul(b[1], mk(h, s));   // w
  b[2] = cmul(b[2], mk(-h, s));  // w^2
  dft3<DIR>(a);
  dft3<DIR>(b);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[2 * k] = a[k];
    v[2 * k + 1] = b[k];
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR(cpx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  if constexpr (R == 3) dft3<DIR>(v);
  if constexpr (R == 4) dft4<DIR>(v);
  if constexpr (R == 6) dft6<DIR>(v);
  if constexpr (R == 8) dft8<DIR>(v);
}

// ---------------------------------------------------------------------------
// In-place Stockham autosort FFT of `batch` contiguous sequences of length M
// held in LDS.  Radix plan: one radix-3 pass if 3 | M, then over the power
// of two either radix-8 passes and one radix-4 or radix-2 pass for what is
// left (R8) or radix-4 passes with one radix-8 pass if the exponent is odd
// (M = 2^a 3^b, b <= 1).  tw[t] = e^{-2 pi i t / M}, t < M; each butterfly
// reads one entry and forms the other powers it needs by complex products.
// Each pass stages its butterflies in registers between two barriers, so the
// transform is in place.  MAXBF bounds the butterflies per thread per pass;
// the caller guarantees batch*M/4 <= MAXBF*nthreads.
// ---------------------------------------------------------------------------
template <int R, int DIR, int MAXBF, typename T>
__device__ __forceinline__ void stockham_pass(cpx<T>* buf, int M, int batch, int Ns,
                                              const cpx<T>* __restrict__ tw, int tid, int nt) {
  const int MR = M / R;
  const int nbf = batch * MR;
  const int tstride = M / (Ns * R);
  cpx<T> v[MAXBF][R];
#pragma unroll
  for (int b = 0; b < MAXBF; ++b) {
    const int bf = tid + b * nt;
    if (bf < nbf) {
      const int s = bf / MR, j = bf - s * MR;
      const cpx<T>* src = buf + s * M + j;
      const int jm = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[r * MR];
      // twiddles w^r, r < R, from one table entry (at most three products deep)
      cpx<T> w[R];
      w[1] = tw[jm * tstride];
      if constexpr (R >= 3) w[2] = cmul(w[1], w[1]);
      if constexpr (R >= 4) w[3] = cmul(w[1], w[2]);
      if constexpr (R == 8) {
        w[4] = cmul(w[2], w[2]);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[b][r] = DIR < 0 ? cmul(v[b][r], w[r]) : cmulc(v[b][r], w[r]);
      dftR<R, DIR>(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXBF; ++b) {
    const int bf = tid + b * nt;
    if (bf < nbf) {
      const int s = bf / MR, j = bf - s * MR;
      const int jm = j % Ns;
      cpx<T>* dst = buf + s * M + (j / Ns) * Ns * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

template <int DIR, int MAXBF, typename T, bool R8 = true>
__device__ __forceinline__ void fft_lds(cpx<T>* buf, int M, int batch, const cpx<T>* __restrict__ tw, int tid,
                        int nt) {
  int Ns = 1;
  int m2 = M;
  if (m2 % 3 == 0) {
    stockham_pass<3, DIR, (MAXBF * 4 + 2) / 3>(buf, M, batch, Ns, tw, tid, nt);
    Ns *= 3;
    m2 /= 3;
  }
  int lg = 31 - __clz(m2);
  if constexpr (R8) {
    // power of two: radix-8 passes, then one radix-4 or radix-2 pass for the
    // rest (fewest passes; for latency-bound launches with few blocks)
    for (; lg >= 3; lg -= 3) {
      stockham_pass<8, DIR, (MAXBF + 1) / 2>(buf, M, batch, Ns, tw, tid, nt);
      Ns *= 8;
    }
    if (lg == 2) stockham_pass<4, DIR, MAXBF>(buf, M, batch, Ns, tw, tid, nt);
    if (lg == 1) stockham_pass<2, DIR, MAXBF * 2>(buf, M, batch, Ns, tw, tid, nt);
  } else {
    // radix-4 passes (one radix-8 pass if the exponent is odd): more threads
    // busy per pass, for launches with many blocks per CU
    if (lg & 1) {
      if (lg >= 3) {
        stockham_pass<8, DIR, (MAXBF + 1) / 2>(buf, M, batch, Ns, tw, tid, nt);
        Ns *= 8;
        lg -= 3;
      } else {
        stockham_pass<2, DIR, MAXBF * 2>(buf, M, batch, Ns, tw, tid, nt);
        Ns *= 2;
        lg -= 1;
      }
    }
    for (; lg > 0; lg -= 2) {
      stockham_pass<4, DIR, MAXBF>(buf, M, batch, Ns, tw, tid, nt);
      Ns *= 4;
    }
  }
}

// ---------------------------------------------------------------------------
// The same transform for a length M known at compile time: the radix plan is
// resolved by the templates and every pass's butterfly indices divide by
// constants (shifts and multiply-highs instead of the integer division
// sequences the runtime version issues per butterfly).  MC = 0 selects the
// runtime version.
// ---------------------------------------------------------------------------
template <int R, int DIR, int MAXBF, int M, int NS, typename T>
__device__ __forceinline__ void stockham_pass_c(cpx<T>* buf, int batch, const cpx<T>* __restrict__ tw,
                                                int tid, int nt) {
  constexpr int MR = M / R, TSTR = M / (NS * R);
  const int nbf = batch * MR;
  cpx<T> v[MAXBF][R];
#pragma unroll
  for (int b = 0; b < MAXBF; ++b) {
    const int bf = tid + b * nt;
    if (bf < nbf) {
      const int s = bf / MR, j = bf - s * MR;
      const cpx<T>* src = buf + s * M + j;
      const int jm = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[r * MR];
      cpx<T> w[R];
      w[1] = tw[jm * TSTR];
      if constexpr (R >= 3) w[2] = cmul(w[1], w[1]);
      if constexpr (R >= 4) w[3] = cmul(w[1], w[2]);
      if constexpr (R >= 6) {
        w[4] = cmul(w[2], w[2]);
        w[5] = cmul(w[1], w[4]);
      }
      if constexpr (R == 8) {
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
      }
#pragma unroll
      for (int r = 1; r < R; ++r) v[b][r] = DIR < 0 ? cmul(v[b][r], w[r]) : cmulc(v[b][r], w[r]);
      dftR<R, DIR>(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXBF; ++b) {
    const int bf = tid + b * nt;
    if (bf < nbf) {
      const int s = bf / MR, j = bf - s * MR;
      const int jm = j % NS;
      cpx<T>* dst = buf + s * M + (j / NS) * NS * R + jm;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * NS] = v[b][r];
    }
  }
  __syncthreads();
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// passes for the part M / NS not yet transformed, in the order of fft_lds;
// with R6 the factor 3 is taken with a factor 2 in one radix-6 pass (384 =
// 6 x 8 x 8: three passes instead of four)
template <int M, int NS, int DIR, int MAXBF, typename T, bool R8, bool R6>
__device__ __forceinline__ void fft_passes_c(cpx<T>* buf, int batch, const cpx<T>* __restrict__ tw, int tid,
                                             int nt) {
  constexpr int rem = M / NS;
  if constexpr (rem > 1) {
    constexpr int lg = ilog2c(rem);
    constexpr int R = rem % 3 == 0 ? (R6 && rem % 6 == 0 ? 6 : 3)
                      : R8         ? (lg >= 3 ? 8 : (lg == 2 ? 4 : 2))
                      : (lg & 1)   ? (lg >= 3 ? 8 : 2)
                                   : 4;
    constexpr int BF = R == 3   ? (MAXBF * 4 + 2) / 3
                       : R == 6 ? (MAXBF * 4 + 5) / 6
                       : R == 8 ? (MAXBF + 1) / 2
                       : R == 4 ? MAXBF
                                : MAXBF * 2;
    stockham_pass_c<R, DIR, BF, M, NS, T>(buf, batch, tw, tid, nt);
    fft_passes_c<M, NS * R, DIR, MAXBF, T, R8, R6>(buf, batch, tw, tid, nt);
  }
}

template <int MC, int DIR, int MAXBF, typename T, bool R8 = true, bool R6 = false>
__device__ __forceinline__ void fft_lds_c(cpx<T>* buf, int M, int batch, const cpx<T>* __restrict__ tw, int tid,
                                          int nt) {
  if constexpr (MC > 0) {
    static_assert(MC % 9 != 0, "at most one factor 3");
    fft_passes_c<MC, 1, DIR, MAXBF, T, R8, R6>(buf, batch, tw, tid, nt);
  } else {
    fft_lds<DIR, MAXBF, T, R8>(buf, M, batch, tw, tid, nt);
  }
}

// ---------------------------------------------------------------------------
// Pencil system layout (2-D: S = 7, 3-D: S = 9).
//  variables per mode (column order):  2-D (w, b, u, p, bz, uz, wz)
//                                      3-D (w, b, u, v, p, bz, uz, vz, wz)
//  equations per mode (row order):     2-D (w, b, u, c, uz, bz, wz)
//                                      3-D (w, b, u, v, c, uz, vz, bz, wz)
//  boundary rows first: q(z=0) for q in evolved, then q(z=1) (gauge p(z=1)
//  in place of w(z=1) at the mean pencil).
// State arrays use the variable order of the C ABI: 2-D (p,b,u,w,bz,uz,wz),
// 3-D (p,b,u,v,w,bz,uz,vz,wz).
// ---------------------------------------------------------------------------
enum Var { VW = 0, VB, VU, VV, VP, VBZ, VUZ, VVZ, VWZ };
enum Eq { EW = 0, EB, EU, EV, EC, EUZ, EVZ, EBZ, EWZ };

struct SysDesc {
  int dim, S, ne, N, kb;
  int var_at[9];      // column position in mode -> Var
  int eq_at[9];       // row position in mode -> Eq
  int var_pos[9];     // Var -> column position in mode (-1 if absent)
  int eq_pos[9];      // Eq -> row position in mode
  int abi_index[9];   // Var -> variable index in the C-ABI state layout
  int bc_var[8];      // boundary row -> Var  (rows 0..kb-1)
  int bc_side[8];     // 0: z = 0, 1: z = 1
  int evolved[4];     // evolved Var in ABI evolved order (b, u, [v], w)
};

constexpr int kMaxNcc = 4;  // Chebyshev terms of the non-constant coefficient

struct PencilCoef {
  double a0, b0, kappa, nu, buoy, kx, ky;
  int mean;
  // linearisation of the explicit term -w d_z b about the conduction profile
  // b0(z) = b_bottom + (b_top - b_bottom) z: lin = b_top - b_bottom times
  // P^L w on the b rows (linear-stability problems only; 0 for the step)
  double lin;
  // non-constant coefficient Gamma(z) = sum_{k < nncc} ncc[k] T_k multiplying
  // w in the b equation (P^L G w on the b rows, G the truncated product matrix)
  int nncc;
  double ncc[kMaxNcc];
};

// G(i, j) of the product matrix of Gamma: <T_i | Gamma T_j> from
// T_k T_j = (T_{k+j} + T_{|k-j|}) / 2 (Sec. II, non-constant coefficients)
__host__ __device__ __forceinline__ double ncc_G(const PencilCoef& pc, int i, int j) {
  double v = 0.0;
  // fixed trip count: the coefficients stay in registers (no scratch array)
#pragma unroll
  for (int k = 0; k < kMaxNcc; ++k) {
    if (k >= pc.nncc) break;
    double t = 0.0;
    if (i == j + k) t += 1.0;
    if (i == (j >= k ? j - k : k - j)) t += 1.0;
    v += 0.5 * pc.ncc[k] * t;
  }
  return v;
}

// Entry (r, c) of a0 M~ + b0 L~ in the interleaved, Dirichlet-recombined,
// real-scaled system of one pencil.  Rows: kb boundary rows, then modes
// n = 0..N-1 with S equation rows each (only continuity at n = N-1).
// Columns: mode-major, S variables per mode.
__host__ __device__ inline int sys_row_mode(const SysDesc& d, int r, int* epos) {
  if (r < d.kb) {
    *epos = -1;
    return -1;
  }
  int q = r - d.kb;
  int n = q / d.S;
  *epos = q - n * d.S;
  if (n == d.N - 1) *epos = d.eq_pos[EC];  // last mode: the continuity row only
  return n;
}

__host__ __device__ inline double cheb_C(int n, int m) {  // P^L (n, m)
  if (m == n) return n == 0 ? 1.0 : 0.5;
  if (m == n + 2) return -0.5;
  return 0.0;
}
__host__ __device__ inline double cheb_D(int n, int m) {  // d/dz (z in [0,1]) T->U
  return m == n + 1 ? 2.0 * m : 0.0;
}

// T-basis entry (row (n, eq), column (m, var)); real-scaled.
__host__ __device__ __forceinline__ double entry_T(const SysDesc& d, const PencilCoef& pc, int n, int eq,
                                          int m, int var) {
  const double k2 = pc.kx * pc.kx + pc.ky * pc.ky;
  switch (eq) {
    case EB:
      if (var == VB) return (pc.a0 + pc.b0 * pc.kappa * k2) * cheb_C(n, m);
      if (var == VBZ) return -pc.b0 * pc.kappa * cheb_D(n, m);
      if (var == VW) {
        // (P^L (lin + G))(n, m) with P^L = C: rows n and n + 2 of G (truncated at N)
        double v = pc.lin * cheb_C(n, m);
        if (pc.nncc) {
          v += (n == 0 ? 1.0 : 0.5) * ncc_G(pc, n, m);
          if (n + 2 < d.N) v -= 0.5 * ncc_G(pc, n + 2, m);
        }
        return pc.b0 * v;
      }
      return 0.0;
    case EU:
      if (var == VU) return (pc.a0 + pc.b0 * pc.nu * k2) * cheb_C(n, m);
      if (var == VUZ) return -pc.b0 * pc.nu * cheb_D(n, m);
      if (var == VP) return -pc.b0 * pc.kx * cheb_C(n, m);
      return 0.0;
    case EV:
      if (var == VV) return (pc.a0 + pc.b0 * pc.nu * k2) * cheb_C(n, m);
      if (var == VVZ) return -pc.b0 * pc.nu * cheb_D(n, m);
      if (var == VP) return -pc.b0 * pc.ky * cheb_C(n, m);
      return 0.0;
    case EW:
      if (var == VW) return (pc.a0 + pc.b0 * pc.nu * k2) * cheb_C(n, m);
      if (var == VWZ) return -pc.b0 * pc.nu * cheb_D(n, m);
      if (var == VP) return pc.b0 * cheb_D(n, m);
      if (var == VB) return -pc.b0 * pc.buoy * cheb_C(n, m);
      return 0.0;
    case EBZ:
      if (var == VBZ) return pc.b0 * cheb_C(n, m);
      if (var == VB) return -pc.b0 * cheb_D(n, m);
      return 0.0;
    case EUZ:
      if (var == VUZ) return pc.b0 * cheb_C(n, m);
      if (var == VU) return -pc.b0 * cheb_D(n, m);
      return 0.0;
    case EVZ:
      if (var == VVZ) return pc.b0 * cheb_C(n, m);
      if (var == VV) return -pc.b0 * cheb_D(n, m);
      return 0.0;
    case EWZ:
      if (var == VWZ) return pc.b0 * cheb_C(n, m);
      if (var == VW) return -pc.b0 * cheb_D(n, m);
      return 0.0;
    case EC:
      if (m != n) return 0.0;
      if (var == VU) return pc.b0 * pc.kx;
      if (var == VV) return pc.b0 * pc.ky;
      if (var == VWZ) return pc.b0;
      return 0.0;
  }
  return 0.0;
}

__host__ __device__ __forceinline__ double sys_entry(const SysDesc& d, const PencilCoef& pc, int r, int c) {
  const int m = c / d.S;
  const int var = d.var_at[c - m * d.S];
  if (r < d.kb) {
    // boundary row: T_m(-1) = (-1)^m, T_m(1) = 1, recombined D_0, D_1 only
    int bv = d.bc_var[r];
    if (pc.mean && bv == VW && d.bc_side[r] == 1) bv = VP;  // gauge p(z=1) = 0
    if (var != bv || m > 1) return 0.0;
    const double val = (d.bc_side[r] == 0 && m == 1) ? -1.0 : 1.0;
    return pc.b0 * val;
  }
  int epos;
  const int n = sys_row_mode(d, r, &epos);
  const int eq = d.eq_at[epos];
  double v = entry_T(d, pc, n, eq, m, var);
  if (m >= 2) v -= entry_T(d, pc, n, eq, m - 2, var);  // right-multiply by P^R
  return v;
}

// ---------------------------------------------------------------------------
// Row r of (a0 M~ + b0 L~) x~ for the real-scaled recombined system, from the
// operator templates (no stored matrix): x_T = P^R x~ per variable, then the
// T-to-U conversion C and derivative D of each equation (the same entries as
// entry_T).  getx(m, var) returns x~ at column (m, var).
// ---------------------------------------------------------------------------
template <typename GX>
__host__ __device__ inline double apply_row(const SysDesc& d, const PencilCoef& pc, int r, GX getx) {
  const int N = d.N;
  auto xT = [&](int var, int m) -> double {
    if (m >= N || d.var_pos[var] < 0) return 0.0;
    double v = getx(m, var);
    if (m + 2 < N) v -= getx(m + 2, var);
    return v;
  };
  auto Cv = [&](int var, int q) {
    double v = xT(var, q) * (q == 0 ? 1.0 : 0.5);
    if (q + 2 < N) v -= 0.5 * xT(var, q + 2);
    return v;
  };
  auto Dv = [&](int var, int q) { return q + 1 < N ? 2.0 * (q + 1) * xT(var, q + 1) : 0.0; };
  if (r < d.kb) {
    int q = d.bc_var[r];
    if (pc.mean && q == VW && d.bc_side[r] == 1) q = VP;
    return pc.b0 * (getx(0, q) + (d.bc_side[r] == 0 ? -1.0 : 1.0) * getx(1, q));  // T_m(-1), T_m(1)
  }
  int epos;
  const int n = sys_row_mode(d, r, &epos);
  const int eq = d.eq_at[epos];
  const double k2 = pc.kx * pc.kx + pc.ky * pc.ky;
  const double ak = pc.a0 + pc.b0 * pc.kappa * k2, an = pc.a0 + pc.b0 * pc.nu * k2;
  switch (eq) {
    case EB: {
      double v = ak * Cv(VB, n) - pc.b0 * pc.kappa * Dv(VBZ, n);
      if (pc.lin != 0.0) v += pc.b0 * pc.lin * Cv(VW, n);  // uniform branch: no reads when absent
      if (pc.nncc) {
        // C (G w_T): (G y)_i = sum_j G(i, j) y_j, the j with i = j + k or
        // i = |j - k|: (G y)_i = sum_k g_k ([i >= k] y_{i-k} + y_{i+k}
        // + [0 < i <= k] y_{k-i}) / 2 over stored modes
        auto Gw = [&](int i) {
          double a = 0.0;
#pragma unroll
          for (int k = 0; k < kMaxNcc; ++k) {
            if (k >= pc.nncc) break;
            double t = xT(VW, i + k);
            if (i >= k) t += xT(VW, i - k);
            if (i > 0 && k >= i) t += xT(VW, k - i);
            a += 0.5 * pc.ncc[k] * t;
          }
          return a;
        };
        double g = (n == 0 ? 1.0 : 0.5) * Gw(n);
        if (n + 2 < N) g -= 0.5 * Gw(n + 2);
        v += pc.b0 * g;
      }
      return v;
    }
    case EU: return an * Cv(VU, n) - pc.b0 * pc.nu * Dv(VUZ, n) - pc.b0 * pc.kx * Cv(VP, n);
    case EV: return an * Cv(VV, n) - pc.b0 * pc.nu * Dv(VVZ, n) - pc.b0 * pc.ky * Cv(VP, n);
    case EW:
      return an * Cv(VW, n) - pc.b0 * pc.nu * Dv(VWZ, n) + pc.b0 * Dv(VP, n) -
             pc.b0 * pc.buoy * Cv(VB, n);
    case EBZ: return pc.b0 * (Cv(VBZ, n) - Dv(VB, n));
    case EUZ: return pc.b0 * (Cv(VUZ, n) - Dv(VU, n));
    case EVZ: return pc.b0 * (Cv(VVZ, n) - Dv(VV, n));
    case EWZ: return pc.b0 * (Cv(VWZ, n) - Dv(VW, n));
    case EC: return pc.b0 * (pc.kx * xT(VU, n) + pc.ky * xT(VV, n) + xT(VWZ, n));
  }
  return 0.0;
}


}  // namespace stau
