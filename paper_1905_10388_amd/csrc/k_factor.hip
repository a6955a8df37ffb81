// Pencil kernels: device-side assembly of a0 M~ + b0 L~ from the operator
// templates, banded LU with partial pivoting (one wavefront per pencil), and
// the batched banded solve (one wavefront per pencil, register windows).
//
// Factor storage per pencil p and column j (n = S*N columns, nst >= n stored
// per pencil, columns n..nst-1 zero):
//   Lf[p][j][FW]  multipliers of column j routed to the physical slot that
//                 holds each pending row in the solve's forward window
//                 (FW = kl + 1 slots; zero for the pivot's slot);
//   sl[p][j]      physical slot holding the pivot row of column j;
//   Uf[p][j][BW]  column j of U rotated into the backward window: lane l
//                 holds U(r, j) for the row r = j - ((j - l) mod BW) it
//                 carries, 1 / U(j, j) on lane j mod BW, zero elsewhere.
// The interchanges are LAPACK's (row j <-> pivot row, applied column by
// column), so the forward sweep follows the same order as the factorisation.
#include <algorithm>

#include "pencil.h"

namespace stau {

// ---------------------------------------------------------------------------
// Factor: banded LU with partial pivoting, one wavefront per pencil, the
// active part of the band in registers.  Before step j, lane l holds one
// column c of the window j..j+63 (c = l mod 64) and rows j..j+kl of it in
// av[0..kl] (av[i] zero for i > kl).  Step j: the pivot row (first largest
// |a_ij|) is found in the lane of column j, rows j and j+d are interchanged in
// every lane (a wave-uniform register swap), the multipliers of column j are
// formed there and read by every lane, and each lane holding a column of
// j+1..j+kv applies the rank-1 update to its rows.  Then the rows move up by
// one and each lane appends row j+kl+1 of its column from the operator
// templates; the lane of column j moves on to column j+64, whose rows
// j+1..j+kl lie outside the band (kl + ku <= 63).  Entries come from band
// templates of the operator (host-built, one row per step and lane: six
// loads issued a step ahead and one combination with the pencil's a0, b0,
// k^2, kx, ky and lin).  Row j of U goes to an LDS
// staging ring (kv + 1 entries for each of the kv + 1 columns j..j+kv that
// receive U rows, entry k = c - r) and column j's
// BW-lane solve record is written when it completes (step j).  The
// multipliers go straight to their forward-window slots.  With a.trans the
// transposed matrix is factored (kl and ku of `a` are then those of the
// transpose), for the adjoint's transposed solves.
// ---------------------------------------------------------------------------
// With tailL (two-block solve), the last Q columns' pivot offsets (tailP) and
// multipliers (tailL, kl per column) are also written in elimination order.
// NR register rows per lane (NR >= kl + 1; the loops over rows run to NR,
// the forward window of the stored multipliers has FW slots).
template <int FW, int NR = FW>
__global__ void __launch_bounds__(kWave) factor_kernel(PencilArgs a, double a0, double b0,
                                                       double* __restrict__ Lf,
                                                       uint8_t* __restrict__ sl,
                                                       double* __restrict__ Uf,
                                                       int* __restrict__ sing,
                                                       double* __restrict__ tailL,
                                                       uint8_t* __restrict__ tailP) {
  extern __shared__ double ustage[];  // [kv + 1][kv + 2]: U(r, c) at (c mod (kv + 1), c - r)
  const int p = blockIdx.x;
  if (!pencil_active(a, p)) return;
  const int lane = threadIdx.x;
  const int n = a.n, kl = a.kl, ku = a.ku, kv = kl + ku, BW = a.BW, us = kv + 2;
  const PencilCoef pc = pencil_coef(a, p, a0, b0);
  double* Lp = Lf + (size_t)p * a.nst * FW;
  double* Up = Uf + (size_t)p * a.nst * BW;
  uint8_t* sp = sl + (size_t)p * a.nst;
  // entry (r, c) of the block's operator from the band templates of the whole
  // operator (row R, column C of A~; of A~^T with a.trans)
  const double k2 = pc.kx * pc.kx + pc.ky * pc.ky;
  const size_t ps = (size_t)a.tplane;
  const double* tp1 = a.tpl + (pc.mean ? 2 : 1) * ps;
  auto tpl_at = [&](int r, int c, double* t) -> bool {
    if (r >= n || c >= n || c - r > ku || r - c > kl) return false;
    int R = r, C = c;
    if (a.blk == 2) {
      R = a.nfull - 1 - r;
      C = a.nfull - 1 - c;
    }
    if (a.trans) {
      const int q = R;
      R = C;
      C = q;
    }
    const size_t o = (size_t)R * a.tw + (C - R + a.tkl);
    t[0] = a.tpl[o];
    t[1] = tp1[o];
    t[2] = a.tpl[3 * ps + o];
    t[3] = a.tpl[4 * ps + o];
    t[4] = a.tpl[5 * ps + o];
    t[5] = a.tpl[6 * ps + o];
    return true;
  };
  auto combine = [&](bool in, const double* t) -> double {
    if (!in) return 0.0;
    return a0 * t[0] + b0 * (t[1] + k2 * t[2] + pc.kx * t[3] + pc.ky * t[4] + pc.lin * t[5]);
  };
  auto entry = [&](int r, int c) -> double {
    double t[6];
    const bool in = tpl_at(r, c, t);
    return combine(in, t);
  };
  int c = lane;  // this lane's column
  // staging ring of the kv + 1 columns j..j+kv that receive U rows: slot
  // c mod RS of this lane's column, slot j mod RS of column j
  const int RS = kv + 1, adv = kWave % RS;
  int cs = lane % RS, js = 0;
  static_assert(NR <= FW, "register rows within the forward window");
  double av[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) av[i] = i <= kl ? entry(i, c) : 0.0;
  int ph = lane;  // lane s < FW: the physical slot of forward-window position s
  for (int j = 0; j < n; ++j) {
    const int pl = j & (kWave - 1);
    const int hi = min(n - 1, j + kl) - j;  // rows j..j+hi exist
    // template entries of row j+1+kl for the end of this step (the lane of
    // column j then holds column j+64), loaded now so that they arrive while
    // the step runs
    double tn[6];
    const bool tin = tpl_at(j + 1 + kl, lane == pl ? c + kWave : c, tn);
    // pivot search (used from lane pl): first index of the largest |a|
    double mag = fabs(av[0]);
    int idx = 0;
#pragma unroll
    for (int i = 1; i < NR; ++i) {
      const double m = fabs(av[i]);
      if (i <= hi && m > mag) {
        mag = m;
        idx = i;
      }
    }
    const int d = __builtin_amdgcn_readlane(idx, pl);
    STAU_BOUND(a.check, d >= 0 && d <= hi && hi < NR, kChkPivot);
    // interchange rows j and j + d in every column
    if (d != 0) {
#pragma unroll
      for (int i = 1; i < NR; ++i)
        if (i == d) {
          const double t = av[0];
          av[0] = av[i];
          av[i] = t;
        }
    }
    double piv = readlane_d(av[0], pl);
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) {
      if (lane == 0) atomicMin(sing, p);
      piv = 1.0;
    }
    const double rinv = 1.0 / piv;
    // multipliers of column j, read by every lane (zero beyond row j + hi)
    double lm[NR];
    lm[0] = 0.0;
#pragma unroll
    for (int i = 1; i < NR; ++i) lm[i] = i <= hi ? readlane_d(av[i], pl) * rinv : 0.0;
    // rank-1 update of columns j+1..j+kv
    if (lane != pl && c <= j + kv) {
#pragma unroll
      for (int i = 1; i < NR; ++i) av[i] -= lm[i] * av[0];
    }
    // row j of U (columns j..j+kv; the pivot as its reciprocal), then the solve
    // record of column j: lane l carries row r = j - ((j - l) mod BW)
    if (c <= j + kv) ustage[cs * us + (c - j)] = c == j ? rinv : av[0];
    __builtin_amdgcn_wave_barrier();
    if (lane < BW) {
      int k = (j - lane) % BW;  // (BW need not be a power of two)
      if (k < 0) k += BW;
      double v = 0.0;
      if (k <= kv && k <= j) v = ustage[js * us + k];
      Up[(size_t)j * BW + lane] = v;
    }
    js = js + 1 == RS ? 0 : js + 1;
    // multipliers routed to the physical slots of the forward window: swap
    // the slots of positions 0 and d, the pivot's slot gets 0, then the
    // window advances (the pivot's slot is refilled by the incoming row)
    const int spv = __shfl(ph, d);
    const int t0 = __shfl(ph, 0);
    if (d != 0) {
      if (lane == 0) ph = spv;
      if (lane == d) ph = t0;
    }
    if (lane == 0) sp[j] = (uint8_t)spv;
    if (lane < FW) {
      double lv = 0.0;
#pragma unroll
      for (int i = 1; i < NR; ++i)
        if (lane == i) lv = lm[i];
      Lp[(size_t)j * FW + ph] = lv;
    }
    if (tailL && j >= n - a.Q) {
      const int q = j - (n - a.Q);
      if (lane < kl) {
        double tv = 0.0;
#pragma unroll
        for (int i = 1; i < NR; ++i)
          if (lane + 1 == i) tv = lm[i];
        tailL[((size_t)p * a.Q + q) * kl + lane] = tv;
      }
      if (lane == 0) tailP[(size_t)p * a.Q + q] = (uint8_t)d;
    }
    {
      int nxt = __shfl_down(ph, 1);
      if (lane == FW - 1) nxt = spv;
      if (lane < FW) ph = nxt;
    }
    // rows j+1..j+1+kl for the next step
    const bool fresh = lane == pl;
    if (fresh) {
      c += kWave;
      cs += adv;
      if (cs >= RS) cs -= RS;
    }
    const double nv = combine(tin, tn);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      double v = (i + 1 < NR && !fresh) ? av[i + 1] : 0.0;
      if (i >= kl) v = i == kl ? nv : 0.0;
      av[i] = v;
    }
  }
}


// ---------------------------------------------------------------------------
// Two-block solve (layout in kernels.h, launch_coupling / launch_solve2).
// ---------------------------------------------------------------------------
// U(r, c), r <= c, from the rotated column storage (1 / U(c, c) on lane c mod BW)
__device__ __forceinline__ double u_entry(const double* __restrict__ Up, int BW, int r, int c) {
  if (r > c || c - r >= BW) return 0.0;
  if (r == c) return 1.0 / Up[(size_t)c * BW + (c % BW)];
  return Up[(size_t)c * BW + (r % BW)];
}

__global__ void __launch_bounds__(kWave) coupling_kernel(
    PencilArgs t, PencilArgs bt, double a0, double b0, const double* __restrict__ tailLt,
    const uint8_t* __restrict__ tailPt, const double* __restrict__ tailLb,
    const uint8_t* __restrict__ tailPb, const double* __restrict__ Uft, const double* __restrict__ Ufb,
    double* __restrict__ Rinv, double* __restrict__ E1o, double* __restrict__ E2o,
    int* __restrict__ sing) {
  extern __shared__ double lds[];
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  if (!pencil_active(t, p)) return;
  const PencilCoef pc = pencil_coef(t, p, a0, b0);
  const int kl = t.kl, ku = t.ku, Q = t.Q, K = kl + ku, m = t.n, n = t.nfull, nb = n - m;
  double* E1 = lds;          // [Q][ku]
  double* E2 = E1 + Q * ku;  // [Q][kl]
  double* R = E2 + Q * kl;   // [K][2K]: [R | I] for Gauss-Jordan
  __shared__ int piv_s;
  __shared__ double mult[64];
  auto opA = [&](int r, int c) -> double {  // entry of the factored operator, whole-system indices
    if (r < 0 || c < 0 || r >= n || c >= n || c - r > ku || r - c > kl) return 0.0;
    return t.trans ? sys_entry(t.desc, pc, c, r) : sys_entry(t.desc, pc, r, c);
  };
  for (int idx = lane; idx < Q * ku; idx += kWave) {
    const int i = idx / ku, k = idx - i * ku;
    E1[idx] = opA(m - Q + i, m + k);
  }
  for (int idx = lane; idx < Q * kl; idx += kWave) {
    const int i = idx / kl, k = idx - i * kl;
    E2[idx] = opA(n - 1 - (nb - Q + i), m - kl + k);
  }
  __syncthreads();
  // replay the last Q elimination steps of a block on its coupling columns
  // (one column per lane)
  auto eliminate = [&](double* E, int ncol, const double* tl, const uint8_t* tp, int klb) {
    for (int q = 0; q < Q; ++q) {
      const int off = tp[(size_t)p * Q + q];
      if (lane < ncol) {
        if (off) {
          const double x = E[q * ncol + lane];
          E[q * ncol + lane] = E[(q + off) * ncol + lane];
          E[(q + off) * ncol + lane] = x;
        }
        const double piv = E[q * ncol + lane];
        for (int i = 1; i <= klb && q + i < Q; ++i)
          E[(q + i) * ncol + lane] -= tl[((size_t)p * Q + q) * klb + i - 1] * piv;
      }
    }
  };
  eliminate(E1, ku, tailLt, tailPt, t.kl);
  eliminate(E2, kl, tailLb, tailPb, bt.kl);
  __syncthreads();
  // interface system [R | I]; unknowns [x1b (kl); yb (ku)], x2t[k] = yb[ku - 1 - k]
  const double* Ut = Uft + (size_t)p * t.nst * t.BW;
  const double* Ub = Ufb + (size_t)p * bt.nst * bt.BW;
  for (int idx = lane; idx < K * 2 * K; idx += kWave) {
    const int i = idx / (2 * K), c = idx - i * 2 * K;
    double v = 0.0;
    if (c >= K) {
      v = (c - K == i) ? 1.0 : 0.0;
    } else if (i < kl) {
      if (c < kl) v = u_entry(Ut, t.BW, m - kl + i, m - kl + c);
      else v = E1[(Q - kl + i) * ku + (ku - 1 - (c - kl))];
    } else {
      const int ib = i - kl;
      if (c < kl) v = E2[(Q - ku + ib) * kl + c];
      else v = u_entry(Ub, bt.BW, nb - ku + ib, nb - ku + (c - kl));
    }
    R[idx] = v;
  }
  __syncthreads();
  // Gauss-Jordan with partial pivoting
  for (int c = 0; c < K; ++c) {
    double mag = -1.0;
    int idx = c;
    if (lane < K - c) {
      mag = fabs(R[(c + lane) * 2 * K + c]);
      idx = c + lane;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double om = __shfl_xor(mag, off);
      const int oi = __shfl_xor(idx, off);
      if (om > mag || (om == mag && oi < idx)) {
        mag = om;
        idx = oi;
      }
    }
    if (lane == 0) piv_s = idx;
    __syncthreads();
    const int pr = piv_s;
    if (pr != c)
      for (int q = lane; q < 2 * K; q += kWave) {
        const double x = R[c * 2 * K + q];
        R[c * 2 * K + q] = R[pr * 2 * K + q];
        R[pr * 2 * K + q] = x;
      }
    __syncthreads();
    double pv = R[c * 2 * K + c];
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) {
      if (lane == 0) atomicMin(sing, p);
      pv = 1.0;
    }
    const double rp = 1.0 / pv;
    __syncthreads();
    for (int q = lane; q < 2 * K; q += kWave) R[c * 2 * K + q] *= rp;
    __syncthreads();
    if (lane < K) mult[lane] = lane == c ? 0.0 : R[lane * 2 * K + c];
    __syncthreads();
    for (int i2 = lane; i2 < K * 2 * K; i2 += kWave) {
      const int i = i2 / (2 * K), q = i2 - i * 2 * K;
      R[i2] -= mult[i] * R[c * 2 * K + q];
    }
    __syncthreads();
  }
  for (int idx = lane; idx < K * K; idx += kWave) {
    const int i = idx / K, c = idx - i * K;
    Rinv[(size_t)p * K * K + idx] = R[i * 2 * K + K + c];
  }
  for (int idx = lane; idx < Q * ku; idx += kWave) E1o[(size_t)p * Q * ku + idx] = E1[idx];
  for (int idx = lane; idx < Q * kl; idx += kWave) E2o[(size_t)p * Q * kl + idx] = E2[idx];
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int factor_stride(int n) { return (n + kCH - 1) / kCH * kCH; }
int factor_slack() { return kRing; }

hipError_t launch_factor(const PencilArgs& a, double a0, double b0, double* Lf, uint8_t* sl,
                         double* Uf, int* sing, hipStream_t st, double* tailL, uint8_t* tailP) {
  const int kv = a.kl + a.ku;
  if (a.kl + 1 > a.FW || kv + 1 > a.BW || kv > kWave - 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)(kv + 1) * (kv + 2) * sizeof(double);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(a.P), dim3(kWave), lds, st, a, a0, b0, Lf, sl, Uf, sing, tailL, tailP);
  };
  // register rows: the kl + 1 = 11 rows of the 3-D operators instead of the
  // whole 16-slot window
  if (a.FW == 8) go(factor_kernel<8>);
  else if (a.FW == 16 && a.kl + 1 <= 11) go(factor_kernel<16, 11>);
  else if (a.FW == 16) go(factor_kernel<16>);
  else if (a.FW == 32) go(factor_kernel<32>);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}


hipError_t launch_coupling(const PencilArgs& t, const PencilArgs& bt, double a0, double b0,
                           const double* tailLt, const uint8_t* tailPt, const double* tailLb,
                           const uint8_t* tailPb, const double* Uft, const double* Ufb,
                           double* Rinv, double* E1, double* E2, int* sing, hipStream_t st) {
  const int K = t.kl + t.ku;
  if (K > 64 || t.Q != K) return hipErrorInvalidValue;
  const size_t lds = (size_t)(t.Q * (t.kl + t.ku) + K * 2 * K) * sizeof(double);
  allow_lds((const void*)coupling_kernel, lds);
  hipLaunchKernelGGL(coupling_kernel, dim3(t.P), dim3(kWave), lds, st, t, bt, a0, b0, tailLt, tailPt,
                     tailLb, tailPb, Uft, Ufb, Rinv, E1, E2, sing);
  return hipGetLastError();
}


}  // namespace stau
