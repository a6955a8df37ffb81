// Register-window sweeps of one real right-hand side through the stored
// banded LU factors of one pencil (the factor layout is described in
// k_factor.hip): shared by the batched solve and the stability solver.
#pragma once

#include "pencil.h"

namespace stau {

// (FW, BW) instances of the sweep kernels: forward window and backward band
// widths of the stored factors
#define STAU_SWEEP_VARIANTS(X) \
  X(8, 32) X(8, 48) X(8, 64) X(16, 32) X(16, 48) X(16, 64) X(32, 32) X(32, 48) X(32, 64)

// ---------------------------------------------------------------------------
// Sweeps of one real right-hand side b (this wavefront's own vector in LDS,
// padded: BW finite values before row 0, FW after row npad - 1, npad = nch *
// kCH) through the stored factors of one pencil:
//   forward  y = L^{-1} P b  (window of FW pending rows in physical slots:
//            lane s holds the row in slot s; the pivot's slot is refilled
//            with the next row, the others take the rank-1 update);
//   backward x = U^{-1} y    (lane l carries row r = l mod BW of the window
//            [j - BW + 1, j]; lane j mod BW holds 1 / U(j, j)).
// Factor coefficients stream from global memory straight into a ring of
// kRing registers per lane, kRing columns ahead of their use: no LDS staging
// and no barrier, so each wavefront sweeps on its own.  The factor arrays
// hold nst = npad columns per pencil (zero beyond n) with kRing columns of
// slack before the first pencil and after the last, so the look-ahead loads
// never leave the allocation (their values past the sweep are not used).
// ---------------------------------------------------------------------------
template <typename T, int FW>
__device__ __forceinline__ void sweep_forward(T* b, const T* __restrict__ Lp,
                                              const uint32_t* __restrict__ sw, int nch, int lane) {
  constexpr int CH = kCH, D = kRing, G = 16;
  static_assert(CH % D == 0 && D % 4 == 0 && CH % G == 0 && FW <= 32, "sweep geometry");
  const int lf = lane & (FW - 1);
  T ring[D];
  uint32_t sring[D / 4];
#pragma unroll
  for (int k = 0; k < D; ++k) ring[k] = Lp[k * FW + lf];
#pragma unroll
  for (int k = 0; k < D / 4; ++k) sring[k] = sw[k];
  T w = lane < FW ? b[lane] : (T)0;
  for (int c = 0; c < nch; ++c) {
    const int j0 = c * CH;
    const T* Ln = Lp + (size_t)(j0 + D) * FW + lf;  // column j0 + D + t at Ln[t * FW]
    const uint32_t* Sn = sw + (j0 + D) / 4;
    T* yo = b + j0;
    T nv[2][G];
#pragma unroll
    for (int k = 0; k < G; ++k) nv[0][k] = yo[k + FW];
#pragma unroll
    for (int k = 0; k < G; ++k) pin(nv[0][k]);
    uint32_t word = 0;
    T yacc = (T)0;  // lane t: y of column j0 + t
    static_for<0, CH / G>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if (g + 1 < CH / G) {
#pragma unroll
        for (int k = 0; k < G; ++k) nv[(g + 1) & 1][k] = yo[(g + 1) * G + k + FW];
      }
      static_for<0, G>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int t = g * G + k;
        if ((t & 3) == 0) word = __builtin_amdgcn_readfirstlane(sring[(t >> 2) % (D / 4)]);
        const int s = (word >> (8 * (t & 3))) & 0xff;
        const T y = readlane_t(w, s);
        put_lane<t>(yacc, y);
        const T l = ring[t % D];
        ring[t % D] = Ln[t * FW];
        if ((t & 3) == 3) sring[(t >> 2) % (D / 4)] = Sn[t >> 2];
        // lane s takes the next row (the lane mask is formed on the scalar
        // unit); its multiplier is 0, so the select is made before the
        // update, beside the lane read instead of after the FMA
        const T ws = __builtin_amdgcn_inverse_ballot_w64(1ull << s) ? nv[g & 1][k] : w;
        w = fma(-l, y, ws);
      });
      if (g + 1 < CH / G) {
#pragma unroll
        for (int k = 0; k < G; ++k) pin(nv[(g + 1) & 1][k]);
      }
    });
    yo[lane] = yacc;
  }

}

// Backward window of BW rows: lane l < BW carries the row r = l mod BW (lanes
// l + BW < 64 carry a copy).  When BW divides the chunk the row of column j
// sits at a compile-time lane of the unrolled loop; otherwise (BW = 48) the
// lane j mod BW is formed on the scalar unit per column from j0 mod BW.
template <int BW>
__device__ __forceinline__ uint64_t window_lanes(int s) {
  uint64_t m = 1ull << s;
  if (s + BW < 64) m |= 1ull << (s + BW);
  return m;
}
template <int BW>
__device__ __forceinline__ int window_lane(int s0, int t) {
  int s = s0 + t;
  if (s >= BW) s -= BW;
  if (s >= BW) s -= BW;
  return s;
}
// row of the last BW rows [npad - BW, npad) that lane lb carries
template <int BW>
__device__ __forceinline__ int window_start_row(int npad, int lb) {
  return npad - BW + (lb - npad % BW + BW) % BW;
}

template <typename T, int BW>
__device__ __forceinline__ void sweep_backward(T* b, const T* __restrict__ Up, int nch, int lane) {
  constexpr int CH = kCH, D = kRing, G = 16;
  static_assert(CH % D == 0 && CH % G == 0 && BW % 16 == 0 && BW <= 64, "sweep geometry");
  constexpr bool kDiv = CH % BW == 0;
  const int npad = nch * CH;
  // columns descending
  const int lb = lane % BW;
  T ring[D];
#pragma unroll
  for (int k = 0; k < D; ++k) ring[k] = Up[(size_t)(npad - D + k) * BW + lb];  // slot j mod D
  // rows npad-BW .. npad-1 (rows >= n hold finite padding; their U
  // coefficients are zero)
  T w = b[window_start_row<BW>(npad, lb)];
  for (int c = nch - 1; c >= 0; --c) {
    const int j0 = c * CH;
    const int s0 = kDiv ? 0 : j0 % BW;
    const T* Un = Up + ((ptrdiff_t)j0 - D) * BW + lb;  // column j0 - D + t at Un[t * BW]
    T* xo = b + j0;
    constexpr int NG = CH / G;
    T nv[2][G];
#pragma unroll
    for (int k = 0; k < G; ++k) nv[(NG - 1) & 1][k] = xo[(NG - 1) * G + k - BW];
#pragma unroll
    for (int k = 0; k < G; ++k) pin(nv[(NG - 1) & 1][k]);
    T xacc = (T)0;  // lane t: x of column j0 + t
    static_for<0, NG>([&](auto gc) {
      constexpr int g = NG - 1 - decltype(gc)::value;
      if (g > 0) {
#pragma unroll
        for (int k = 0; k < G; ++k) nv[(g - 1) & 1][k] = xo[(g - 1) * G + k - BW];
      }
      static_for<0, G>([&](auto kc) {
        constexpr int k = G - 1 - decltype(kc)::value;
        constexpr int t = g * G + k;
        const int sj = kDiv ? t % BW : window_lane<BW>(s0, t);
        const uint64_t msj = window_lanes<BW>(sj);
        const T u = ring[t % D];
        ring[t % D] = Un[t * BW];
        const T x = readlane_t(w * u, sj);
        put_lane<t>(xacc, x);
        w = __builtin_amdgcn_inverse_ballot_w64(msj) ? nv[g & 1][k] : fma(-u, x, w);  // lanes l = sj mod BW
      });
      if (g > 0) {
#pragma unroll
        for (int k = 0; k < G; ++k) pin(nv[(g - 1) & 1][k]);
      }
    });
    xo[lane] = xacc;
  }}

template <typename T, int FW, int BW>
__device__ __forceinline__ void sweeps(T* b, const T* __restrict__ Lp, const uint32_t* __restrict__ sw,
                                       const T* __restrict__ Up, int nch, int lane) {
  sweep_forward<T, FW>(b, Lp, sw, nch, lane);
  sweep_backward<T, BW>(b, Up, nch, lane);
}

}  // namespace stau
