// Pencil solve kernels: the batched banded solve (one wavefront per pencil
// and real part, register windows), its two-block and transposed forms and
// the refined mixed-precision solve.  The factor layout they read is
// described in k_factor.hip.
#include <algorithm>

#include "sweeps.h"

namespace stau {

// ---------------------------------------------------------------------------
// Sweeps with the factor columns staged through LDS.  A 64-lane global load
// costs the load unit of a compute unit about 16 cycles whatever the number
// of distinct addresses, so one load per column and wavefront limits a
// sweep once four or more wavefronts share a compute unit.  Here the columns
// move in units of SU columns with loads of 64 distinct addresses (16 bytes
// per lane, 1 KB per instruction; 8 bytes for a 512-byte unit), K units
// ahead of their use, through two LDS buffers per wavefront, and each column
// is then one LDS read into a ring of kSR registers.  K units are in flight
// in registers (unit u in register set u mod K): at the start of processing
// unit v the data of unit v + 1 is written to LDS buffer (v + 1) mod 2 and
// unit v + 1 + K is loaded into the freed registers; reads of unit v + 1
// begin kSR columns before it.  K sets how far ahead of their use the
// global loads are issued (K SU columns), which must cover the memory
// latency when only a few wavefronts share a SIMD.  Every load is issued
// unconditionally (past the last unit the last one again): a load under a
// branch makes the compiler wait for all outstanding loads (vmcnt 0) before
// the next LDS store, which would expose the full latency once per unit.  The
// forward sweep's slot bytes come with each unit (a vector load of its words,
// one lane read per four columns): a separate stream of
// them made the compiler wait for nearly all loads at each chunk, and a
// scalar load would share the LDS wait counter with the ring reads.
// ---------------------------------------------------------------------------
constexpr int kSR = 8;  // LDS-read look-ahead (columns)

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// registers of one staging unit of BYTES bytes
template <int BYTES>
struct UnitRegs {
  using V = typename std::conditional<BYTES % 1024 == 0, u32x4, u32x2>::type;
  static constexpr int NL = BYTES / (64 * (int)sizeof(V));
  static_assert(NL >= 1 && NL * 64 * (int)sizeof(V) == BYTES, "staging unit size");
  V r[NL];
  __device__ __forceinline__ void load(const void* __restrict__ src, int lane) {
#pragma unroll
    for (int i = 0; i < NL; ++i) r[i] = ((const V*)src)[i * 64 + lane];
  }
  __device__ __forceinline__ void store(void* dst, int lane) const {
#pragma unroll
    for (int i = 0; i < NL; ++i) ((V*)dst)[i * 64 + lane] = r[i];
  }
};

// LDS bytes of the factor stage of one wavefront (forward and backward reuse it)
template <typename T, int FW, int BW, int SU>
constexpr int stage_bytes() {
  return 2 * SU * (FW > BW ? FW : BW) * (int)sizeof(T);
}

// Two sweeping wavefronts share each SIMD in the two-block solve, and the
// instruction arbiter prefers the older one, so the second block on a compute
// unit ran its sweeps about 1.5x slower than the first.  Taking turns at a
// raised wave priority in the forward sweeps, chunk by chunk (psel = 0 or 1
// for the two blocks that share a unit), evens their progress (forward 93k /
// 137k cycles -> 101k / 115k); the slowest wavefront sets the kernel time.
// Turns every 16 columns, or also in the backward sweeps (whose skew is
// small), measured slower.
__device__ __forceinline__ void prio_turn(int chunk, int psel) {
  if ((chunk + psel) & 1)
    __builtin_amdgcn_s_setprio(1);
  else
    __builtin_amdgcn_s_setprio(0);
}

template <typename T, int FW, int SU, int K = 2>
__device__ __forceinline__ void sweep_forward_staged(T* b, const T* __restrict__ Lp,
                                                     const uint32_t* __restrict__ sw, int nch,
                                                     int lane, T* st, int psel = -1) {
  constexpr int CH = kCH, G = 16, R = kSR, UPC = CH / SU;
  static_assert(CH % SU == 0 && UPC % 2 == 0 && UPC % K == 0 && K >= 2 && R <= SU &&
                    CH % G == 0 && FW <= 32,
                "sweep geometry");
  constexpr int FB = SU * FW * (int)sizeof(T);
  constexpr int SWU = SU / 4;  // slot words of a unit (four columns per word)
  const int nu = nch * UPC;
  const int lf = lane & (FW - 1);
  // units in flight: unit u in r[u mod K], its slot words in swr[u mod K]
  // (lane i holds word i mod SWU: a lane-dependent address keeps it a vector
  // load); the words travel with the unit's data, so that one wait covers both
  UnitRegs<FB> r[K];
  uint32_t swr[K];
  auto load_unit = [&](int k, int u) {
    r[k].load(Lp + (size_t)u * SU * FW, lane);
    swr[k] = sw[u * SWU + (lane & (SWU - 1))];
  };
  load_unit(0, 0);
#pragma unroll
  for (int u = 1; u < K; ++u) load_unit(u, u < nu ? u : nu - 1);
  r[0].store(st, lane);
  // slot words of the next and the current unit, read into scalar registers
  // when the unit's data goes to LDS (copies of loaded vector registers
  // across the chunk loop would wait for every load in flight)
  uint32_t wnx[SWU], wcur[SWU];
#pragma unroll
  for (int i = 0; i < SWU; ++i) wnx[i] = (uint32_t)__builtin_amdgcn_readlane(swr[0], i);
  load_unit(0, K < nu ? K : nu - 1);
  T ring[R];
#pragma unroll
  for (int k = 0; k < R; ++k) ring[k] = st[k * FW + lf];
  T w = lane < FW ? b[lane] : (T)0;
  for (int c = 0; c < nch; ++c) {
    if (psel >= 0) prio_turn(c, psel);
    const int j0 = c * CH;
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
        if constexpr (t % SU == 0) {
          // start of unit v = c UPC + t / SU: unit v + 1 to LDS, unit v + 1 + K
          // requested (c UPC is a multiple of K, so the register set is fixed)
          const int vk = c * UPC + t / SU + 1 + K;
          constexpr int rs = (t / SU + 1) % K;
          // (the pin keeps the lane reads here: the compiler would hoist every
          // unit's reads to the top of the chunk, waiting for all loads)
          asm volatile("" : "+v"(swr[rs]));
#pragma unroll
          for (int i = 0; i < SWU; ++i) {
            wcur[i] = wnx[i];
            wnx[i] = (uint32_t)__builtin_amdgcn_readlane(swr[rs], i);
          }
          r[rs].store(st + ((t / SU + 1) & 1) * SU * FW, lane);
          load_unit(rs, vk < nu ? vk : nu - 1);
        }
        if constexpr ((t & 3) == 0) word = wcur[(t % SU) >> 2];
        const int s = (word >> (8 * (t & 3))) & 0xff;
        const T y = readlane_t(w, s);
        put_lane<t>(yacc, y);
        const T l = ring[t % R];
        constexpr int tn = t + R;  // column read ahead, buffer by its unit's parity
        ring[t % R] = st[((tn / SU) & 1) * SU * FW + (tn % SU) * FW + lf];
        const T ws = __builtin_amdgcn_inverse_ballot_w64(1ull << s) ? nv[g & 1][k] : w;
        w = fma(-l, y, ws);  // multiplier 0 at the pivot slot: the select precedes the update
      });
      if (g + 1 < CH / G) {
#pragma unroll
        for (int k = 0; k < G; ++k) pin(nv[(g + 1) & 1][k]);
      }
    });
    yo[lane] = yacc;
  }
}

template <typename T, int BW, int SU, int K = 2>
__device__ __forceinline__ void sweep_backward_staged(T* b, const T* __restrict__ Up, int nch,
                                                      int lane, T* st) {
  constexpr int CH = kCH, G = 16, R = kSR, UPC = CH / SU;
  static_assert(CH % SU == 0 && UPC % 2 == 0 && UPC % K == 0 && K >= 2 && R <= SU &&
                    CH % G == 0 && BW % 16 == 0 && BW <= 64,
                "sweep geometry");
  constexpr bool kDiv = CH % BW == 0;
  constexpr int UB = SU * BW * (int)sizeof(T);
  const int npad = nch * CH, nu = nch * UPC;
  // processing index v covers unit nu - 1 - v (columns descending); index v
  // in flight in r[v mod K]
  const int lb = lane % BW;
  UnitRegs<UB> r[K];
  r[0].load(Up + (size_t)(nu - 1) * SU * BW, lane);
#pragma unroll
  for (int u = 1; u < K; ++u)
    r[u].load(Up + (size_t)(u < nu ? nu - 1 - u : 0) * SU * BW, lane);
  r[0].store(st, lane);
  r[0].load(Up + (size_t)(K < nu ? nu - 1 - K : 0) * SU * BW, lane);
  // processing unit v sits in LDS buffer v mod 2; column SU - 1 - k of unit
  // nu - 1 is ring entry k
  T ring[R];
#pragma unroll
  for (int k = 0; k < R; ++k) ring[k] = st[(SU - 1 - k) * BW + lb];
  // rows npad-BW .. npad-1 (rows >= n hold finite padding; their U
  // coefficients are zero)
  T w = b[window_start_row<BW>(npad, lb)];
  for (int c = nch - 1; c >= 0; --c) {
    const int j0 = c * CH;
    const int s0 = kDiv ? 0 : j0 % BW;
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
        constexpr int q = CH - 1 - t;  // position in processing order within the chunk
        if constexpr (q % SU == 0) {
          // unit of processing index v = UPC (nch - 1 - c) + q / SU starts
          const int vk = UPC * (nch - 1 - c) + q / SU + 1 + K;
          constexpr int rs = (q / SU + 1) % K;
          r[rs].store(st + ((q / SU + 1) & 1) * SU * BW, lane);
          r[rs].load(Up + (size_t)(vk < nu ? nu - 1 - vk : 0) * SU * BW, lane);
        }
        const int sj = kDiv ? t % BW : window_lane<BW>(s0, t);
        const uint64_t msj = window_lanes<BW>(sj);
        const T u = ring[q % R];
        constexpr int qn = q + R;  // processing position read ahead
        ring[q % R] = st[((qn / SU) & 1) * SU * BW + (SU - 1 - qn % SU) * BW + lb];
        const T x = readlane_t(w * u, sj);
        put_lane<t>(xacc, x);
        w = __builtin_amdgcn_inverse_ballot_w64(msj) ? nv[g & 1][k] : fma(-u, x, w);
      });
      if (g > 0) {
#pragma unroll
        for (int k = 0; k < G; ++k) pin(nv[(g - 1) & 1][k]);
      }
    });
    xo[lane] = xacc;
  }
}

// Both real parts of one pencil in one wavefront: the right-hand sides b0
// (real part) and b1 (imaginary part) share the stored factors, so each
// staged unit, slot word and LDS read of a column serves two independent
// update chains, whose instructions interleave: the latency of one chain's
// lane read and fused multiply-add is covered by the other's.  Staging as in
// the one-vector sweeps (K units in flight); the incoming rows are read
// from LDS G = 8 columns ahead.
template <typename T, int FW, int SU, int K>
__device__ __forceinline__ void sweep_forward_pair(T* b0, T* b1, const T* __restrict__ Lp,
                                                   const uint32_t* __restrict__ sw, int nch, int lane,
                                                   T* st) {
  constexpr int CH = kCH, G = 8, R = kSR, UPC = CH / SU;
  static_assert(CH % SU == 0 && UPC % 2 == 0 && UPC % K == 0 && K >= 2 && R <= SU &&
                    CH % G == 0 && FW <= 32,
                "sweep geometry");
  constexpr int FB = SU * FW * (int)sizeof(T);
  constexpr int SWU = SU / 4;
  const int nu = nch * UPC;
  const int lf = lane & (FW - 1);
  UnitRegs<FB> r[K];
  uint32_t swr[K];
  auto load_unit = [&](int k, int u) {
    r[k].load(Lp + (size_t)u * SU * FW, lane);
    swr[k] = sw[u * SWU + (lane & (SWU - 1))];
  };
  load_unit(0, 0);
#pragma unroll
  for (int u = 1; u < K; ++u) load_unit(u, u < nu ? u : nu - 1);
  r[0].store(st, lane);
  uint32_t wnx[SWU], wcur[SWU];
#pragma unroll
  for (int i = 0; i < SWU; ++i) wnx[i] = (uint32_t)__builtin_amdgcn_readlane(swr[0], i);
  load_unit(0, K < nu ? K : nu - 1);
  T ring[R];
#pragma unroll
  for (int k = 0; k < R; ++k) ring[k] = st[k * FW + lf];
  T w0 = lane < FW ? b0[lane] : (T)0, w1 = lane < FW ? b1[lane] : (T)0;
  for (int c = 0; c < nch; ++c) {
    const int j0 = c * CH;
    T* yo0 = b0 + j0;
    T* yo1 = b1 + j0;
    T n0[2][G], n1[2][G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      n0[0][k] = yo0[k + FW];
      n1[0][k] = yo1[k + FW];
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      pin(n0[0][k]);
      pin(n1[0][k]);
    }
    uint32_t word = 0;
    T ya0 = (T)0, ya1 = (T)0;  // lane t: y of column j0 + t
    static_for<0, CH / G>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if (g + 1 < CH / G) {
#pragma unroll
        for (int k = 0; k < G; ++k) {
          n0[(g + 1) & 1][k] = yo0[(g + 1) * G + k + FW];
          n1[(g + 1) & 1][k] = yo1[(g + 1) * G + k + FW];
        }
      }
      static_for<0, G>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int t = g * G + k;
        if constexpr (t % SU == 0) {
          const int vk = c * UPC + t / SU + 1 + K;
          constexpr int rs = (t / SU + 1) % K;
          asm volatile("" : "+v"(swr[rs]));
#pragma unroll
          for (int i = 0; i < SWU; ++i) {
            wcur[i] = wnx[i];
            wnx[i] = (uint32_t)__builtin_amdgcn_readlane(swr[rs], i);
          }
          r[rs].store(st + ((t / SU + 1) & 1) * SU * FW, lane);
          load_unit(rs, vk < nu ? vk : nu - 1);
        }
        if constexpr ((t & 3) == 0) word = wcur[(t % SU) >> 2];
        const int s = (word >> (8 * (t & 3))) & 0xff;
        const T y0 = readlane_t(w0, s), y1 = readlane_t(w1, s);
        put_lane<t>(ya0, y0);
        put_lane<t>(ya1, y1);
        const T l = ring[t % R];
        constexpr int tn = t + R;
        ring[t % R] = st[((tn / SU) & 1) * SU * FW + (tn % SU) * FW + lf];
        const bool in = __builtin_amdgcn_inverse_ballot_w64(1ull << s);
        const T ws0 = in ? n0[g & 1][k] : w0;
        const T ws1 = in ? n1[g & 1][k] : w1;
        w0 = fma(-l, y0, ws0);
        w1 = fma(-l, y1, ws1);
      });
      if (g + 1 < CH / G) {
#pragma unroll
        for (int k = 0; k < G; ++k) {
          pin(n0[(g + 1) & 1][k]);
          pin(n1[(g + 1) & 1][k]);
        }
      }
    });
    yo0[lane] = ya0;
    yo1[lane] = ya1;
  }
}

template <typename T, int BW, int SU, int K>
__device__ __forceinline__ void sweep_backward_pair(T* b0, T* b1, const T* __restrict__ Up, int nch,
                                                    int lane, T* st) {
  constexpr int CH = kCH, G = 8, R = kSR, UPC = CH / SU;
  static_assert(CH % SU == 0 && UPC % 2 == 0 && UPC % K == 0 && K >= 2 && R <= SU &&
                    CH % G == 0 && BW % 16 == 0 && BW <= 64,
                "sweep geometry");
  constexpr bool kDiv = CH % BW == 0;
  constexpr int UB = SU * BW * (int)sizeof(T);
  const int npad = nch * CH, nu = nch * UPC;
  const int lb = lane % BW;
  UnitRegs<UB> r[K];
  r[0].load(Up + (size_t)(nu - 1) * SU * BW, lane);
#pragma unroll
  for (int u = 1; u < K; ++u) r[u].load(Up + (size_t)(u < nu ? nu - 1 - u : 0) * SU * BW, lane);
  r[0].store(st, lane);
  r[0].load(Up + (size_t)(K < nu ? nu - 1 - K : 0) * SU * BW, lane);
  T ring[R];
#pragma unroll
  for (int k = 0; k < R; ++k) ring[k] = st[(SU - 1 - k) * BW + lb];
  const int r0 = window_start_row<BW>(npad, lb);
  T w0 = b0[r0], w1 = b1[r0];
  for (int c = nch - 1; c >= 0; --c) {
    const int j0 = c * CH;
    const int s0 = kDiv ? 0 : j0 % BW;
    T* xo0 = b0 + j0;
    T* xo1 = b1 + j0;
    constexpr int NG = CH / G;
    T n0[2][G], n1[2][G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      n0[(NG - 1) & 1][k] = xo0[(NG - 1) * G + k - BW];
      n1[(NG - 1) & 1][k] = xo1[(NG - 1) * G + k - BW];
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      pin(n0[(NG - 1) & 1][k]);
      pin(n1[(NG - 1) & 1][k]);
    }
    T xa0 = (T)0, xa1 = (T)0;  // lane t: x of column j0 + t
    static_for<0, NG>([&](auto gc) {
      constexpr int g = NG - 1 - decltype(gc)::value;
      if (g > 0) {
#pragma unroll
        for (int k = 0; k < G; ++k) {
          n0[(g - 1) & 1][k] = xo0[(g - 1) * G + k - BW];
          n1[(g - 1) & 1][k] = xo1[(g - 1) * G + k - BW];
        }
      }
      static_for<0, G>([&](auto kc) {
        constexpr int k = G - 1 - decltype(kc)::value;
        constexpr int t = g * G + k;
        constexpr int q = CH - 1 - t;
        if constexpr (q % SU == 0) {
          const int vk = UPC * (nch - 1 - c) + q / SU + 1 + K;
          constexpr int rs = (q / SU + 1) % K;
          r[rs].store(st + ((q / SU + 1) & 1) * SU * BW, lane);
          r[rs].load(Up + (size_t)(vk < nu ? nu - 1 - vk : 0) * SU * BW, lane);
        }
        const int sj = kDiv ? t % BW : window_lane<BW>(s0, t);
        const uint64_t msj = window_lanes<BW>(sj);
        const T u = ring[q % R];
        constexpr int qn = q + R;
        ring[q % R] = st[((qn / SU) & 1) * SU * BW + (SU - 1 - qn % SU) * BW + lb];
        const T x0 = readlane_t(w0 * u, sj), x1 = readlane_t(w1 * u, sj);
        put_lane<t>(xa0, x0);
        put_lane<t>(xa1, x1);
        const bool in = __builtin_amdgcn_inverse_ballot_w64(msj);
        w0 = in ? n0[g & 1][k] : fma(-u, x0, w0);
        w1 = in ? n1[g & 1][k] : fma(-u, x1, w1);
      });
      if (g > 0) {
#pragma unroll
        for (int k = 0; k < G; ++k) {
          pin(n0[(g - 1) & 1][k]);
          pin(n1[(g - 1) & 1][k]);
        }
      }
    });
    xo0[lane] = xa0;
    xo1[lane] = xa1;
  }
}

// Staged sweeps of the single-block solve: the forward sweep keeps its
// register ring of global loads (faster at one wavefront per SIMD), the
// backward sweep stages its BW-wide columns in units of 32.
constexpr int kSU = 32;

// Both sweeps staged in small units (su3 columns) for launches with many
// blocks per compute unit: each column's factor then costs an LDS read
// instead of a 64-lane global load, whose load-unit cost (about 16 cycles per
// unit whatever the addresses) limits the unstaged sweeps once several
// wavefronts share a unit; small units keep two blocks per unit.
// (8 columns for FP64, 16 for FP32: a unit holds at least 512 bytes)
template <typename T>
constexpr int su3() {
  return sizeof(T) == 8 ? 8 : 16;
}

template <typename T, int FW, int BW, int K = 2>
__device__ __forceinline__ void sweeps_staged_both(T* b, const T* __restrict__ Lp,
                                                   const uint32_t* __restrict__ sw,
                                                   const T* __restrict__ Up, int nch, int lane, T* st) {
  sweep_forward_staged<T, FW, su3<T>(), K>(b, Lp, sw, nch, lane, st);
  sweep_backward_staged<T, BW, su3<T>(), K>(b, Up, nch, lane, st);
}

template <typename T, int FW, int BW>
__device__ __forceinline__ void sweeps_staged(T* b, const T* __restrict__ Lp,
                                              const uint32_t* __restrict__ sw,
                                              const T* __restrict__ Up, int nch, int lane, T* st) {
  sweep_forward<T, FW>(b, Lp, sw, nch, lane);
  sweep_backward_staged<T, BW, kSU>(b, Up, nch, lane, st);
}

// Right-hand side of the real-scaled system for one pencil, one real part
// (part 0: real, 1: imaginary), written to b[-BW .. npad + FW): boundary rows
// take the Dirichlet values (b at the mean pencil, real part), the evolved-
// equation U-rows n <= N-2 the entries of Bev (u, v rows times i), all else
// zero.  The zero fill comes first and the Bev entries are then read in
// their own order (coalesced, independent loads) and scattered to their rows;
// both passes belong to one wavefront, whose LDS accesses stay in order.
template <typename T>
__device__ __forceinline__ void build_rhs(const PencilArgs& a, const PencilCoef& pc,
                                          const double2* __restrict__ Bp, int part, T* b, double* b64,
                                          int BW, int FW, int npad, int lane) {
  const SysDesc& d = a.desc;
  const int n = a.n, N = d.N, S = d.S, kb = d.kb, ne = d.ne;
  for (int r = lane - BW; r < npad + FW; r += kWave) {
    double v = 0.0;
    if (part == 0 && r >= 0 && r < kb && pc.mean && d.bc_var[r] == VB)
      v = d.bc_side[r] == 0 ? a.b_bottom : a.b_top;
    b[r] = (T)v;
    if (b64 && r >= 0 && r < n) b64[r] = v;
  }
  const int Nm = N - 1;
#pragma unroll 4
  for (int i = lane; i < ne * Nm; i += kWave) {
    const int e = i / Nm, m = i - e * Nm;
    const int eq = e == 0 ? EB : (e == ne - 1 ? EW : (e == 1 ? EU : EV));
    const double2 v = Bp[e * N + m];
    const bool scaled = eq == EU || eq == EV;  // row scaled by i
    const double val = part == 0 ? (scaled ? -v.y : v.x) : (scaled ? v.x : v.y);
    const int r = kb + m * S + d.eq_pos[eq];
    b[r] = (T)val;
    if (b64) b64[r] = val;
  }
}

// X = P^R x~ with the real scaling undone, state layout (both parts in LDS).
__device__ __forceinline__ void write_state(const PencilArgs& a, const double* xr_, const double* xi_,
                                            double2* __restrict__ Xp, int tid, int nt) {
  const SysDesc& d = a.desc;
  const int N = d.N, S = d.S;
  for (int i = tid; i < S * N; i += nt) {
    const int vabi = i / N, m = i - vabi * N;
    const int var = a.var_of_abi[vabi];
    const int pos = d.var_pos[var];
    double xr = xr_[m * S + pos], xi = xi_[m * S + pos];
    if (m + 2 < N) {
      xr -= xr_[(m + 2) * S + pos];
      xi -= xi_[(m + 2) * S + pos];
    }
    if (var == VU || var == VUZ || var == VV || var == VVZ)
      Xp[i] = make_double2(xi, -xr);  // u = -i u~
    else
      Xp[i] = make_double2(xr, xi);
  }
}

// ---------------------------------------------------------------------------
// Pencil blocks: two pencils per block of four wavefronts, wave 2 q + part
// for pencil 2 blockIdx.x + q and real part `part` (the real-scaled matrix is
// real, so the real and imaginary parts of the right-hand side are two
// independent real solves).  Blocks cover pencils [0, plaunch); block 0 also
// zeroes the state of the inactive pencils [plaunch, P) (in 2-D the Nyquist
// pencil), so that a launch of plaunch / 2 <= #CU blocks can place one block
// per compute unit and one sweeping wavefront per SIMD.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void zero_pencils(double2* __restrict__ X, size_t first, size_t last,
                                             int stride, int tid, int nt) {
  for (size_t i = first * stride + tid; i < last * stride; i += nt) X[i] = make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------------------
// Solve: each wavefront builds its real vector in LDS, overwrites it by
// y = L^{-1} P b and x~ = U^{-1} y, and after one barrier the pencil's two
// wavefronts write X = P^R x~.
// ---------------------------------------------------------------------------
// STG: 0 unstaged sweeps, 1 backward sweep staged (kSU), 2 both staged (kSU3)
template <int FW, int BW, int STG>
__global__ void __launch_bounds__(4 * kWave) solve_kernel(PencilArgs a, int plaunch,
                                                          const double2* __restrict__ Bev,
                                                          const double* __restrict__ Lf,
                                                          const uint8_t* __restrict__ sl,
                                                          const double* __restrict__ Uf,
                                                          double2* __restrict__ X) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = wv >> 1, part = wv & 1;
  const int p = blockIdx.x * 2 + q;
  const SysDesc& d = a.desc;
  const int N = d.N, S = d.S, ne = d.ne;
  if (blockIdx.x == 0 && plaunch < a.P) zero_pencils(X, plaunch, a.P, S * N, tid, 4 * kWave);
  const bool live = p < plaunch;
  const bool act = live && pencil_active(a, p);
  const int npad = a.nst, nch = npad / kCH;
  const int span = BW + npad + FW;
  double* bre = lds + (size_t)q * 2 * span + BW;
  double* bim = bre + span;
  if (act) {
    const PencilCoef pc = pencil_coef(a, p, 0.0, 0.0);
    double* b = part == 0 ? bre : bim;
    build_rhs<double>(a, pc, Bev + (size_t)p * ne * N, part, b, nullptr, BW, FW, npad, lane);
    const double* Lp = Lf + (size_t)p * npad * FW;
    const uint32_t* swp = (const uint32_t*)(sl + (size_t)p * npad);
    const double* Up = Uf + (size_t)p * npad * BW;
    if constexpr (STG == 2) {
      // eight units (64 columns) of loads in flight: at two blocks per compute
      // unit, two units left the sweeps waiting on memory (solve of the
      // 256 x 256 x 128 workload 5.77 ms with two, 5.38 with four, 5.21 with eight)
      double* stg = lds + (size_t)4 * span + (size_t)wv * (stage_bytes<double, FW, BW, su3<double>()>() / 8);
      sweeps_staged_both<double, FW, BW, 8>(b, Lp, swp, Up, nch, lane, stg);
    } else if constexpr (STG == 1) {
      double* stg = lds + (size_t)4 * span + (size_t)wv * (stage_bytes<double, 1, BW, kSU>() / 8);
      sweeps_staged<double, FW, BW>(b, Lp, swp, Up, nch, lane, stg);
    } else {
      sweeps<double, FW, BW>(b, Lp, swp, Up, nch, lane);
    }
  }
  __syncthreads();
  if (act)
    write_state(a, bre, bim, X + (size_t)p * S * N, tid & (2 * kWave - 1), 2 * kWave);
  else if (live)
    zero_pencils(X, p, p + 1, S * N, tid & (2 * kWave - 1), 2 * kWave);
}

// ---------------------------------------------------------------------------
// Solve with both real parts of a pencil in one wavefront (sweep_*_pair):
// two pencils per block of two wavefronts, wave q for pencil 2 blockIdx.x + q.
// For launches with many blocks per compute unit: half the waves of
// solve_kernel, each with two update chains, and one factor stage per pencil.
// ---------------------------------------------------------------------------
template <int FW, int BW>
__global__ void __launch_bounds__(2 * kWave) solve_pair_kernel(PencilArgs a, int plaunch,
                                                               const double2* __restrict__ Bev,
                                                               const double* __restrict__ Lf,
                                                               const uint8_t* __restrict__ sl,
                                                               const double* __restrict__ Uf,
                                                               double2* __restrict__ X) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int q = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int p = blockIdx.x * 2 + q;
  const SysDesc& d = a.desc;
  const int N = d.N, S = d.S, ne = d.ne;
  if (blockIdx.x == 0 && plaunch < a.P) zero_pencils(X, plaunch, a.P, S * N, tid, 2 * kWave);
  const bool live = p < plaunch;
  const bool act = live && pencil_active(a, p);
  const int npad = a.nst, nch = npad / kCH;
  const int span = BW + npad + FW;
  double* bre = lds + (size_t)q * 2 * span + BW;
  double* bim = bre + span;
  if (act) {
    const PencilCoef pc = pencil_coef(a, p, 0.0, 0.0);
    const double2* Bp = Bev + (size_t)p * ne * N;
    build_rhs<double>(a, pc, Bp, 0, bre, nullptr, BW, FW, npad, lane);
    build_rhs<double>(a, pc, Bp, 1, bim, nullptr, BW, FW, npad, lane);
    const double* Lp = Lf + (size_t)p * npad * FW;
    const uint32_t* swp = (const uint32_t*)(sl + (size_t)p * npad);
    const double* Up = Uf + (size_t)p * npad * BW;
    double* stg = lds + (size_t)4 * span + (size_t)q * (stage_bytes<double, FW, BW, su3<double>()>() / 8);
    sweep_forward_pair<double, FW, su3<double>(), 8>(bre, bim, Lp, swp, nch, lane, stg);
    sweep_backward_pair<double, BW, su3<double>(), 8>(bre, bim, Up, nch, lane, stg);
  }
  __syncthreads();
  if (act)
    write_state(a, bre, bim, X + (size_t)p * S * N, lane, kWave);
  else if (live)
    zero_pencils(X, p, p + 1, S * N, lane, kWave);
}

// ---------------------------------------------------------------------------
// Streamed solve: the pair sweeps with the pencil's vectors outside LDS, so
// that a compute unit holds about three times the pencils (LDS per
// wavefront: the factor stage and two 64-row rings of incoming rows).
//   * forward: the incoming rows j0 + FW + t of each chunk are formed from
//     Bev (and the boundary values) one chunk ahead, into an LDS ring; the
//     results y of each chunk go to the workspace a.ysp [p][part][nst];
//   * backward: the incoming rows j0 - BW + t come back from the workspace
//     one chunk ahead, into the same ring; each chunk's x~ is recombined at
//     once, X_m = x~_m - x~_{m+2} (the partner 2S columns on, in this chunk
//     or the one before it), and written to the state.
// One wavefront per pencil (both real parts), one pencil per block.
// ---------------------------------------------------------------------------
// right-hand side row r of pencil p, both parts (rows outside [0, n): 0)
__device__ __forceinline__ void rhs_row(const PencilArgs& a, const double2* __restrict__ Bp, bool mean,
                                        int r, double& v0, double& v1) {
  const SysDesc& d = a.desc;
  v0 = v1 = 0.0;
  if (r < 0 || r >= a.n) return;
  if (r < d.kb) {
    if (mean && d.bc_var[r] == VB) v0 = d.bc_side[r] == 0 ? a.b_bottom : a.b_top;
    return;
  }
  const int m = (r - d.kb) / d.S, q = r - d.kb - m * d.S;
  if (m > d.N - 2) return;
  const int eq = d.eq_at[q];
  int e;
  if (eq == EB) e = 0;
  else if (eq == EU) e = 1;
  else if (eq == EV) e = 2;
  else if (eq == EW) e = d.ne - 1;
  else return;
  const double2 v = Bp[e * d.N + m];
  const bool scaled = eq == EU || eq == EV;  // row scaled by i
  v0 = scaled ? -v.y : v.x;
  v1 = scaled ? v.x : v.y;
}

template <int FW, int BW, int K>
__global__ void __launch_bounds__(kWave) solve_stream_kernel(PencilArgs a, int plaunch,
                                                             const double2* __restrict__ Bev,
                                                             const double* __restrict__ Lf,
                                                             const uint8_t* __restrict__ sl,
                                                             const double* __restrict__ Uf,
                                                             double2* __restrict__ X) {
  using T = double;
  extern __shared__ double lds[];
  constexpr int CH = kCH, G = 4, R = kSR, SU = su3<double>(), UPC = CH / SU;
  const int lane = threadIdx.x;
  const int p = blockIdx.x;
  const SysDesc& d = a.desc;
  const int N = d.N, S = d.S, ne = d.ne;
  if (blockIdx.x == 0 && plaunch < a.P) zero_pencils(X, plaunch, a.P, S * N, lane, kWave);
  if (p >= plaunch) return;
  if (!pencil_active(a, p)) {
    zero_pencils(X, p, p + 1, S * N, lane, kWave);
    return;
  }
  const PencilCoef pc = pencil_coef(a, p, 0.0, 0.0);
  const double2* Bp = Bev + (size_t)p * ne * N;
  const int npad = a.nst, nch = npad / CH, n = a.n;
  double* ring = lds;                       // [2 buffers][2 parts][64]
  double* st = lds + 4 * kWave;             // factor stage
  double* Y0 = a.ysp + (size_t)p * 2 * npad;
  double* Y1 = Y0 + npad;
  const double* Lp = Lf + (size_t)p * npad * FW;
  const uint32_t* sw = (const uint32_t*)(sl + (size_t)p * npad);
  const double* Up = Uf + (size_t)p * npad * BW;

  // ---- forward ----
  {
    constexpr int FB = SU * FW * (int)sizeof(T);
    constexpr int SWU = SU / 4;
    const int nu = nch * UPC;
    const int lf = lane & (FW - 1);
    UnitRegs<FB> r[K];
    uint32_t swr[K];
    auto load_unit = [&](int k, int u) {
      r[k].load(Lp + (size_t)u * SU * FW, lane);
      swr[k] = sw[u * SWU + (lane & (SWU - 1))];
    };
    load_unit(0, 0);
#pragma unroll
    for (int u = 1; u < K; ++u) load_unit(u, u < nu ? u : nu - 1);
    r[0].store(st, lane);
    uint32_t wnx[SWU], wcur[SWU];
#pragma unroll
    for (int i = 0; i < SWU; ++i) wnx[i] = (uint32_t)__builtin_amdgcn_readlane(swr[0], i);
    load_unit(0, K < nu ? K : nu - 1);
    T rg[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rg[k] = st[k * FW + lf];
    T w0, w1;
    rhs_row(a, Bp, pc.mean, lane < FW ? lane : -1, w0, w1);
    {
      double i0, i1;
      rhs_row(a, Bp, pc.mean, FW + lane, i0, i1);
      ring[lane] = i0;
      ring[kWave + lane] = i1;
    }
    for (int c = 0; c < nch; ++c) {
      const int j0 = c * CH;
      const double* in0 = ring + (c & 1) * 2 * kWave;
      const double* in1 = in0 + kWave;
      // the next chunk's incoming rows, requested now, stored at the end
      double q0, q1;
      rhs_row(a, Bp, pc.mean, j0 + CH + FW + lane, q0, q1);
      T n0[2][G], n1[2][G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        n0[0][k] = in0[k];
        n1[0][k] = in1[k];
      }
      uint32_t word = 0;
      T ya0 = (T)0, ya1 = (T)0;
      static_for<0, CH / G>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (g + 1 < CH / G) {
#pragma unroll
          for (int k = 0; k < G; ++k) {
            n0[(g + 1) & 1][k] = in0[(g + 1) * G + k];
            n1[(g + 1) & 1][k] = in1[(g + 1) * G + k];
          }
        }
        static_for<0, G>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          constexpr int t = g * G + k;
          if constexpr (t % SU == 0) {
            const int vk = c * UPC + t / SU + 1 + K;
            constexpr int rs = (t / SU + 1) % K;
            asm volatile("" : "+v"(swr[rs]));
#pragma unroll
            for (int i = 0; i < SWU; ++i) {
              wcur[i] = wnx[i];
              wnx[i] = (uint32_t)__builtin_amdgcn_readlane(swr[rs], i);
            }
            r[rs].store(st + ((t / SU + 1) & 1) * SU * FW, lane);
            load_unit(rs, vk < nu ? vk : nu - 1);
          }
          if constexpr ((t & 3) == 0) word = wcur[(t % SU) >> 2];
          const int s = (word >> (8 * (t & 3))) & 0xff;
          STAU_BOUND(a.check, s < FW, kChkSlot);
          const T y0 = readlane_t(w0, s), y1 = readlane_t(w1, s);
          put_lane<t>(ya0, y0);
          put_lane<t>(ya1, y1);
          const T l = rg[t % R];
          constexpr int tn = t + R;
          rg[t % R] = st[((tn / SU) & 1) * SU * FW + (tn % SU) * FW + lf];
          const bool inw = __builtin_amdgcn_inverse_ballot_w64(1ull << s);
          const T ws0 = inw ? n0[g & 1][k] : w0;
          const T ws1 = inw ? n1[g & 1][k] : w1;
          w0 = fma(-l, y0, ws0);
          w1 = fma(-l, y1, ws1);
        });
      });
      Y0[j0 + lane] = ya0;
      Y1[j0 + lane] = ya1;
      double* nx = ring + ((c + 1) & 1) * 2 * kWave;
      nx[lane] = q0;
      nx[kWave + lane] = q1;
    }
  }
  // the workspace rows written above are read back below by this wavefront
  __threadfence_block();

  // ---- backward ----
  {
    constexpr bool kDiv = CH % BW == 0;
    constexpr int UB = SU * BW * (int)sizeof(T);
    const int nu = nch * UPC;
    const int lb = lane % BW;
    UnitRegs<UB> r[K];
    r[0].load(Up + (size_t)(nu - 1) * SU * BW, lane);
#pragma unroll
    for (int u = 1; u < K; ++u) r[u].load(Up + (size_t)(u < nu ? nu - 1 - u : 0) * SU * BW, lane);
    r[0].store(st, lane);
    r[0].load(Up + (size_t)(K < nu ? nu - 1 - K : 0) * SU * BW, lane);
    T rg[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rg[k] = st[(SU - 1 - k) * BW + lb];
    const int r0 = window_start_row<BW>(npad, lb);
    T w0 = Y0[r0], w1 = Y1[r0];
    {
      const int rr = (nch - 1) * CH - BW + lane;  // incoming rows of the last chunk
      ring[lane] = rr >= 0 ? Y0[rr] : 0.0;
      ring[kWave + lane] = rr >= 0 ? Y1[rr] : 0.0;
    }
    // recombination partner: column c + 2S, in this chunk or the one after it
    const int S2 = 2 * S;
    T xp0 = (T)0, xp1 = (T)0;  // x~ of the chunk above
    for (int c = nch - 1; c >= 0; --c) {
      const int j0 = c * CH;
      const int s0 = kDiv ? 0 : j0 % BW;
      const int bsel = (nch - 1 - c) & 1;
      const double* in0 = ring + bsel * 2 * kWave;
      const double* in1 = in0 + kWave;
      double q0 = 0.0, q1 = 0.0;
      {
        const int rr = j0 - CH - BW + lane;  // the next (lower) chunk's incoming rows
        if (c > 0 && rr >= 0) {
          q0 = Y0[rr];
          q1 = Y1[rr];
        }
      }
      constexpr int NG = CH / G;
      T n0[2][G], n1[2][G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        n0[(NG - 1) & 1][k] = in0[(NG - 1) * G + k];
        n1[(NG - 1) & 1][k] = in1[(NG - 1) * G + k];
      }
      T xa0 = (T)0, xa1 = (T)0;
      static_for<0, NG>([&](auto gc) {
        constexpr int g = NG - 1 - decltype(gc)::value;
        if (g > 0) {
#pragma unroll
          for (int k = 0; k < G; ++k) {
            n0[(g - 1) & 1][k] = in0[(g - 1) * G + k];
            n1[(g - 1) & 1][k] = in1[(g - 1) * G + k];
          }
        }
        static_for<0, G>([&](auto kc) {
          constexpr int k = G - 1 - decltype(kc)::value;
          constexpr int t = g * G + k;
          constexpr int q = CH - 1 - t;
          if constexpr (q % SU == 0) {
            const int vk = UPC * (nch - 1 - c) + q / SU + 1 + K;
            constexpr int rs = (q / SU + 1) % K;
            r[rs].store(st + ((q / SU + 1) & 1) * SU * BW, lane);
            r[rs].load(Up + (size_t)(vk < nu ? nu - 1 - vk : 0) * SU * BW, lane);
          }
          const int sj = kDiv ? t % BW : window_lane<BW>(s0, t);
          const uint64_t msj = window_lanes<BW>(sj);
          const T u = rg[q % R];
          constexpr int qn = q + R;
          rg[q % R] = st[((qn / SU) & 1) * SU * BW + (SU - 1 - qn % SU) * BW + lb];
          const T x0 = readlane_t(w0 * u, sj), x1 = readlane_t(w1 * u, sj);
          put_lane<t>(xa0, x0);
          put_lane<t>(xa1, x1);
          const bool inw = __builtin_amdgcn_inverse_ballot_w64(msj);
          w0 = inw ? n0[g & 1][k] : fma(-u, x0, w0);
          w1 = inw ? n1[g & 1][k] : fma(-u, x1, w1);
        });
      });
      // X = P^R x~ for the chunk's columns j0 + lane
      {
        const int sl2 = (lane + S2) & (kWave - 1);
        const bool here = lane + S2 < kWave;
        const T a0 = __shfl(xa0, sl2), b0 = __shfl(xp0, sl2);
        const T a1 = __shfl(xa1, sl2), b1 = __shfl(xp1, sl2);
        const int col = j0 + lane;
        if (col < n) {
          const int m = col / S, pos = col - m * S;
          double v0 = xa0, v1 = xa1;
          if (m + 2 < N) {
            v0 -= here ? a0 : b0;
            v1 -= here ? a1 : b1;
          }
          const int var = d.var_at[pos];
          const double2 xv = (var == VU || var == VUZ || var == VV || var == VVZ) ? make_double2(v1, -v0)
                                                                                  : make_double2(v0, v1);
          X[((size_t)p * S + d.abi_index[var]) * N + m] = xv;
        }
      }
      xp0 = xa0;
      xp1 = xa1;
      double* nx = ring + (bsel ^ 1) * 2 * kWave;
      nx[lane] = q0;
      nx[kWave + lane] = q1;
    }
  }
}

// ---------------------------------------------------------------------------
// Sparse factor records for the streamed solve.  The whole-band factors are
// mostly zeros: the pencil operators hold about six nonzeros per row, and the
// 3-D factors about 11 nonzeros per column of U and 4 multipliers per column
// of L against the 48 + 16 stored slots.  After each factorisation the
// nonzeros are packed per pencil and unit of kSpU columns into records of
// fixed stride, which the streamed solve reads with bounds-checked buffer
// loads (bytes past a record's length are neither fetched nor used):
//   forward record: [0, 16) per column a 16-bit mask of the forward-window
//     slots with a nonzero multiplier, [16, 24) the pivot slot byte per
//     column, [24, 32) zero, then the multipliers, column by column in slot
//     order;
//   backward record: [0, 64) per column a 64-bit mask of the rows of a
//     64-row window (row r at bit r mod 64) with a nonzero of U (the diagonal
//     as its reciprocal), then the entries, columns in descending order, rows
//     in bit order;
//   lengths: per pencil and direction kSpLen bytes, record lengths in 16-byte
//     words.
// A missing entry is a zero of the whole-band factors, which only adds a zero
// product to a row, so both forms give the same results.
// ---------------------------------------------------------------------------
constexpr unsigned kBufWord3 = 0x00020000u;  // raw buffer descriptor word 3: 32-bit data format

// Pack the records of every active pencil from the whole-band factors: a
// block of kPackWaves wavefronts per pencil, wavefront w packing the units
// w, w + kPackWaves, ... (each record at its fixed stride), the eight
// columns' loads of a unit issued together.
constexpr int kPackWaves = 4;

template <int FW, int BW>
__global__ void __launch_bounds__(kPackWaves * kWave) sparse_records_kernel(PencilArgs a,
                                                                            const double* __restrict__ Lf,
                                                                            const uint8_t* __restrict__ sl,
                                                                            const double* __restrict__ Uf,
                                                                            SparseFactors sf) {
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int npad = a.nst, nu = npad / kSpU;
  uint8_t* lf = sf.lenF + (size_t)p * kSpLen;
  uint8_t* lb = sf.lenB + (size_t)p * kSpLen;
  if (!pencil_active(a, p)) {
    for (int u = tid; u < kSpLen; u += kPackWaves * kWave) {
      lf[u] = 0;
      lb[u] = 0;
    }
    return;
  }
  for (int u = nu + tid; u < kSpLen; u += kPackWaves * kWave) {
    lf[u] = 0;
    lb[u] = 0;
  }
  const double* Lp = Lf + (size_t)p * npad * FW;
  const double* Up = Uf + (size_t)p * npad * BW;
  const uint8_t* sp = sl + (size_t)p * npad;
  uint8_t* Fp = sf.F + (size_t)p * nu * sf.strideF;
  uint8_t* Bp = sf.B + (size_t)p * nu * sf.strideB;
  const uint64_t below = (1ull << lane) - 1;  // lanes under this one
  // the strides hold the most entries the band allows (kl multipliers and
  // kl + ku + 1 entries of U per column); nothing is written past them
  const int capF = (sf.strideF - 32) / 8, capB = (sf.strideB - 64) / 8;
  for (int u = wv; u < nu; u += kPackWaves) {
    // forward record
    double lv[kSpU];
#pragma unroll
    for (int t = 0; t < kSpU; ++t) lv[t] = lane < FW ? Lp[(size_t)(u * kSpU + t) * FW + lane] : 0.0;
    uint8_t* rf = Fp + (size_t)u * sf.strideF;
    double* vf = (double*)(rf + 32);
    int cnt = 0;
    uint32_t mine = 0;  // lane t < kSpU: mask of column t
#pragma unroll
    for (int t = 0; t < kSpU; ++t) {
      const double v = lv[t];
      const uint64_t m = __ballot(v != 0.0);
      const int idx = cnt + __popcll(m & below);
      if (v != 0.0 && idx < capF) vf[idx] = v;
      if (lane == t) mine = (uint32_t)m;
      cnt += __popcll(m);
    }
    if (lane < kSpU) {
      ((uint16_t*)rf)[lane] = (uint16_t)mine;
      rf[16 + lane] = sp[u * kSpU + lane];
      rf[24 + lane] = 0;
    }
    const int fb = 32 + 8 * min(cnt, capF);
    if (lane == 0 && (fb & 15)) *(double*)(rf + fb) = 0.0;
    if (lane == 0) lf[u] = (uint8_t)((fb + 15) >> 4);
    // backward record: column j of U moved from the BW-row window of the
    // whole-band form (lane l: row j - ((j - l) mod BW)) to lane r mod 64
    double uv[kSpU];
#pragma unroll
    for (int t = 0; t < kSpU; ++t) uv[t] = lane < BW ? Up[(size_t)(u * kSpU + t) * BW + lane] : 0.0;
    uint8_t* rb = Bp + (size_t)u * sf.strideB;
    double* vb = (double*)(rb + 64);
    int cb = 0;
    uint64_t mb = 0;
#pragma unroll
    for (int q = 0; q < kSpU; ++q) {
      const int t = kSpU - 1 - q, j = u * kSpU + t;
      // this lane's row r = j - k (k = (j - lane) mod 64) sits in the band
      // form's lane r mod BW when k < BW and r >= 0
      const int k = (j - lane) & (kWave - 1);
      int src = (j - k) % BW;
      if (src < 0) src += BW;
      const double g = __shfl(uv[t], src);
      const double v = (k < BW && k <= j) ? g : 0.0;
      const uint64_t m = __ballot(v != 0.0);
      const int idx = cb + __popcll(m & below);
      if (v != 0.0 && idx < capB) vb[idx] = v;
      if (lane == t) mb = m;
      cb += __popcll(m);
    }
    if (lane < kSpU) ((uint64_t*)rb)[lane] = mb;
    STAU_BOUND(a.check, cnt <= capF && cb <= capB, kChkRecord);
    const int bb = 64 + 8 * min(cb, capB);
    if (lane == 0 && (bb & 15)) *(double*)(rb + bb) = 0.0;
    if (lane == 0) lb[u] = (uint8_t)((bb + 15) >> 4);
  }
}

// registers of one record: NB loads of 16 bytes per lane from a record of
// `bytes` bytes (lanes past the end read zeros without a memory access)
template <int NB>
struct RecordRegs {
  u32x4 r[NB];
  __device__ __forceinline__ void load(const uint8_t* rec, int bytes, int lane) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)rec, (short)0, bytes, kBufWord3);
#pragma unroll
    for (int i = 0; i < NB; ++i) r[i] = __builtin_amdgcn_raw_buffer_load_b128(rs, (i * kWave + lane) * 16, 0, 0);
  }
  __device__ __forceinline__ void store(void* dst, int lane) const {
#pragma unroll
    for (int i = 0; i < NB; ++i) ((u32x4*)dst)[i * kWave + lane] = r[i];
  }
};

// record length in bytes of unit u from the lane-held length bytes (lane i:
// units 4i .. 4i + 3)
__device__ __forceinline__ int record_bytes(uint32_t lens, int u) {
  const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)lens, u >> 2);
  return (int)((w >> (8 * (u & 3))) & 0xffu) * 16;
}

// Streamed solve over the sparse records: the flow of solve_stream_kernel
// (incoming rows through an LDS ring, forward results through the workspace,
// recombination per chunk) with the factor columns taken from the records.
// Each column's entry of a lane is read from the staged record at the
// lane's rank among the column's set bits (or from a zero when its bit is
// clear); the backward window has 64 rows, one per lane.  NBB: 16-byte loads
// per lane of a backward record.
template <int FW, int NBB, int K>
__global__ void __launch_bounds__(kWave) solve_sparse_kernel(PencilArgs a, int plaunch,
                                                             const double2* __restrict__ Bev, SparseFactors sf,
                                                             double2* __restrict__ X) {
  using T = double;
  extern __shared__ double lds[];
  constexpr int CH = kCH, G = 4, R = kSR, SU = kSpU, UPC = CH / SU, BW = kWave;
  static_assert(R == SU && UPC % K == 0 && FW <= 16, "record geometry");
  constexpr int SF = 1024 / 8, SB = NBB * 1024 / 8;  // doubles per stage buffer
  const int lane = threadIdx.x;
  const int p = blockIdx.x;
  const SysDesc& d = a.desc;
  const int N = d.N, S = d.S, ne = d.ne;
  if (blockIdx.x == 0 && plaunch < a.P) zero_pencils(X, plaunch, a.P, S * N, lane, kWave);
  if (p >= plaunch) return;
  if (!pencil_active(a, p)) {
    zero_pencils(X, p, p + 1, S * N, lane, kWave);
    return;
  }
  const PencilCoef pc = pencil_coef(a, p, 0.0, 0.0);
  const double2* Bp = Bev + (size_t)p * ne * N;
  const int npad = a.nst, nch = npad / CH, n = a.n, nu = npad / SU;
  // LDS: the ring of incoming rows [2 buffers][2 parts][64], the record stage
  // (two buffers) and a zero read where a mask bit is clear
  double* ring = lds;
  double* st = lds + 4 * kWave;
  const int zoff = 2 * (SF > SB ? SF : SB);
  if (lane == 0) st[zoff] = 0.0;
  const uint32_t zaddr = (uint32_t)((4 * kWave + zoff) * sizeof(double));  // byte address in LDS
  // entry of this lane in a record column with mask m: the value at the
  // lane's rank among the set bits after the column's first rank la (a byte
  // offset in the stage buffer, so one shift-add forms the address)
  auto ld_entry = [&](uint64_t m, uint32_t rank, int first_byte) -> T {
    const uint32_t addr = (rank << 3) + (uint32_t)first_byte;
    const uint32_t sel = __builtin_amdgcn_inverse_ballot_w64(m) ? addr : zaddr;
    // the dynamic LDS array starts at LDS address 0 (no static LDS in this kernel)
    return *(const __attribute__((address_space(3))) T*)(size_t)sel;
  };
  double* Y0 = a.ysp + (size_t)p * 2 * npad;
  double* Y1 = Y0 + npad;
  const uint8_t* Fr = sf.F + (size_t)p * nu * sf.strideF;
  const uint8_t* Br = sf.B + (size_t)p * nu * sf.strideB;
  const uint32_t lensF = ((const uint32_t*)(sf.lenF + (size_t)p * kSpLen))[lane];
  const uint32_t lensB = ((const uint32_t*)(sf.lenB + (size_t)p * kSpLen))[lane];

  // ---- forward ----
  {
    RecordRegs<1> r[K];
    auto load_unit = [&](int k, int u) { r[k].load(Fr + (size_t)u * sf.strideF, record_bytes(lensF, u), lane); };
#pragma unroll
    for (int u = 0; u < K; ++u) load_unit(u, u < nu ? u : nu - 1);
    // header of a record in registers: lane 0 holds the four mask words,
    // lane 1 the two slot words
    uint32_t mnx[4], wnx[2], wcur[2];
    auto header = [&](const RecordRegs<1>& q) {
#pragma unroll
      for (int i = 0; i < 4; ++i) mnx[i] = (uint32_t)__builtin_amdgcn_readlane((int)q.r[0][i], 0);
#pragma unroll
      for (int i = 0; i < 2; ++i) wnx[i] = (uint32_t)__builtin_amdgcn_readlane((int)q.r[0][i], 1);
    };
    header(r[0]);
    r[0].store(st, lane);
    load_unit(0, K < nu ? K : nu - 1);
    // entry of this lane in column c of the staged record in buffer b; la is
    // the rank of the column's first entry in the record
    int la = 0;
    auto entry = [&](int b, int c) -> T {
      const uint32_t m = (mnx[c >> 1] >> (16 * (c & 1))) & 0xffffu;
      const T v = ld_entry(m, __builtin_amdgcn_mbcnt_lo(m, 0u), (4 * kWave + b * SF + 4 + la) * 8);
      la += __builtin_popcount(m);
      return v;
    };
    T rg[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rg[k] = entry(0, k);
    T w0, w1;
    rhs_row(a, Bp, pc.mean, lane < FW ? lane : -1, w0, w1);
    {
      double i0, i1;
      rhs_row(a, Bp, pc.mean, FW + lane, i0, i1);
      ring[lane] = i0;
      ring[kWave + lane] = i1;
    }
    for (int c = 0; c < nch; ++c) {
      const int j0 = c * CH;
      const double* in0 = ring + (c & 1) * 2 * kWave;
      const double* in1 = in0 + kWave;
      double q0, q1;
      rhs_row(a, Bp, pc.mean, j0 + CH + FW + lane, q0, q1);
      T n0[2][G], n1[2][G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        n0[0][k] = in0[k];
        n1[0][k] = in1[k];
      }
      uint32_t word = 0;
      T ya0 = (T)0, ya1 = (T)0;
      static_for<0, CH / G>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (g + 1 < CH / G) {
#pragma unroll
          for (int k = 0; k < G; ++k) {
            n0[(g + 1) & 1][k] = in0[(g + 1) * G + k];
            n1[(g + 1) & 1][k] = in1[(g + 1) * G + k];
          }
        }
        static_for<0, G>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          constexpr int t = g * G + k;
          if constexpr (t % SU == 0) {
            // unit i = c UPC + t / SU starts: unit i + 1 to the stage, its
            // header to scalars, unit i + 1 + K requested
            const int vk = c * UPC + t / SU + 1 + K;
            constexpr int rs = (t / SU + 1) % K;
            wcur[0] = wnx[0];
            wcur[1] = wnx[1];
            header(r[rs]);
#ifdef STAU_CHECK_BOUNDS
            {
              const int ui = c * UPC + t / SU + 1 < nu ? c * UPC + t / SU + 1 : nu - 1;
              int cntf = 0;
              for (int i = 0; i < 4; ++i) cntf += __builtin_popcount(mnx[i]);
              STAU_BOUND(a.check, 32 + 8 * cntf <= record_bytes(lensF, ui), kChkRank);
            }
#endif
            r[rs].store(st + ((t / SU + 1) & 1) * SF, lane);
            load_unit(rs, vk < nu ? vk : nu - 1);
            la = 0;
          }
          if constexpr ((t & 3) == 0) word = wcur[(t % SU) >> 2];
          const int s = (word >> (8 * (t & 3))) & 0xff;
          STAU_BOUND(a.check, s < FW, kChkSlot);
          const T y0 = readlane_t(w0, s), y1 = readlane_t(w1, s);
          put_lane<t>(ya0, y0);
          put_lane<t>(ya1, y1);
          const bool inw = __builtin_amdgcn_inverse_ballot_w64(1ull << s);
          const T l = rg[t % R];
          constexpr int tn = t + R;
          rg[t % R] = entry((tn / SU) & 1, tn % SU);
          const T ws0 = inw ? n0[g & 1][k] : w0;
          const T ws1 = inw ? n1[g & 1][k] : w1;
          w0 = fma(-l, y0, ws0);
          w1 = fma(-l, y1, ws1);
        });
      });
      Y0[j0 + lane] = ya0;
      Y1[j0 + lane] = ya1;
      double* nx = ring + ((c + 1) & 1) * 2 * kWave;
      nx[lane] = q0;
      nx[kWave + lane] = q1;
    }
  }
  // the workspace rows written above are read back below by this wavefront
  __threadfence_block();

  // ---- backward ----
  {
    RecordRegs<NBB> r[K];
    auto load_unit = [&](int k, int v) {  // v-th unit from the top
      const int u = v < nu ? nu - 1 - v : 0;
      r[k].load(Br + (size_t)u * sf.strideB, record_bytes(lensB, u), lane);
    };
#pragma unroll
    for (int v = 0; v < K; ++v) load_unit(v, v);
    // header: lanes 0 .. 3 hold the eight 64-bit masks (two per lane)
    uint64_t mb[kSpU];
    auto header = [&](const RecordRegs<NBB>& q) {
#pragma unroll
      for (int i = 0; i < kSpU; ++i) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)q.r[0][2 * (i & 1)], i >> 1);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)q.r[0][2 * (i & 1) + 1], i >> 1);
        mb[i] = ((uint64_t)hi << 32) | lo;
      }
    };
    header(r[0]);
    r[0].store(st, lane);
    load_unit(0, K);
    int la = 0;
    auto entry = [&](int b, int cpos) -> T {
      const uint64_t m = mb[cpos];
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      const T v = ld_entry(m, rank, (4 * kWave + b * SB + 8 + la) * 8);
      la += __builtin_popcountll(m);
      return v;
    };
    T rg[R];
#pragma unroll
    for (int k = 0; k < R; ++k) rg[k] = entry(0, SU - 1 - k);
    const int r0 = window_start_row<BW>(npad, lane);
    T w0 = Y0[r0], w1 = Y1[r0];
    {
      const int rr = (nch - 1) * CH - BW + lane;  // incoming rows of the last chunk
      ring[lane] = rr >= 0 ? Y0[rr] : 0.0;
      ring[kWave + lane] = rr >= 0 ? Y1[rr] : 0.0;
    }
    const int S2 = 2 * S;
    T xp0 = (T)0, xp1 = (T)0;  // x~ of the chunk above
    for (int c = nch - 1; c >= 0; --c) {
      const int j0 = c * CH;
      const int bsel = (nch - 1 - c) & 1;
      const double* in0 = ring + bsel * 2 * kWave;
      const double* in1 = in0 + kWave;
      double q0 = 0.0, q1 = 0.0;
      {
        const int rr = j0 - CH - BW + lane;  // the next (lower) chunk's incoming rows
        if (c > 0 && rr >= 0) {
          q0 = Y0[rr];
          q1 = Y1[rr];
        }
      }
      constexpr int NG = CH / G;
      T n0[2][G], n1[2][G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        n0[(NG - 1) & 1][k] = in0[(NG - 1) * G + k];
        n1[(NG - 1) & 1][k] = in1[(NG - 1) * G + k];
      }
      T xa0 = (T)0, xa1 = (T)0;
      static_for<0, NG>([&](auto gc) {
        constexpr int g = NG - 1 - decltype(gc)::value;
        if (g > 0) {
#pragma unroll
          for (int k = 0; k < G; ++k) {
            n0[(g - 1) & 1][k] = in0[(g - 1) * G + k];
            n1[(g - 1) & 1][k] = in1[(g - 1) * G + k];
          }
        }
        static_for<0, G>([&](auto kc) {
          constexpr int k = G - 1 - decltype(kc)::value;
          constexpr int t = g * G + k;
          constexpr int q = CH - 1 - t;
          if constexpr (q % SU == 0) {
            const int vk = UPC * (nch - 1 - c) + q / SU + 1 + K;
            constexpr int rs = (q / SU + 1) % K;
            header(r[rs]);
#ifdef STAU_CHECK_BOUNDS
            {
              const int vi = UPC * (nch - 1 - c) + q / SU + 1;
              const int ui = vi < nu ? nu - 1 - vi : 0;
              int cntb = 0;
              for (int i = 0; i < kSpU; ++i) cntb += __builtin_popcountll(mb[i]);
              STAU_BOUND(a.check, 64 + 8 * cntb <= record_bytes(lensB, ui), kChkRank);
            }
#endif
            r[rs].store(st + ((q / SU + 1) & 1) * SB, lane);
            load_unit(rs, vk);
            la = 0;
          }
          constexpr uint64_t msj = 1ull << t;
          const T u = rg[q % R];
          constexpr int qn = q + R;
          rg[q % R] = entry((qn / SU) & 1, SU - 1 - qn % SU);
          const T x0 = readlane_t(w0 * u, t), x1 = readlane_t(w1 * u, t);
          put_lane<t>(xa0, x0);
          put_lane<t>(xa1, x1);
          const bool inw = __builtin_amdgcn_inverse_ballot_w64(msj);
          w0 = inw ? n0[g & 1][k] : fma(-u, x0, w0);
          w1 = inw ? n1[g & 1][k] : fma(-u, x1, w1);
        });
      });
      // X = P^R x~ for the chunk's columns j0 + lane
      {
        const int sl2 = (lane + S2) & (kWave - 1);
        const bool here = lane + S2 < kWave;
        const T a0 = __shfl(xa0, sl2), b0 = __shfl(xp0, sl2);
        const T a1 = __shfl(xa1, sl2), b1 = __shfl(xp1, sl2);
        const int col = j0 + lane;
        if (col < n) {
          const int m = col / S, pos = col - m * S;
          double v0 = xa0, v1 = xa1;
          if (m + 2 < N) {
            v0 -= here ? a0 : b0;
            v1 -= here ? a1 : b1;
          }
          const int var = d.var_at[pos];
          const double2 xv = (var == VU || var == VUZ || var == VV || var == VVZ) ? make_double2(v1, -v0)
                                                                                  : make_double2(v0, v1);
          X[((size_t)p * S + d.abi_index[var]) * N + m] = xv;
        }
      }
      xp0 = xa0;
      xp1 = xa1;
      double* nx = ring + (bsel ^ 1) * 2 * kWave;
      nx[lane] = q0;
      nx[kWave + lane] = q1;
    }
  }
}

// ---------------------------------------------------------------------------
// Refined mixed-precision solve: FP32 sweeps on FP32 copies of the FP64
// factors, the FP64 residual r = b - A x^ of the first solution (A applied
// from the operator templates, every row including the boundary rows; b
// re-read from Bev in FP64), one FP32 correction sweep, and x = x^ + d summed
// in FP64 when the state is written.  Per wavefront (one real part) in LDS:
// the FP32 sweep vector w (padded, span) and x^ (n).  STG: 0 unstaged sweeps,
// 2 both sweeps staged in su3<float>() column units (launches with more
// blocks than compute units).
// ---------------------------------------------------------------------------
// Entry of the real-scaled right-hand side at row r (as build_rhs writes it)
__device__ __forceinline__ double rhs_entry(const PencilArgs& a, const PencilCoef& pc,
                                            const double2* __restrict__ Bp, int part, int r) {
  const SysDesc& d = a.desc;
  if (r < d.kb) {
    if (part == 0 && pc.mean && d.bc_var[r] == VB) return d.bc_side[r] == 0 ? a.b_bottom : a.b_top;
    return 0.0;
  }
  const int q = r - d.kb, mo = q / d.S;
  const int eq = d.eq_at[q - mo * d.S];
  if (mo >= d.N - 1) return 0.0;
  int e = -1;
  if (eq == EB) e = 0;
  else if (eq == EU) e = 1;
  else if (eq == EV) e = 2;
  else if (eq == EW) e = d.ne - 1;
  if (e < 0) return 0.0;
  const double2 v = Bp[e * d.N + mo];
  const bool scaled = eq == EU || eq == EV;  // rows scaled by i
  return part == 0 ? (scaled ? -v.y : v.x) : (scaled ? v.x : v.y);
}

template <int FW, int BW, int STG>
__global__ void __launch_bounds__(4 * kWave) solve_refined_kernel(PencilArgs a, int plaunch,
                                                                  const double2* __restrict__ Bev,
                                                                  const float* __restrict__ Lf,
                                                                  const uint8_t* __restrict__ sl,
                                                                  const float* __restrict__ Uf,
                                                                  double2* __restrict__ X) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = wv >> 1, part = wv & 1;
  const int p = blockIdx.x * 2 + q;
  const SysDesc& d = a.desc;
  const int n = a.n, N = d.N, S = d.S, ne = d.ne;
  if (blockIdx.x == 0 && plaunch < a.P) zero_pencils(X, plaunch, a.P, S * N, tid, 4 * kWave);
  const bool live = p < plaunch;
  const bool act = live && pencil_active(a, p);
  const int npad = a.nst, nch = npad / kCH;
  const int span = BW + npad + FW;
  const int per = (span + n + 3) / 4 * 4;  // floats per wavefront, 16-byte multiple
  float* base = (float*)lds + (size_t)wv * per;
  float* w = base + BW;          // sweep vector, rows -BW .. npad + FW
  float* xh = base + span;       // first solution x^
  float* stg = (float*)lds + (size_t)4 * per + (size_t)wv * (stage_bytes<float, FW, BW, su3<float>()>() / 4);
  if (act) {
    const PencilCoef pc = pencil_coef(a, p, 0.0, 0.0);
    const double2* Bp = Bev + (size_t)p * ne * N;
    const float* Lp = Lf + (size_t)p * npad * FW;
    const uint32_t* swp = (const uint32_t*)(sl + (size_t)p * npad);
    const float* Up = Uf + (size_t)p * npad * BW;
    auto sweep = [&]() {
      if constexpr (STG == 2)
        sweeps_staged_both<float, FW, BW>(w, Lp, swp, Up, nch, lane, stg);
      else
        sweeps<float, FW, BW>(w, Lp, swp, Up, nch, lane);
    };
    build_rhs<float>(a, pc, Bp, part, w, nullptr, BW, FW, npad, lane);
    sweep();
    for (int r = lane; r < n; r += kWave) xh[r] = w[r];
    // FP64 residual of x^ (every row of the system), rounded to FP32
    const PencilCoef pa = pencil_coef(a, p, a.refine_a0, a.refine_b0);
    for (int r = lane - BW; r < npad + FW; r += kWave) {
      float v = 0.0f;
      if (r >= 0 && r < n) {
        const double ax =
            apply_row(d, pa, r, [&](int m, int var) { return (double)xh[m * S + d.var_pos[var]]; });
        v = (float)(rhs_entry(a, pc, Bp, part, r) - ax);
      }
      w[r] = v;
    }
    sweep();
  }
  __syncthreads();
  if (act) {
    // X = P^R (x^ + d) with the real scaling undone, summed in FP64
    const float* hr = (const float*)lds + (size_t)(2 * q) * per + span;
    const float* hi = (const float*)lds + (size_t)(2 * q + 1) * per + span;
    const float* dr = (const float*)lds + (size_t)(2 * q) * per + BW;
    const float* di = (const float*)lds + (size_t)(2 * q + 1) * per + BW;
    double2* Xp = X + (size_t)p * S * N;
    for (int i = tid & (2 * kWave - 1); i < S * N; i += 2 * kWave) {
      const int vabi = i / N, m = i - vabi * N;
      const int var = a.var_of_abi[vabi];
      const int c = m * S + d.var_pos[var];
      double xr = (double)hr[c] + (double)dr[c], xi = (double)hi[c] + (double)di[c];
      if (m + 2 < N) {
        xr -= (double)hr[c + 2 * S] + (double)dr[c + 2 * S];
        xi -= (double)hi[c + 2 * S] + (double)di[c + 2 * S];
      }
      if (var == VU || var == VUZ || var == VV || var == VVZ)
        Xp[i] = make_double2(xi, -xr);  // u = -i u~
      else
        Xp[i] = make_double2(xr, xi);
    }
  } else if (live) {
    zero_pencils(X, p, p + 1, S * N, tid & (2 * kWave - 1), 2 * kWave);
  }
}

__global__ void round_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                    size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ---------------------------------------------------------------------------
// Transposed solve (adjoint of solve_kernel): B_bar = S_L^H A~^{-T} S_R^H
// (P^R)^T X_bar, where A~ is the real-scaled recombined matrix, S_R the
// column scaling (u = -i u~) and S_L the row scaling (u rows times i).  A~^T
// has its own banded LU with partial pivoting (factor_kernel with a.trans),
// so A~^{-T} is the same pair of sweeps as the forward solve, on the
// transposed factors.
// Epilogue (per pencil): the multistep history adjoints,
//   F~_bar = c1 B_bar + hF,  MX_bar = -a1 B_bar + hM,  hF <- c2 B_bar,
//   hM <- -a2 B_bar,  F_bar = (P^L)^T F~_bar,  X_bar_out = (P^L)^T MX_bar on
//   the evolved variables, zero elsewhere.
// ---------------------------------------------------------------------------
// Entry c (system column order, 0 <= c < n) of the transposed solve's
// right-hand side x~_bar = S_R^H (P^R)^T X_bar, real part (part 0) or
// imaginary part (part 1).
__device__ __forceinline__ double solveT_col(const SysDesc& d, const double2* Xp, int c,
                                            int part) {
  const int N = d.N, S = d.S;
  const int m = c / S, pos = c - m * S;
  const int var = d.var_at[pos];
  const int vabi = d.abi_index[var];
  double2 v = Xp[(size_t)vabi * N + m];
  if (m >= 2) {
    const double2 w2 = Xp[(size_t)vabi * N + m - 2];
    v.x -= w2.x;
    v.y -= w2.y;
  }
  if (var == VU || var == VUZ || var == VV || var == VVZ) return part == 0 ? -v.y : v.x;  // i v
  return part == 0 ? v.x : v.y;
}

// Right-hand side of the transposed solve for one real part, written to
// b[-BW .. npad + FW) (zero outside the n columns).
__device__ __forceinline__ void solveT_rhs(const PencilArgs& a, const double2* Xp,
                                           int part, double* b, int BW, int FW, int npad, int lane) {
  for (int c = lane - BW; c < npad + FW; c += kWave)
    b[c] = (c >= 0 && c < a.n) ? solveT_col(a.desc, Xp, c, part) : 0.0;
}

// Epilogue of the transposed solve (per pencil, all threads of the block):
// history adjoints, (P^L)^T, state-layout outputs, from the solution's real
// and imaginary parts bre / bim (system order).
// sol(row) returns the solution's (real, imaginary) parts at system row `row`.
template <typename SOL>
__device__ __forceinline__ void solveT_epilogue_g(const PencilArgs& a, const AdjRhsArgs& r, SOL sol,
                                                  double2* Xo, double2* Fb, double2* hb, int tid,
                                                  int nt) {
  const SysDesc& d = a.desc;
  const int N = d.N, S = d.S, kb = d.kb, ne = d.ne;
  auto bbar = [&](int e, int m) -> double2 {
    if (m < 0 || m > N - 2) return make_double2(0.0, 0.0);
    const int eq = e == 0 ? EB : (e == ne - 1 ? EW : (e == 1 ? EU : EV));
    const int row = kb + m * S + d.eq_pos[eq];
    const double2 rv = sol(row);
    const double vr = rv.x, vi = rv.y;
    if (eq == EU || eq == EV) return make_double2(vi, -vr);  // -i v
    return make_double2(vr, vi);
  };
  for (int i = tid; i < ne * N; i += nt) {
    const int e = i / N, m = i - e * N;
    const size_t hF = ((size_t)0 * ne + e) * N, hM = ((size_t)1 * ne + e) * N;
    auto ft = [&](int q) -> double2 {  // F~_bar_q
      if (q < 0 || q > N - 2) return make_double2(0.0, 0.0);
      const double2 bb = bbar(e, q), h = hb[hF + q];
      return make_double2(r.c1 * bb.x + h.x, r.c1 * bb.y + h.y);
    };
    auto mx = [&](int q) -> double2 {  // MX_bar_q
      if (q < 0 || q > N - 2) return make_double2(0.0, 0.0);
      const double2 bb = bbar(e, q), h = hb[hM + q];
      return make_double2(-r.a1 * bb.x + h.x, -r.a1 * bb.y + h.y);
    };
    const double cm = m == 0 ? 1.0 : 0.5;
    const double2 f0 = ft(m), f2 = ft(m - 2), x0 = mx(m), x2 = mx(m - 2);
    Fb[(size_t)e * N + m] = make_double2(cm * f0.x - 0.5 * f2.x, cm * f0.y - 0.5 * f2.y);
    Xo[(size_t)(e + 1) * N + m] = make_double2(cm * x0.x - 0.5 * x2.x, cm * x0.y - 0.5 * x2.y);
  }
  for (int i = tid; i < S * N; i += nt) {
    const int v = i / N;
    if (v == 0 || v > ne) Xo[i] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int i = tid; i < ne * N; i += nt) {
    const int e = i / N, m = i - e * N;
    const double2 bb = bbar(e, m);
    hb[((size_t)0 * ne + e) * N + m] = make_double2(r.c2 * bb.x, r.c2 * bb.y);
    hb[((size_t)1 * ne + e) * N + m] = make_double2(-r.a2 * bb.x, -r.a2 * bb.y);
  }
}

__device__ __forceinline__ void solveT_epilogue(const PencilArgs& a, const AdjRhsArgs& r,
                                                const double* bre, const double* bim,
                                                double2* __restrict__ Xo, double2* __restrict__ Fb,
                                                double2* __restrict__ hb, int tid, int nt) {
  solveT_epilogue_g(a, r, [&](int row) { return make_double2(bre[row], bim[row]); }, Xo, Fb, hb, tid,
                    nt);
}

// zero outputs of an inactive pencil in the transposed solve
__device__ __forceinline__ void solveT_zero(const PencilArgs& a, double2* __restrict__ Xo,
                                            double2* __restrict__ Fb, double2* __restrict__ hb,
                                            int tid, int nt) {
  const int N = a.desc.N, S = a.desc.S, ne = a.desc.ne;
  for (int i = tid; i < S * N; i += nt) Xo[i] = make_double2(0.0, 0.0);
  for (int i = tid; i < ne * N; i += nt) Fb[i] = make_double2(0.0, 0.0);
  for (int i = tid; i < 2 * ne * N; i += nt) hb[i] = make_double2(0.0, 0.0);
}

constexpr int kSU2 = 16;  // staging unit of the two-block solve (two blocks per compute unit)

// LDS doubles of a pencil's coupling data (Rinv, E1, E2), rounded to 16 bytes
__host__ __device__ inline int solve2_coupling_doubles(int K, int Q) { return (K * K + Q * K + 1) / 2 * 2; }

// Two-block solve: one pencil per block of four wavefronts, wave 2 half + part
// (half 0: leading block, 1: trailing block; part: real / imaginary).
// TRANS: the adjoint's transposed solve on the two-block factors of A~^T
// (t, bt with trans set): right-hand side from X_bar (XinT), the transposed
// solve's epilogue with r, X_bar written to XoutT (the same array: these two
// are not restrict-qualified; Bev and X are unused).
template <int FWT, int BWT, int FWB, int BWB, bool TRANS>
__global__ void __launch_bounds__(4 * kWave) solve2_kernel(
    PencilArgs t, PencilArgs bt, int plaunch, const double2* __restrict__ Bev,
    const double* __restrict__ Lft, const uint8_t* __restrict__ slt, const double* __restrict__ Uft,
    const double* __restrict__ Lfb, const uint8_t* __restrict__ slb, const double* __restrict__ Ufb,
    const double* __restrict__ Rinv, const double* __restrict__ E1, const double* __restrict__ E2,
    double2* __restrict__ X, const double2* XinT, double2* XoutT, AdjRhsArgs r) {
  extern __shared__ double lds[];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int part = wv & 1, half = wv >> 1;
  const SysDesc& d = t.desc;
  const int N = d.N, S = d.S, ne = d.ne, kb = d.kb;
  const int n = t.nfull, m = t.n, nb = bt.n, kl = t.kl, ku = t.ku, Q = t.Q, K = kl + ku;
  if constexpr (TRANS) {
    if (blockIdx.x == 0)
      for (int q = plaunch; q < t.P; ++q)
        solveT_zero(t, XoutT + (size_t)q * S * N, r.Fbar + (size_t)q * ne * N,
                    r.hbar + (size_t)q * 2 * ne * N, tid, 4 * kWave);
  } else {
    if (blockIdx.x == 0 && plaunch < t.P) zero_pencils(X, plaunch, t.P, S * N, tid, 4 * kWave);
  }
  double2* Xp = (TRANS ? XoutT : X) + (size_t)p * S * N;
  if (!pencil_active(t, p)) {
    if constexpr (TRANS)
      solveT_zero(t, Xp, r.Fbar + (size_t)p * ne * N, r.hbar + (size_t)p * 2 * ne * N, tid, 4 * kWave);
    else
      zero_pencils(X, p, p + 1, S * N, tid, 4 * kWave);
    return;
  }
  const PencilCoef pc = pencil_coef(t, p, 0.0, 0.0);
  const int spanT = BWT + t.nst + FWT, spanB = BWB + bt.nst + FWB;
  double* vt0 = lds + BWT;
  double* vt1 = vt0 + spanT;
  double* vb0 = lds + 2 * spanT + BWB;
  double* vb1 = vb0 + spanB;
  double* z = lds + 2 * spanT + 2 * spanB;  // [2][K]
  double* cR = z + 2 * 64;                  // coupling data: Rinv [K][K], E1 [Q][ku], E2 [Q][kl]
  double* cE1 = cR + K * K;
  double* cE2 = cE1 + Q * ku;
  constexpr int SB = stage_bytes<double, (FWT > FWB ? FWT : FWB), (BWT > BWB ? BWT : BWB), kSU2>() / 8;
  double* stg = cR + solve2_coupling_doubles(K, Q) + (size_t)wv * SB;
  double* v = half == 0 ? (part == 0 ? vt0 : vt1) : (part == 0 ? vb0 : vb1);
  // the pencil's coupling data, loaded now and stored to LDS after the
  // forward sweeps (needed only then)
  constexpr int kCpl = 8;  // coupling doubles per thread (K K + Q (kl + ku) <= 8 * 256)
  double cpl[kCpl];
  {
    const int nR = K * K, nE1 = Q * ku, nE2 = Q * kl;
#pragma unroll
    for (int u = 0; u < kCpl; ++u) {
      const int i = tid + u * 4 * kWave;
      cpl[u] = 0.0;
      if (i < nR) cpl[u] = Rinv[(size_t)p * nR + i];
      else if (i < nR + nE1) cpl[u] = E1[(size_t)p * nE1 + i - nR];
      else if (i < nR + nE1 + nE2) cpl[u] = E2[(size_t)p * nE2 + i - nR - nE1];
    }
  }
  // right-hand side: zero fill (boundary values in the leading block), then
  // the evolved entries scattered to their rows (whole row R: leading block R,
  // trailing block n - 1 - R).  TRANS: x~_bar by whole column (leading block
  // c, trailing block n - 1 - c).
  if constexpr (TRANS) {
    const int BWx = half == 0 ? BWT : BWB, FWx = half == 0 ? FWT : FWB;
    const int npad = half == 0 ? t.nst : bt.nst, nloc = half == 0 ? m : nb;
    const double2* Xs = XinT + (size_t)p * S * N;
    for (int c = lane - BWx; c < npad + FWx; c += kWave)
      v[c] = (c >= 0 && c < nloc) ? solveT_col(d, Xs, half == 0 ? c : n - 1 - c, part) : 0.0;
  } else {
    const int BWx = half == 0 ? BWT : BWB, FWx = half == 0 ? FWT : FWB;
    const int npad = half == 0 ? t.nst : bt.nst;
    for (int r = lane - BWx; r < npad + FWx; r += kWave) {
      double val = 0.0;
      if (half == 0 && part == 0 && r >= 0 && r < kb && pc.mean && d.bc_var[r] == VB)
        val = d.bc_side[r] == 0 ? t.b_bottom : t.b_top;
      v[r] = val;
    }
    const double2* Bp = Bev + (size_t)p * ne * N;
    // modes whose rows can fall in this half (row kb + mo S + pos, pos < S)
    const int mcut = (m - kb) / S;
    const int mlo = half == 0 ? 0 : (mcut > 0 ? mcut - 1 : 0);
    const int mhi = half == 0 ? (mcut + 1 < N - 1 ? mcut + 1 : N - 1) : N - 1;
    const int Nm = mhi - mlo;
    // groups of kRG entries per lane: all loads of a group in flight together
    constexpr int kRG = 8;
    for (int i0 = lane; i0 < ne * Nm; i0 += kRG * kWave) {
      double2 b2[kRG];
      int dst[kRG];
#pragma unroll
      for (int u = 0; u < kRG; ++u) {
        const int i = i0 + u * kWave;
        dst[u] = -1;
        b2[u] = make_double2(0.0, 0.0);
        if (i < ne * Nm) {
          const int e = i / Nm, mo = mlo + (i - e * Nm);
          const int eq = e == 0 ? EB : (e == ne - 1 ? EW : (e == 1 ? EU : EV));
          const int Rw = kb + mo * S + d.eq_pos[eq];
          if ((half == 0) == (Rw < m)) {
            b2[u] = Bp[e * N + mo];
            // rows scaled by i (u, v equations) take (-Im, Re)
            dst[u] = (half == 0 ? Rw : n - 1 - Rw) * 2 + ((eq == EU || eq == EV) ? 1 : 0);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kRG; ++u) {
        if (dst[u] < 0) continue;
        const bool scaled = dst[u] & 1;
        v[dst[u] >> 1] = part == 0 ? (scaled ? -b2[u].y : b2[u].x) : (scaled ? b2[u].x : b2[u].y);
      }
    }
  }
  // blocks p and p + gridDim / 2 share a compute unit (two per unit)
  const int psel = p >= (int)(gridDim.x / 2) ? 1 : 0;
  if (half == 0)
    sweep_forward_staged<double, FWT, kSU2>(v, Lft + (size_t)p * t.nst * FWT,
                                            (const uint32_t*)(slt + (size_t)p * t.nst), t.nst / kCH,
                                            lane, stg, psel);
  else
    sweep_forward_staged<double, FWB, kSU2>(v, Lfb + (size_t)p * bt.nst * FWB,
                                            (const uint32_t*)(slb + (size_t)p * bt.nst), bt.nst / kCH,
                                            lane, stg, psel);
  __builtin_amdgcn_s_setprio(0);
  // the coupling data, loaded at the start, reach LDS only now (their loads
  // completed during the sweep instead of delaying it)
#pragma unroll
  for (int u = 0; u < kCpl; ++u) {
    const int i = tid + u * 4 * kWave;
    if (i < solve2_coupling_doubles(K, Q)) cR[i] = cpl[u];
  }
  __syncthreads();
  if (half == 0 && lane < K) {
    // interface system of this part: z = Rinv [g1b; g2b]
    const double* Rp = cR + lane * K;
    const double* g1 = part == 0 ? vt0 : vt1;
    const double* g2 = part == 0 ? vb0 : vb1;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc = fma(Rp[k], k < kl ? g1[m - kl + k] : g2[nb - ku + (k - kl)], acc);
    z[part * 64 + lane] = acc;
  }
  __syncthreads();
  if (lane < Q) {
    if (half == 0) {
      // g1[m - Q + i] -= sum_k E1[i][k] x2t[k],  x2t[k] = yb[ku - 1 - k]
      const double* Ep = cE1 + lane * ku;
      double acc = 0.0;
      for (int k = 0; k < ku; ++k) acc = fma(Ep[k], z[part * 64 + kl + ku - 1 - k], acc);
      v[m - Q + lane] -= acc;
    } else {
      const double* Ep = cE2 + lane * kl;
      double acc = 0.0;
      for (int k = 0; k < kl; ++k) acc = fma(Ep[k], z[part * 64 + k], acc);
      v[nb - Q + lane] -= acc;
    }
  }
  if (half == 0)
    sweep_backward_staged<double, BWT, kSU2>(v, Uft + (size_t)p * t.nst * BWT, t.nst / kCH, lane, stg);
  else
    sweep_backward_staged<double, BWB, kSU2>(v, Ufb + (size_t)p * bt.nst * BWB, bt.nst / kCH, lane, stg);
  __syncthreads();
  if constexpr (TRANS) {
    // solution row c: leading block for c < m, else the reversed trailing block
    solveT_epilogue_g(
        t, r,
        [&](int c) {
          return c < m ? make_double2(vt0[c], vt1[c]) : make_double2(vb0[n - 1 - c], vb1[n - 1 - c]);
        },
        Xp, r.Fbar + (size_t)p * ne * N, r.hbar + (size_t)p * 2 * ne * N, tid, 4 * kWave);
    return;
  }
  // X = P^R x~ (x~ row c: leading block for c < m, else the reversed trailing block)
  for (int i = tid; i < S * N; i += 4 * kWave) {
    const int vabi = i / N, mo = i - vabi * N;
    const int var = t.var_of_abi[vabi];
    const int pos = d.var_pos[var];
    auto xt = [&](int pp, int c) -> double {
      return c < m ? (pp == 0 ? vt0 : vt1)[c] : (pp == 0 ? vb0 : vb1)[n - 1 - c];
    };
    const int c0 = mo * S + pos;
    double xr = xt(0, c0), xi = xt(1, c0);
    if (mo + 2 < N) {
      xr -= xt(0, c0 + 2 * S);
      xi -= xt(1, c0 + 2 * S);
    }
    if (var == VU || var == VUZ || var == VV || var == VVZ)
      Xp[i] = make_double2(xi, -xr);  // u = -i u~
    else
      Xp[i] = make_double2(xr, xi);
  }
}

// ---------------------------------------------------------------------------
// Two-block refined mixed-precision solve: the two-block solve of
// solve2_kernel with FP32 sweeps on FP32 copies of the block factors (the
// interface system and the corrections in FP64 from the FP64 coupling data),
// then the FP64 residual r = b - A x^ of the whole system from the operator
// templates, a second FP32 two-block pass on r, and X = P^R (x^ + d) summed in
// FP64.  LDS: the interface unknowns and coupling data (double), the four
// FP32 block vectors, x^ in whole-system order ([2][n] FP32) and the FP32
// staging units.
// ---------------------------------------------------------------------------
template <int FWT, int BWT, int FWB, int BWB>
__global__ void __launch_bounds__(4 * kWave) solve2_refined_kernel(
    PencilArgs t, PencilArgs bt, int plaunch, const double2* __restrict__ Bev,
    const float* __restrict__ Lft, const uint8_t* __restrict__ slt, const float* __restrict__ Uft,
    const float* __restrict__ Lfb, const uint8_t* __restrict__ slb, const float* __restrict__ Ufb,
    const double* __restrict__ Rinv, const double* __restrict__ E1, const double* __restrict__ E2,
    double2* __restrict__ X) {
  extern __shared__ double lds[];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int part = wv & 1, half = wv >> 1;
  const SysDesc& d = t.desc;
  const int N = d.N, S = d.S, ne = d.ne, kb = d.kb;
  const int n = t.nfull, m = t.n, nb = bt.n, kl = t.kl, ku = t.ku, Q = t.Q, K = kl + ku;
  if (blockIdx.x == 0 && plaunch < t.P) zero_pencils(X, plaunch, t.P, S * N, tid, 4 * kWave);
  double2* Xp = X + (size_t)p * S * N;
  if (!pencil_active(t, p)) {
    zero_pencils(X, p, p + 1, S * N, tid, 4 * kWave);
    return;
  }
  const PencilCoef pc = pencil_coef(t, p, 0.0, 0.0);
  const PencilCoef pa = pencil_coef(t, p, t.refine_a0, t.refine_b0);
  const int spanT = BWT + t.nst + FWT, spanB = BWB + bt.nst + FWB;
  double* z = lds;         // [2][64] interface unknowns
  double* cR = z + 2 * 64;  // Rinv [K][K], E1 [Q][ku], E2 [Q][kl]
  double* cE1 = cR + K * K;
  double* cE2 = cE1 + Q * ku;
  float* fb = (float*)(cR + solve2_coupling_doubles(K, Q));
  float* vt0 = fb + BWT;
  float* vt1 = vt0 + spanT;
  float* vb0 = fb + 2 * spanT + BWB;
  float* vb1 = vb0 + spanB;
  float* xh = fb + 2 * spanT + 2 * spanB;  // [2][n]
  constexpr int SB = stage_bytes<float, (FWT > FWB ? FWT : FWB), (BWT > BWB ? BWT : BWB), kSU2>() / 4;
  float* stg = xh + (2 * n + 3) / 4 * 4 + (size_t)wv * SB;
  float* v = half == 0 ? (part == 0 ? vt0 : vt1) : (part == 0 ? vb0 : vb1);
  {
    const int nR = K * K, nE1 = Q * ku, nE2 = Q * kl;
    for (int i = tid; i < nR + nE1 + nE2; i += 4 * kWave)
      cR[i] = i < nR ? Rinv[(size_t)p * nR + i]
                     : (i < nR + nE1 ? E1[(size_t)p * nE1 + i - nR] : E2[(size_t)p * nE2 + i - nR - nE1]);
  }
  const double2* Bp = Bev + (size_t)p * ne * N;
  {
    // right-hand side (FP32): zero fill with the boundary values, then the
    // evolved entries (whole row R: leading block R, trailing block n - 1 - R)
    const int BWx = half == 0 ? BWT : BWB, FWx = half == 0 ? FWT : FWB;
    const int npad = half == 0 ? t.nst : bt.nst;
    for (int r = lane - BWx; r < npad + FWx; r += kWave) {
      double val = 0.0;
      if (half == 0 && part == 0 && r >= 0 && r < kb && pc.mean && d.bc_var[r] == VB)
        val = d.bc_side[r] == 0 ? t.b_bottom : t.b_top;
      v[r] = (float)val;
    }
    const int Nm = N - 1;
    for (int i = lane; i < ne * Nm; i += kWave) {
      const int e = i / Nm, mo = i - e * Nm;
      const int eq = e == 0 ? EB : (e == ne - 1 ? EW : (e == 1 ? EU : EV));
      const int Rw = kb + mo * S + d.eq_pos[eq];
      if ((half == 0) != (Rw < m)) continue;
      const double2 b2 = Bp[e * N + mo];
      const bool scaled = eq == EU || eq == EV;
      v[half == 0 ? Rw : n - 1 - Rw] = (float)(part == 0 ? (scaled ? -b2.y : b2.x) : (scaled ? b2.x : b2.y));
    }
  }
  const int psel = p >= (int)(gridDim.x / 2) ? 1 : 0;
  auto pass = [&]() {
    if (half == 0)
      sweep_forward_staged<float, FWT, kSU2>(v, Lft + (size_t)p * t.nst * FWT,
                                             (const uint32_t*)(slt + (size_t)p * t.nst), t.nst / kCH,
                                             lane, stg, psel);
    else
      sweep_forward_staged<float, FWB, kSU2>(v, Lfb + (size_t)p * bt.nst * FWB,
                                             (const uint32_t*)(slb + (size_t)p * bt.nst), bt.nst / kCH,
                                             lane, stg, psel);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    if (half == 0 && lane < K) {
      const double* Rp = cR + lane * K;
      const float* g1 = part == 0 ? vt0 : vt1;
      const float* g2 = part == 0 ? vb0 : vb1;
      double acc = 0.0;
      for (int k = 0; k < K; ++k)
        acc = fma(Rp[k], (double)(k < kl ? g1[m - kl + k] : g2[nb - ku + (k - kl)]), acc);
      z[part * 64 + lane] = acc;
    }
    __syncthreads();
    if (lane < Q) {
      double acc = 0.0;
      if (half == 0) {
        const double* Ep = cE1 + lane * ku;
        for (int k = 0; k < ku; ++k) acc = fma(Ep[k], z[part * 64 + kl + ku - 1 - k], acc);
        v[m - Q + lane] = (float)((double)v[m - Q + lane] - acc);
      } else {
        const double* Ep = cE2 + lane * kl;
        for (int k = 0; k < kl; ++k) acc = fma(Ep[k], z[part * 64 + k], acc);
        v[nb - Q + lane] = (float)((double)v[nb - Q + lane] - acc);
      }
    }
    if (half == 0)
      sweep_backward_staged<float, BWT, kSU2>(v, Uft + (size_t)p * t.nst * BWT, t.nst / kCH, lane, stg);
    else
      sweep_backward_staged<float, BWB, kSU2>(v, Ufb + (size_t)p * bt.nst * BWB, bt.nst / kCH, lane, stg);
    __syncthreads();
  };
  pass();
  // x^ in whole-system order
  for (int c = tid; c < n; c += 4 * kWave) {
    xh[c] = c < m ? vt0[c] : vb0[n - 1 - c];
    xh[n + c] = c < m ? vt1[c] : vb1[n - 1 - c];
  }
  __syncthreads();
  // FP64 residual of x^ into the block vectors (padding zero)
  for (int i = tid; i < 2 * (spanT + spanB); i += 4 * kWave) {
    const int q = i < 2 * spanT ? (i < spanT ? 0 : 1) : ((i - 2 * spanT) < spanB ? 0 : 1);
    const bool lead = i < 2 * spanT;
    const int pos = lead ? (i - q * spanT) - BWT : (i - 2 * spanT - q * spanB) - BWB;
    const int loc = lead ? m : nb;
    float val = 0.0f;
    if (pos >= 0 && pos < loc) {
      const int R = lead ? pos : n - 1 - pos;
      const float* x = xh + (size_t)q * n;
      const double ax = apply_row(d, pa, R, [&](int mo, int var) { return (double)x[mo * S + d.var_pos[var]]; });
      val = (float)(rhs_entry(t, pc, Bp, q, R) - ax);
    }
    (lead ? fb : fb + 2 * spanT)[i - (lead ? 0 : 2 * spanT)] = val;
  }
  __syncthreads();
  pass();
  // X = P^R (x^ + d), real scaling undone
  for (int i = tid; i < S * N; i += 4 * kWave) {
    const int vabi = i / N, mo = i - vabi * N;
    const int var = t.var_of_abi[vabi];
    const int pos = d.var_pos[var];
    auto xt = [&](int pp, int c) -> double {
      const double dd = c < m ? (pp == 0 ? vt0 : vt1)[c] : (pp == 0 ? vb0 : vb1)[n - 1 - c];
      return (double)xh[(size_t)pp * n + c] + dd;
    };
    const int c0 = mo * S + pos;
    double xr = xt(0, c0), xi = xt(1, c0);
    if (mo + 2 < N) {
      xr -= xt(0, c0 + 2 * S);
      xi -= xt(1, c0 + 2 * S);
    }
    if (var == VU || var == VUZ || var == VV || var == VVZ)
      Xp[i] = make_double2(xi, -xr);  // u = -i u~
    else
      Xp[i] = make_double2(xr, xi);
  }
}

// STAGED: both sweeps staged in su3-column units.  Blocks cover pencils
// [0, plaunch); block 0 also zeroes the outputs of the inactive pencils
// [plaunch, P) (in 2-D the Nyquist pencil), so that a launch of plaunch <= #CU
// blocks places at most one block per compute unit.
template <int FW, int BW, bool STAGED>
__global__ void __launch_bounds__(2 * kWave) solveT_kernel(PencilArgs a, int plaunch,
                                                           const double2* Xin,
                                                           const double* __restrict__ Lf,
                                                           const uint8_t* __restrict__ sl,
                                                           const double* __restrict__ Uf,
                                                           double2* Xout, AdjRhsArgs r) {
  extern __shared__ double lds[];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int N = a.desc.N, S = a.desc.S, ne = a.desc.ne;
  if (blockIdx.x == 0)
    for (int q = plaunch; q < a.P; ++q)
      solveT_zero(a, Xout + (size_t)q * S * N, r.Fbar + (size_t)q * ne * N,
                  r.hbar + (size_t)q * 2 * ne * N, tid, 2 * kWave);
  const double2* Xp = Xin + (size_t)p * S * N;
  double2* Xo = Xout + (size_t)p * S * N;
  double2* Fb = r.Fbar + (size_t)p * ne * N;
  double2* hb = r.hbar + (size_t)p * 2 * ne * N;
  if (!pencil_active(a, p)) {
    __syncthreads();
    solveT_zero(a, Xo, Fb, hb, tid, 2 * kWave);
    return;
  }
  const int npad = a.nst, nch = npad / kCH;
  const int span = BW + npad + FW;
  double* bre = lds + BW;
  double* bim = lds + span + BW;
  double* b = wv == 0 ? bre : bim;
  solveT_rhs(a, Xp, wv, b, BW, FW, npad, lane);
  const double* Lp = Lf + (size_t)p * npad * FW;
  const uint32_t* swp = (const uint32_t*)(sl + (size_t)p * npad);
  const double* Up = Uf + (size_t)p * npad * BW;
  if constexpr (STAGED) {
    double* stg = lds + (size_t)2 * span + (size_t)wv * (stage_bytes<double, FW, BW, su3<double>()>() / 8);
    sweeps_staged_both<double, FW, BW>(b, Lp, swp, Up, nch, lane, stg);
  } else {
    sweeps<double, FW, BW>(b, Lp, swp, Up, nch, lane);
  }
  __syncthreads();
  solveT_epilogue(a, r, bre, bim, Xo, Fb, hb, tid, 2 * kWave);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Launch shape of the two-pencil blocks: pencils covered (the leading active
// pencils in 2-D, all in 3-D), block count, and the LDS request.  When the
// blocks fit one per compute unit the request is raised above half of a
// unit's LDS, so that no unit takes two blocks (two sweeping wavefronts on
// one SIMD) while others idle.
// When the blocks fit one per compute unit, the factor columns are staged
// through LDS (stage_lds more bytes per block) if that fits.
struct PencilGrid {
  int plaunch, blocks;
  size_t lds;
  bool staged;
};

static PencilGrid pencil_grid(const PencilArgs& a, size_t lds_per_pencil, size_t stage_lds) {
  PencilGrid g;
  g.plaunch = a.desc.dim == 2 ? a.Px - 1 : a.P;
  g.blocks = (g.plaunch + 1) / 2;
  g.lds = 2 * lds_per_pencil;
  g.staged = false;
  int dev = 0, cus = 0, lds_cu = 0, lds_blk = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      hipDeviceGetAttribute(&lds_blk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
      g.blocks <= cus) {
    const size_t lim = std::min((size_t)lds_cu, (size_t)lds_blk);
    if (g.lds + stage_lds <= lim) {
      g.lds += stage_lds;
      g.staged = true;
    }
    const size_t want = (size_t)lds_cu / 2 + 1024;
    if (g.lds < want && want <= (size_t)lds_blk) g.lds = want;
  }
  return g;
}

template <int FW, int BW>
static hipError_t launch_solve_t(const PencilArgs& a, const void* Bev, const double* Lf,
                                 const uint8_t* sl, const double* Uf, void* X, hipStream_t st) {
  const size_t per_pencil = (size_t)2 * (BW + a.nst + FW) * sizeof(double);
  const PencilGrid g = pencil_grid(a, per_pencil, (size_t)4 * stage_bytes<double, 1, BW, kSU>());
  auto go = [&](auto kern, size_t lds) {
    allow_lds((const void*)kern, lds);
    hipLaunchKernelGGL(kern, dim3(g.blocks), dim3(4 * kWave), lds, st, a, g.plaunch, (const double2*)Bev,
                       Lf, sl, Uf, (double2*)X);
  };
  if (g.staged) {
    go(solve_kernel<FW, BW, 1>, g.lds);
    return hipGetLastError();
  }
  // more blocks than compute units: both sweeps staged in small units when two
  // blocks still fit a unit's LDS
  int dev = 0, cus = 0, lds_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      g.blocks > cus) {
    const size_t lds2 = 2 * per_pencil + (size_t)4 * stage_bytes<double, FW, BW, su3<double>()>();
    const size_t ldsp = 2 * per_pencil + (size_t)2 * stage_bytes<double, FW, BW, su3<double>()>();
    // both real parts per wavefront where three blocks of two pencils fit a
    // unit (256 x 256 x 128: 5.06 -> 4.91 ms; 4096 x 64: 97.5 -> 93.1 us)
    // many pencils per compute unit: vectors streamed through HBM, one pencil
    // per wavefront and about twice the pencils resident (256 x 256 x 128:
    // 4.92 -> 4.44 ms; at 4096 x 64, eight pencils per unit, the pair form
    // is faster: 91.9 against 100.1 us).  Four units of factor loads in
    // flight (eight, or four waves per SIMD with two, measured no faster).
    if (a.ysp && g.plaunch >= 32 * cus) {
      const size_t ldss = (size_t)4 * kWave * sizeof(double) + stage_bytes<double, FW, BW, su3<double>()>();
      hipLaunchKernelGGL((solve_stream_kernel<FW, BW, 4>), dim3(g.plaunch), dim3(kWave), ldss, st, a,
                         g.plaunch, (const double2*)Bev, Lf, sl, Uf, (double2*)X);
      return hipGetLastError();
    }
    if (2 * ldsp <= (size_t)lds_cu) {
      allow_lds((const void*)solve_pair_kernel<FW, BW>, ldsp);
      hipLaunchKernelGGL((solve_pair_kernel<FW, BW>), dim3(g.blocks), dim3(2 * kWave), ldsp, st, a,
                         g.plaunch, (const double2*)Bev, Lf, sl, Uf, (double2*)X);
      return hipGetLastError();
    }
    if (2 * lds2 <= (size_t)lds_cu) {
      go(solve_kernel<FW, BW, 2>, lds2);
      return hipGetLastError();
    }
  }
  go(solve_kernel<FW, BW, 0>, g.lds);
  return hipGetLastError();
}

hipError_t launch_solve(const PencilArgs& a, const void* Bev, const double* Lf, const uint8_t* sl,
                        const double* Uf, void* X, hipStream_t st) {
#define STAU_CASE(F, B) \
  if (a.FW == F && a.BW == B) return launch_solve_t<F, B>(a, Bev, Lf, sl, Uf, X, st);
  STAU_SWEEP_VARIANTS(STAU_CASE)
#undef STAU_CASE
  return hipErrorInvalidValue;
}

// Sparse records where the streamed solve runs: the single-block FP64 solve
// with more than 32 pencils per compute unit, forward windows of at most 16
// rows, at most kSpLen units and backward records of at most three KiB.  (At
// 4096 x 64, eight pencils per unit, the streamed solve on records took
// 110 us against the LDS-resident pair solve's 93 us on the whole band.)
bool sparse_records_apply(const PencilArgs& a, SparseFactors* geom) {
  const int nu = a.nst / kSpU, kv = a.kl + a.ku;
  const int sf = (32 + 64 * a.kl + 15) / 16 * 16, sb = (64 + 64 * (kv + 1) + 15) / 16 * 16;
  int dev = 0, cus = 0;
  if (!a.ysp || a.trans || a.blk != 0 || a.FW > 16 || nu > kSpLen || sb > 3 * 1024 || sf > 1024 ||
      hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  const int plaunch = a.desc.dim == 2 ? a.Px - 1 : a.P;
  if (plaunch < 32 * cus) return false;
  if (geom) {
    geom->strideF = sf;
    geom->strideB = sb;
  }
  return true;
}

hipError_t launch_sparse_records(const PencilArgs& a, const double* Lf, const uint8_t* sl, const double* Uf,
                                 const SparseFactors& sf, hipStream_t st) {
#define STAU_CASE(F, B)                                                                               \
  if (a.FW == F && a.BW == B) {                                                                       \
    hipLaunchKernelGGL((sparse_records_kernel<F, B>), dim3(a.P), dim3(kPackWaves * kWave), 0, st, a, Lf, sl, Uf, sf); \
    return hipGetLastError();                                                                         \
  }
  STAU_SWEEP_VARIANTS(STAU_CASE)
#undef STAU_CASE
  return hipErrorInvalidValue;
}

template <int FW, int NBB>
static hipError_t launch_solve_sparse_t(const PencilArgs& a, const void* Bev, const SparseFactors& sf, void* X,
                                        hipStream_t st) {
  const int plaunch = a.desc.dim == 2 ? a.Px - 1 : a.P;
  const size_t stage = (size_t)2 * (NBB > 1 ? NBB : 1) * 1024;
  const size_t lds = (size_t)4 * kWave * sizeof(double) + stage + 16;
  // two records in flight per direction: 127 VGPRs, four wavefronts per SIMD
  // (four records, 163 VGPRs and three wavefronts, measured 5 % slower at
  // 256 x 256 x 128)
  hipLaunchKernelGGL((solve_sparse_kernel<FW, NBB, 2>), dim3(plaunch), dim3(kWave), lds, st, a, plaunch,
                     (const double2*)Bev, sf, (double2*)X);
  return hipGetLastError();
}

hipError_t launch_solve_sparse(const PencilArgs& a, const void* Bev, const SparseFactors& sf, void* X,
                               hipStream_t st) {
  const int nbb = (sf.strideB + 1023) / 1024;
  if (a.FW == 8) {
    if (nbb == 1) return launch_solve_sparse_t<8, 1>(a, Bev, sf, X, st);
    if (nbb == 2) return launch_solve_sparse_t<8, 2>(a, Bev, sf, X, st);
    if (nbb == 3) return launch_solve_sparse_t<8, 3>(a, Bev, sf, X, st);
  }
  if (a.FW == 16) {
    if (nbb == 1) return launch_solve_sparse_t<16, 1>(a, Bev, sf, X, st);
    if (nbb == 2) return launch_solve_sparse_t<16, 2>(a, Bev, sf, X, st);
    if (nbb == 3) return launch_solve_sparse_t<16, 3>(a, Bev, sf, X, st);
  }
  return hipErrorInvalidValue;
}

template <int FW, int BW>
static hipError_t launch_solve_refined_t(const PencilArgs& a, const void* Bev, const float* Lf,
                                         const uint8_t* sl, const float* Uf, void* X, hipStream_t st) {
  const int span = BW + a.nst + FW;
  const size_t per = (size_t)(span + a.n + 3) / 4 * 4 * sizeof(float);
  const int plaunch = a.desc.dim == 2 ? a.Px - 1 : a.P;
  const int blocks = (plaunch + 1) / 2;
  int dev = 0, cus = 0;
  const bool many = hipGetDevice(&dev) == hipSuccess &&
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                    blocks > cus;
  auto go = [&](auto kern, size_t lds) {
    allow_lds((const void*)kern, lds);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(4 * kWave), lds, st, a, plaunch, (const double2*)Bev,
                       Lf, sl, Uf, (double2*)X);
  };
  if (many)
    go(solve_refined_kernel<FW, BW, 2>, 4 * per + (size_t)4 * stage_bytes<float, FW, BW, su3<float>()>());
  else
    go(solve_refined_kernel<FW, BW, 0>, 4 * per);
  return hipGetLastError();
}

hipError_t launch_solve_refined(const PencilArgs& a, const void* Bev, const float* Lf, const uint8_t* sl,
                                const float* Uf, void* X, hipStream_t st) {
#define STAU_CASE(F, B) \
  if (a.FW == F && a.BW == B) return launch_solve_refined_t<F, B>(a, Bev, Lf, sl, Uf, X, st);
  STAU_SWEEP_VARIANTS(STAU_CASE)
#undef STAU_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_round_f32(const double* src, float* dst, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(round_to_f32_kernel, dim3(1024), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}


template <int FWT, int BWT, int FWB, int BWB, bool TRANS>
static hipError_t launch_solve2_t(const PencilArgs& t, const PencilArgs& bt, const void* Bev,
                                  const double* Lft, const uint8_t* slt, const double* Uft,
                                  const double* Lfb, const uint8_t* slb, const double* Ufb,
                                  const double* Rinv, const double* E1, const double* E2, void* X,
                                  const AdjRhsArgs& r, hipStream_t st) {
  const int plaunch = t.desc.dim == 2 ? t.Px - 1 : t.P;
  constexpr int SB = stage_bytes<double, (FWT > FWB ? FWT : FWB), (BWT > BWB ? BWT : BWB), kSU2>();
  const int K = t.kl + t.ku;
  if (K * K + t.Q * K > 8 * 4 * kWave) return hipErrorInvalidValue;
  const size_t lds = (size_t)(2 * (BWT + t.nst + FWT) + 2 * (BWB + bt.nst + FWB) + 2 * 64 +
                              solve2_coupling_doubles(K, t.Q)) * sizeof(double) + (size_t)4 * SB;
  auto fn = solve2_kernel<FWT, BWT, FWB, BWB, TRANS>;
  allow_lds((const void*)fn, lds);
  if constexpr (TRANS)
    hipLaunchKernelGGL(fn, dim3(plaunch), dim3(4 * kWave), lds, st, t, bt, plaunch, nullptr, Lft, slt,
                       Uft, Lfb, slb, Ufb, Rinv, E1, E2, nullptr, (const double2*)Bev, (double2*)X, r);
  else
    hipLaunchKernelGGL(fn, dim3(plaunch), dim3(4 * kWave), lds, st, t, bt, plaunch, (const double2*)Bev,
                       Lft, slt, Uft, Lfb, slb, Ufb, Rinv, E1, E2, (double2*)X, nullptr, nullptr, r);
  return hipGetLastError();
}

// forward (leading FW 8 or 16) and transposed (leading FW 32, trailing 8) block widths
#define STAU_SOLVE2_VARIANTS(X) X(8, 32, 32, 32) X(16, 32, 32, 32) X(32, 32, 8, 32)

bool solve2_supported(const PencilArgs& t, const PencilArgs& bt) {
#define STAU_CASE2(FT, BT, FB, BB) \
  if (t.FW == FT && t.BW == BT && bt.FW == FB && bt.BW == BB) return true;
  STAU_SOLVE2_VARIANTS(STAU_CASE2)
#undef STAU_CASE2
  return false;
}

hipError_t launch_solve2(const PencilArgs& t, const PencilArgs& bt, const void* Bev,
                         const double* Lft, const uint8_t* slt, const double* Uft,
                         const double* Lfb, const uint8_t* slb, const double* Ufb,
                         const double* Rinv, const double* E1, const double* E2, void* X,
                         hipStream_t st) {
  const AdjRhsArgs none{};
#define STAU_CASE2(FT, BT, FB, BB)                                                                    \
  if (t.FW == FT && t.BW == BT && bt.FW == FB && bt.BW == BB)                                         \
    return launch_solve2_t<FT, BT, FB, BB, false>(t, bt, Bev, Lft, slt, Uft, Lfb, slb, Ufb, Rinv, E1, \
                                                  E2, X, none, st);
  STAU_SOLVE2_VARIANTS(STAU_CASE2)
#undef STAU_CASE2
  return hipErrorInvalidValue;
}

template <int FWT, int BWT, int FWB, int BWB>
static hipError_t launch_solve2_refined_t(const PencilArgs& t, const PencilArgs& bt, const void* Bev,
                                          const float* Lft, const uint8_t* slt, const float* Uft,
                                          const float* Lfb, const uint8_t* slb, const float* Ufb,
                                          const double* Rinv, const double* E1, const double* E2,
                                          void* X, hipStream_t st) {
  const int plaunch = t.Px - 1;
  constexpr int SB = stage_bytes<float, (FWT > FWB ? FWT : FWB), (BWT > BWB ? BWT : BWB), kSU2>();
  const int K = t.kl + t.ku;
  const size_t floats = (size_t)2 * (BWT + t.nst + FWT) + 2 * (BWB + bt.nst + FWB);
  const size_t lds = (size_t)(2 * 64 + solve2_coupling_doubles(K, t.Q)) * sizeof(double) +
                     (floats + (size_t)(2 * t.nfull + 3) / 4 * 4) * sizeof(float) + (size_t)4 * SB;
  auto fn = solve2_refined_kernel<FWT, BWT, FWB, BWB>;
  allow_lds((const void*)fn, lds);
  hipLaunchKernelGGL(fn, dim3(plaunch), dim3(4 * kWave), lds, st, t, bt, plaunch, (const double2*)Bev, Lft,
                     slt, Uft, Lfb, slb, Ufb, Rinv, E1, E2, (double2*)X);
  return hipGetLastError();
}

hipError_t launch_solve2_refined(const PencilArgs& t, const PencilArgs& bt, const void* Bev,
                                 const float* Lft, const uint8_t* slt, const float* Uft,
                                 const float* Lfb, const uint8_t* slb, const float* Ufb,
                                 const double* Rinv, const double* E1, const double* E2, void* X,
                                 hipStream_t st) {
  if (t.trans || t.desc.dim != 2) return hipErrorInvalidValue;
  if (t.FW == 8 && t.BW == 32 && bt.FW == 32 && bt.BW == 32)
    return launch_solve2_refined_t<8, 32, 32, 32>(t, bt, Bev, Lft, slt, Uft, Lfb, slb, Ufb, Rinv, E1, E2, X, st);
  if (t.FW == 16 && t.BW == 32 && bt.FW == 32 && bt.BW == 32)
    return launch_solve2_refined_t<16, 32, 32, 32>(t, bt, Bev, Lft, slt, Uft, Lfb, slb, Ufb, Rinv, E1, E2, X, st);
  return hipErrorInvalidValue;
}

hipError_t launch_solve2T(const PencilArgs& t, const PencilArgs& bt, const void* Xin,
                          const double* Lft, const uint8_t* slt, const double* Uft,
                          const double* Lfb, const uint8_t* slb, const double* Ufb,
                          const double* Rinv, const double* E1, const double* E2, void* Xout,
                          const AdjRhsArgs& r, hipStream_t st) {
  if (!t.trans || !bt.trans) return hipErrorInvalidValue;
  if (t.FW == 32 && t.BW == 32 && bt.FW == 8 && bt.BW == 32)
    return launch_solve2_t<32, 32, 8, 32, true>(t, bt, Xin, Lft, slt, Uft, Lfb, slb, Ufb, Rinv, E1, E2,
                                                Xout, r, st);
  return hipErrorInvalidValue;
}

// One pencil per block of two wavefronts.  More blocks than compute units:
// both sweeps staged (su3 columns) when two blocks fit a unit's LDS (512
// blocks and more share units; 4096x64 adjoint step 432 -> 342 us); up to one
// block per unit: unstaged (staging the backward sweep, or both, measured
// 3-14 us slower at 512x128).
template <int FW, int BW>
static hipError_t launch_solveT_t(const PencilArgs& a, const void* Xin, const double* Lf,
                                  const uint8_t* sl, const double* Uf, void* Xout,
                                  const AdjRhsArgs& r, hipStream_t st) {
  const size_t vec = (size_t)2 * (BW + a.nst + FW) * sizeof(double);
  const int plaunch = a.desc.dim == 2 ? a.Px - 1 : a.P;
  auto go = [&](auto kern, size_t lds) {
    allow_lds((const void*)kern, lds);
    hipLaunchKernelGGL(kern, dim3(plaunch), dim3(2 * kWave), lds, st, a, plaunch,
                       (const double2*)Xin, Lf, sl, Uf, (double2*)Xout, r);
  };
  int dev = 0, cus = 0, lds_cu = 0;
  const size_t lds2 = vec + (size_t)2 * stage_bytes<double, FW, BW, su3<double>()>();
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      plaunch > cus && 2 * lds2 <= (size_t)lds_cu) {
    go(solveT_kernel<FW, BW, true>, lds2);
    return hipGetLastError();
  }
  go(solveT_kernel<FW, BW, false>, vec);
  return hipGetLastError();
}

hipError_t launch_solveT(const PencilArgs& a, const void* Xin, const double* Lf, const uint8_t* sl,
                         const double* Uf, void* Xout, const AdjRhsArgs& r, hipStream_t st) {
#define STAU_CASE(F, B) \
  if (a.FW == F && a.BW == B) return launch_solveT_t<F, B>(a, Xin, Lf, sl, Uf, Xout, r, st);
  STAU_SWEEP_VARIANTS(STAU_CASE)
#undef STAU_CASE
  return hipErrorInvalidValue;
}

}  // namespace stau
