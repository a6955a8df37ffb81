// Device helpers shared by the pencil kernels (factorisation, coupling and
// sweeps): lane reads and writes, compile-time loops, per-pencil
// coefficients and activity, and the sweep geometry constants.
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace stau {

constexpr int kWave = 64;

// Index checks of the check build (STAU_CHECK_BOUNDS): a failed check sets
// its bit in the pencils' check word (read by stau_check); no trap, and
// nothing at all in other builds.
enum CheckBits : unsigned { kChkPivot = 1u, kChkRecord = 2u, kChkSlot = 4u, kChkRank = 8u };
#ifdef STAU_CHECK_BOUNDS
#define STAU_BOUND(word, cond, bit)              \
  do {                                           \
    if (!(cond) && (word)) atomicOr((word), (unsigned)(bit)); \
  } while (0)
#else
#define STAU_BOUND(word, cond, bit) \
  do {                              \
  } while (0)
#endif
constexpr int kCH = 64;  // sweep chunk: columns per unrolled loop body
constexpr int kRing = 32;  // look-ahead of the factor loads in the sweeps (columns)

// Materialise a loaded value in its register here: the loads it depends on
// complete before this point and cannot be sunk past it by the scheduler.
__device__ __forceinline__ void pin(double& x) { asm volatile("" : "+v"(x)); }

__device__ __forceinline__ void pin(float& x) { asm volatile("" : "+v"(x)); }

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_t(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane_t(double v, int lane) { return readlane_d(v, lane); }

// acc[lane L] = v (v uniform, L an immediate): the sweeps collect one result
// per column in a register this way and store a whole chunk at once, so no
// SGPR copy of the result stays live until an LDS store.
template <int L>
__device__ __forceinline__ void put_lane(float& acc, float v) {
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(acc) : "s"(__float_as_int(v)), "i"(L));
}
template <int L>
__device__ __forceinline__ void put_lane(double& acc, double v) {
  int lo = __double2loint(acc), hi = __double2hiint(acc);
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(lo) : "s"(__double2loint(v)), "i"(L));
  asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(hi) : "s"(__double2hiint(v)), "i"(L));
  acc = __hiloint2double(hi, lo);
}

// compile-time loop helper: f(std::integral_constant<int, I>) for I < N
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

__device__ __forceinline__ PencilCoef pencil_coef(const PencilArgs& a, int p, double a0, double b0) {
  PencilCoef pc;
  pc.a0 = a0;
  pc.b0 = b0;
  pc.kappa = a.kappa;
  pc.nu = a.nu;
  pc.buoy = a.buoyancy;
  int ix, iy;
  if (a.desc.dim == 2) {
    ix = p;
    iy = 0;
    pc.ky = 0.0;
  } else {
    iy = p / a.Px;
    ix = p - iy * a.Px;
    int kyi = iy < (a.Ny + 1) / 2 ? iy : iy - a.Ny;
    pc.ky = a.two_pi_over_Ly * (double)kyi;
  }
  pc.kx = a.two_pi_over_Lx * (double)ix;
  pc.mean = (ix == 0 && iy == 0);
  pc.lin = a.lin;
  pc.nncc = a.nncc;
#pragma unroll
  for (int k = 0; k < kMaxNcc; ++k) pc.ncc[k] = a.ncc[k];
  return pc;
}

__device__ __forceinline__ bool pencil_active(const PencilArgs& a, int p) {
  if (a.desc.dim == 2) return p < a.Px - 1;
  int iy = p / a.Px;
  int ix = p - iy * a.Px;
  return ix < a.Px - 1 && iy != a.Ny / 2;
}


}  // namespace stau
