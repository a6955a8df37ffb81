// Helpers shared by the transform kernels: complex loads and stores in FP64
// or FP32 workspaces, wavenumbers and activity of a pencil slot, the z-tile
// geometry and the host-side launch helpers.
#pragma once

#include "common.h"
#include "kernels.h"

namespace stau {

using cd = cpx<double>;

__device__ __forceinline__ cd ld2(const double2* p) {
  double2 v = *p;
  return mk(v.x, v.y);
}
__device__ __forceinline__ void st2(double2* p, cd v) { *p = make_double2(v.x, v.y); }

// storage of complex T in workspaces (double2 / float2)
template <typename T>
struct V2;
template <>
struct V2<double> {
  using type = double2;
};
template <>
struct V2<float> {
  using type = float2;
};
template <typename T>
__device__ __forceinline__ cpx<T> ldv(const typename V2<T>::type* p) {
  auto v = *p;
  return mk<T>(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void stv(typename V2<T>::type* p, cpx<T> v) {
  typename V2<T>::type o;
  o.x = v.x;
  o.y = v.y;
  *p = o;
}
template <typename T>
__device__ __forceinline__ cpx<T> tw_of(const XformArgs& a, const void* t64, const void* t32, int i) {
  if constexpr (sizeof(T) == 8) return ld2((const double2*)t64 + i);
  else {
    const float2 v = ((const float2*)t32)[i];
    return mk<float>(v.x, v.y);
  }
}

__device__ __forceinline__ double kx_of(const XformArgs& a, int p) {
  const int ix = a.dim == 2 ? p : p % a.Px;
  return a.two_pi_over_Lx * (double)ix;
}
__device__ __forceinline__ double ky_of(const XformArgs& a, int p) {
  if (a.dim == 2) return 0.0;
  const int iy = p / a.Px;
  const int kyi = iy < (a.Ny + 1) / 2 ? iy : iy - a.Ny;
  return a.two_pi_over_Ly * (double)kyi;
}
__device__ __forceinline__ bool active(const XformArgs& a, int p) {
  if (p >= a.P) return false;
  if (a.dim == 2) return p < a.Pa;
  const int iy = p / a.Px, ix = p - iy * a.Px;
  return ix < a.Pa && iy != a.Ny / 2;
}

// Pencil p0 + s of a block whose first pencil is p0, without an integer
// division per element: (iy0, ix0) of p0 from one division, then s added to
// ix0 with carries into iy.
struct PencilBase {
  int p0, iy0, ix0;
};
__device__ __forceinline__ PencilBase pencil_base(const XformArgs& a, int p0) {
  PencilBase b{p0, 0, p0};
  if (a.dim == 3) {
    b.iy0 = p0 / a.Px;
    b.ix0 = p0 - b.iy0 * a.Px;
  }
  return b;
}
__device__ __forceinline__ void pencil_xy(const XformArgs& a, const PencilBase& b, int s, int& ix, int& iy) {
  ix = b.ix0 + s;
  iy = b.iy0;
  if (a.dim == 3)
    while (ix >= a.Px) {
      ix -= a.Px;
      ++iy;
    }
}
__device__ __forceinline__ bool active_at(const XformArgs& a, const PencilBase& b, int s) {
  if (b.p0 + s >= a.P) return false;
  if (a.dim == 2) return b.p0 + s < a.Pa;
  int ix, iy;
  pencil_xy(a, b, s, ix, iy);
  return ix < a.Pa && iy != a.Ny / 2;
}
__device__ __forceinline__ double kx_at(const XformArgs& a, const PencilBase& b, int s) {
  int ix, iy;
  pencil_xy(a, b, s, ix, iy);
  return a.two_pi_over_Lx * (double)ix;
}
__device__ __forceinline__ double ky_at(const XformArgs& a, const PencilBase& b, int s) {
  if (a.dim == 2) return 0.0;
  int ix, iy;
  pencil_xy(a, b, s, ix, iy);
  const int kyi = iy < (a.Ny + 1) / 2 ? iy : iy - a.Ny;
  return a.two_pi_over_Ly * (double)kyi;
}

// ---------------------------------------------------------------------------
// z transforms: TP pencils of M points per block of 256 threads, TP * M =
// kZPts (z_tile), so every thread owns exactly kZPts / 256 points of the
// block.  The FFT and DCT twiddle tables (M entries each) are staged in LDS
// behind the data, and each thread issues all of its global loads before it
// uses any, so that their latencies overlap instead of adding up.
// ---------------------------------------------------------------------------
constexpr int kZPts = 3072;
constexpr int kZThreads = 256;
constexpr int kZEpt = kZPts / kZThreads;

template <typename T>
__device__ __forceinline__ void stage_z_tables(const XformArgs& a, cpx<T>* twl, cpx<T>* dcl, int M,
                                               int tid) {
  for (int i = tid; i < M; i += kZThreads) {
    twl[i] = tw_of<T>(a, a.twz, a.twz32, i);
    dcl[i] = tw_of<T>(a, a.dctz, a.dctz32, i);
  }
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
inline void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

inline int z_tile(int M) { return M >= 3072 ? 1 : 3072 / M; }
inline int x_threads(int L) {
  int nt = (L + 5) / 6;
  nt = (nt + 63) / 64 * 64;
  if (nt < 64) nt = 64;
  if (nt > 1024) nt = 1024;
  return nt;
}

// Half-size z tiles (kZPts / 2 points, 6 per thread).  With few blocks per
// compute unit, more and smaller blocks keep every unit busy (1024x256: z
// backward 28.2 -> 24.9 us, z forward 30.8 -> 25.7 us; quarter tiles measured
// no better); with many, the half tile's LDS (30 instead of 55 KB at M = 192)
// holds five blocks per unit instead of two (256x256x128, about 100 blocks
// per unit: z backward 602 -> 454 us, z forward unchanged).  So the step's
// transforms (per_cu = 0) always take them; the adjoint's transforms
// (per_cu > 0) take them when the full-size grid has fewer than per_cu blocks
// per compute unit.  Returns the divisor (1 or 2).
inline int z_split(int blocks, int M, int per_cu = 0) {
  if (M > kZPts / 2) return 1;
  if (per_cu == 0) return 2;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1;
  return blocks < per_cu * cus ? 2 : 1;
}


}  // namespace stau
