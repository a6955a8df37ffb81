// Grid <-> coefficient transforms of selected state variables (Sec. VI "Data
// manipulation": a field's grid data and its coefficient data; Sec. IV
// "Scaled transforms & dealiasing": grids at scale 1 or 3/2), and their
// adjoints.  The z and y stages reuse the step's transform kernels; this file
// holds the x stage on the caller's grid layout and the gathers.
//
// Grid layout (real float64): g[f][ix][l][jz] (2-D: g[f][ix][jz]), with
// ix < Lg = scale Nx, l < scale Ny, jz < Mg = scale Nz on the ascending
// Chebyshev Gauss grid; spectral rows (complex) s[f][jz][l][kx], kx < Px.
//
//   DIR +1 (x synthesis): g = s0 Re c_0 + 2 s1 Re sum_{1 <= k < Pa} c_k e^{2 pi i k ix / Lg}
//   DIR -1 (x analysis):  c_0 = s0 sum_ix g,  c_k = s1 sum_ix g e^{-2 pi i k ix / Lg}  (k < Pa),
//                         c_k = 0 for Pa <= k < Px
//
// The synthesis at s0 = s1 = 1 is the complex-to-real transform of the half
// spectrum (Nyquist and padding zero); the analysis at s0 = s1 = 1 / Lg is the
// truncating forward transform.  Their adjoints under the real inner product
// (complex coefficients as pairs of reals) are the analysis with s0 = 1,
// s1 = 2 and the synthesis with s0 = 1 / Lg, s1 = 1 / (2 Lg).
//
// One block transforms TZ consecutive z levels of one (field, y level): the
// grid values of a fixed ix are TZ contiguous doubles, and two real rows are
// packed into each complex FFT (TZ / 2 sequences of Lg points in LDS).
#include "common.h"
#include "kernels.h"

namespace stau {

namespace {

using cd = cpx<double>;
constexpr int kGThreads = 256;
constexpr int kGMaxBF = 6;          // butterflies per thread per radix-4 pass
constexpr int kGMaxPoints = 6144;   // (TZ / 2) * Lg complex points per block

template <int DIR>
__global__ void __launch_bounds__(kGThreads) xgrid_kernel(XformArgs a, int Lg, int Ngy, int Mg,
                                                          const double2* __restrict__ tw,
                                                          const void* __restrict__ in,
                                                          void* __restrict__ out, double s0,
                                                          double s1, int TZ) {
  extern __shared__ double2 smem[];
  cd* buf = (cd*)smem;
  const int jz0 = blockIdx.x * TZ, l = blockIdx.y, f = blockIdx.z;
  const int Pa = a.Pa, Px = a.Px, tid = threadIdx.x;
  const int half = TZ / 2;
  auto grow = [&](int ix) { return (((size_t)f * Lg + ix) * Ngy + l) * Mg + jz0; };
  auto srow = [&](int t) { return (((size_t)f * Mg + jz0 + t) * Ngy + l) * Px; };
  if constexpr (DIR > 0) {
    const double2* S = (const double2*)in;
    double* g = (double*)out;
    for (int idx = tid; idx < half * Lg; idx += kGThreads) {
      const int s = idx / Lg, k = idx - s * Lg;
      const int kk = k < Pa ? k : (k > Lg - Pa ? Lg - k : -1);
      cd z = mk(0.0, 0.0);
      if (kk >= 0) {
        const double2 A = S[srow(2 * s) + kk], B = S[srow(2 * s + 1) + kk];
        const double w = kk == 0 ? s0 : s1;
        cd Ak = mk(w * A.x, kk == 0 ? 0.0 : w * A.y), Bk = mk(w * B.x, kk == 0 ? 0.0 : w * B.y);
        // rows A, B packed as A + i B: positive frequencies A_k + i B_k,
        // negative ones conj(A_k) + i conj(B_k)
        z = k < Pa ? mk(Ak.x - Bk.y, Ak.y + Bk.x) : mk(Ak.x + Bk.y, Bk.x - Ak.y);
      }
      buf[idx] = z;
    }
    __syncthreads();
    fft_lds<+1, kGMaxBF>(buf, Lg, half, (const cd*)tw, tid, kGThreads);
    for (int idx = tid; idx < TZ * Lg; idx += kGThreads) {
      const int ix = idx / TZ, t = idx - ix * TZ;
      const cd v = buf[(t >> 1) * Lg + ix];
      g[grow(ix) + t] = (t & 1) ? v.y : v.x;
    }
  } else {
    const double* g = (const double*)in;
    double2* S = (double2*)out;
    double* bd = (double*)smem;
    for (int idx = tid; idx < TZ * Lg; idx += kGThreads) {
      const int ix = idx / TZ, t = idx - ix * TZ;
      bd[2 * ((t >> 1) * Lg + ix) + (t & 1)] = g[grow(ix) + t];
    }
    __syncthreads();
    fft_lds<-1, kGMaxBF>(buf, Lg, half, (const cd*)tw, tid, kGThreads);
    for (int idx = tid; idx < TZ * Px; idx += kGThreads) {
      const int t = idx / Px, k = idx - t * Px;
      double2 v = make_double2(0.0, 0.0);
      if (k < Pa) {
        const cd Z = buf[(t >> 1) * Lg + k], Zm = buf[(t >> 1) * Lg + (k == 0 ? 0 : Lg - k)];
        // unpack: A_k = (Z_k + conj Z_{-k}) / 2, B_k = (Z_k - conj Z_{-k}) / (2 i)
        const cd A = mk(0.5 * (Z.x + Zm.x), 0.5 * (Z.y - Zm.y));
        const cd B = mk(0.5 * (Z.y + Zm.y), -0.5 * (Z.x - Zm.x));
        const cd c = (t & 1) ? B : A;
        const double w = k == 0 ? s0 : s1;
        v = make_double2(w * c.x, w * c.y);
      }
      S[srow(t) + k] = v;
    }
  }
}

// F[p][f][n] (nf fields) -> X[p][var_f][n] for every pencil slot
__global__ void put_vars_kernel(int P, int S, int N, FieldList fl, const double2* __restrict__ F,
                                double2* __restrict__ X) {
  const size_t total = (size_t)P * fl.nf * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(i % N);
    const size_t q = i / N;
    const int f = (int)(q % fl.nf);
    const size_t p = q / fl.nf;
    X[(p * S + fl.var[f]) * N + n] = F[i];
  }
}

// zero the variables of fl in X[p][var][n]
__global__ void zero_vars_kernel(int P, int S, int N, FieldList fl, double2* __restrict__ X) {
  const size_t total = (size_t)P * fl.nf * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(i % N);
    const size_t q = i / N;
    const int f = (int)(q % fl.nf);
    const size_t p = q / fl.nf;
    X[(p * S + fl.var[f]) * N + n] = make_double2(0.0, 0.0);
  }
}

int grid_blocks(size_t total) {
  const size_t b = (total + 255) / 256;
  return (int)(b < 8192 ? (b ? b : 1) : 8192);
}

}  // namespace

bool xgrid_supported(int Lg, int Mg) {
  int TZ = 2;
  while (TZ < 16 && Mg % (2 * TZ) == 0 && TZ * Lg <= kGMaxPoints) TZ *= 2;
  return Mg % 2 == 0 && (TZ / 2) * Lg <= kGMaxPoints;
}

hipError_t launch_xgrid(const XformArgs& a, int dir, int nf, int Lg, int Ngy, int Mg,
                        const double2* tw, const void* in, void* out, double s0, double s1,
                        hipStream_t st) {
  if (!xgrid_supported(Lg, Mg)) return hipErrorInvalidValue;
  // the largest power of two TZ <= 16 dividing Mg with (TZ / 2) Lg points in LDS
  int TZ = 2;
  while (TZ < 16 && Mg % (2 * TZ) == 0 && TZ * Lg <= kGMaxPoints) TZ *= 2;
  const size_t lds = (size_t)(TZ / 2) * Lg * sizeof(double2);
  const dim3 grid(Mg / TZ, Ngy, nf);
  const void* fn = dir > 0 ? (const void*)xgrid_kernel<+1> : (const void*)xgrid_kernel<-1>;
  if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (dir > 0)
    hipLaunchKernelGGL(xgrid_kernel<+1>, grid, dim3(kGThreads), lds, st, a, Lg, Ngy, Mg, tw, in, out,
                       s0, s1, TZ);
  else
    hipLaunchKernelGGL(xgrid_kernel<-1>, grid, dim3(kGThreads), lds, st, a, Lg, Ngy, Mg, tw, in, out,
                       s0, s1, TZ);
  return hipGetLastError();
}

hipError_t launch_put_vars(int P, int S, int N, const FieldList& fl, const void* F, void* X,
                           hipStream_t st) {
  hipLaunchKernelGGL(put_vars_kernel, dim3(grid_blocks((size_t)P * fl.nf * N)), dim3(256), 0, st, P,
                     S, N, fl, (const double2*)F, (double2*)X);
  return hipGetLastError();
}

hipError_t launch_zero_vars(int P, int S, int N, const FieldList& fl, void* X, hipStream_t st) {
  hipLaunchKernelGGL(zero_vars_kernel, dim3(grid_blocks((size_t)P * fl.nf * N)), dim3(256), 0, st, P,
                     S, N, fl, (double2*)X);
  return hipGetLastError();
}

}  // namespace stau
