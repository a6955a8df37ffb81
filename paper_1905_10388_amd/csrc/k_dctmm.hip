// Chebyshev z transforms as dense matrix products on the FP64 matrix cores.
//   backward  G_f[j][p] = sum_n Bz[j][n] c_f[p][n],     Bz[j][n] = T_n(z_j)
//   forward   c[p][n]   = sum_j Fz[n][j] h[j][p],       Fz[n][j] = (2 - delta_n0)/M T_n(z_j)
// (z_j the ascending Gauss grid of M = 3N/2 points; with P^L folded into the
// forward matrix, the product gives the U-row coefficients F~ = P^L c that the
// multistep right-hand side uses).  Complex coefficients are pairs of real
// columns, 16 pencils (32 real columns) per block.
//
// v_mfma_f64_16x16x4f64, lane l: A[i][k] at i = l mod 16, k = l / 16;
// B[k][j] at j = l mod 16, k = l / 16; D[i][j] in lane j + 16 (i mod 4),
// register i / 4.  The matrices are stored in that fragment order:
// Afrag[(rb * KS + ks) * 64 + l] = A[16 rb + l mod 16][4 ks + l / 16].
#include "common.h"
#include "kernels.h"

namespace stau {

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {
__device__ __forceinline__ bool mm_active(const XformArgs& a, int p) {
  if (p >= a.P) return false;
  if (a.dim == 2) return p < a.Pa;
  const int iy = p / a.Px, ix = p - iy * a.Px;
  return ix < a.Pa && iy != a.Ny / 2;
}
__device__ __forceinline__ double mm_k(const XformArgs& a, int p, int der) {
  if (der == 1) {
    const int ix = a.dim == 2 ? p : p % a.Px;
    return a.two_pi_over_Lx * (double)ix;
  }
  const int iy = p / a.Px;
  const int kyi = iy < (a.Ny + 1) / 2 ? iy : iy - a.Ny;
  return a.two_pi_over_Ly * (double)kyi;
}

// acc[c] += A(row block rb) x Bt(column block c), c = 0, 1; Bt[k][32] in LDS
__device__ __forceinline__ void mm_tile2(const double* __restrict__ Afrag, const double* Bt, int rb,
                                         int KS, int lane, v4d& acc0, v4d& acc1) {
  const double* Ap = Afrag + (size_t)rb * KS * 64 + lane;
  const double* Bp = Bt + (lane >> 4) * 32 + (lane & 15);
#pragma unroll 4
  for (int ks = 0; ks < KS; ++ks) {
    const double av = Ap[ks * 64];
    const double b0 = Bp[ks * 128];
    const double b1 = Bp[ks * 128 + 16];
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc1, 0, 0, 0);
  }
}
}  // namespace

// ---------------------------------------------------------------------------
// Backward z transform of the fields of `fl` (derivative flags as in
// zb_kernel): G[f][j][p] for 16 pencils per block, field blockIdx.y.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) zb_mm_kernel(XformArgs a, FieldList fl,
                                                    const double2* __restrict__ X,
                                                    double2* __restrict__ G,
                                                    const double* __restrict__ Bfrag) {
  extern __shared__ double smem[];  // Bt[N][32]
  const int f = blockIdx.y, p0 = blockIdx.x * 16;
  const int M = a.M, N = a.N, S = fl.src_S ? fl.src_S : a.S;
  const int var = fl.var[f], der = fl.deriv[f];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int idx = tid; idx < 16 * N; idx += 256) {
    const int s = idx / N, n = idx - s * N;
    const int p = p0 + s;
    double re = 0.0, im = 0.0;
    if (mm_active(a, p)) {
      const double2 c = X[((size_t)p * S + var) * N + n];
      if (der) {
        const double kk = mm_k(a, p, der);
        re = -kk * c.y;  // i k c
        im = kk * c.x;
      } else {
        re = c.x;
        im = c.y;
      }
    }
    smem[n * 32 + 2 * s] = re;
    smem[n * 32 + 2 * s + 1] = im;
  }
  __syncthreads();
  const int RB = M / 16, KS = N / 4;
  for (int rb = wv; rb < RB; rb += 4) {
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    mm_tile2(Bfrag, smem, rb, KS, lane, acc0, acc1);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = c * 16 + (lane & 15);
      const int p = p0 + (col >> 1), part = col & 1;
      if (p < a.P) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb * 16 + 4 * r + (lane >> 4);
          ((double*)(G + ((size_t)f * M + row) * a.P + p))[part] = c == 0 ? acc0[r] : acc1[r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Forward z transform of the ne explicit-term fields H[e][j][p] with the
// epilogue of zf_kernel: mode 0 writes c (Ffrag = Fz), mode 1 assembles the
// SBDF right-hand side from F~ (Ffrag = P^L Fz) and writes the history.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) zf_mm_kernel(XformArgs a, const double2* __restrict__ H,
                                                    double2* __restrict__ out, RhsArgs r,
                                                    const double* __restrict__ Ffrag) {
  extern __shared__ double smem[];  // Bt[M][32], then Ct[32][N + 1]
  const int e = blockIdx.y, p0 = blockIdx.x * 16;
  const int M = a.M, N = a.N, ne = a.ne;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int idx = tid; idx < 16 * M; idx += 256) {
    const int j = idx >> 4, s = idx & 15;  // coalesced along p
    const int p = p0 + s;
    double2 v = make_double2(0.0, 0.0);
    if (p < a.P) v = H[((size_t)e * M + j) * a.P + p];
    smem[j * 32 + 2 * s] = v.x;
    smem[j * 32 + 2 * s + 1] = v.y;
  }
  __syncthreads();
  const int RB = N / 16, KS = M / 4;
  v4d acc[4][2];  // row blocks wv, wv + 4, wv + 8, wv + 12 (N <= 256)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rb = wv + 4 * q;
    acc[q][0] = v4d{0.0, 0.0, 0.0, 0.0};
    acc[q][1] = v4d{0.0, 0.0, 0.0, 0.0};
    if (rb < RB) mm_tile2(Ffrag, smem, rb, KS, lane, acc[q][0], acc[q][1]);
  }
  __syncthreads();
  const int ld = N + 1;
  double* Ct = smem;  // Ct[col][n]
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rb = wv + 4 * q;
    if (rb >= RB) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = c * 16 + (lane & 15);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) Ct[col * ld + rb * 16 + 4 * rr + (lane >> 4)] = acc[q][c][rr];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < 16 * N; idx += 256) {
    const int s = idx / N, nn = idx - s * N;
    const int p = p0 + s;
    if (p >= a.P) continue;
    const size_t o = ((size_t)p * ne + e) * N + nn;
    const double2 v = make_double2(Ct[(2 * s) * ld + nn], Ct[(2 * s + 1) * ld + nn]);
    if (r.mode == 0) {
      out[o] = v;
      continue;
    }
    double2 Ft = make_double2(0.0, 0.0), MX = make_double2(0.0, 0.0), B = make_double2(0.0, 0.0);
    if (mm_active(a, p) && nn <= N - 2) {
      Ft = v;
      const double cnn = nn == 0 ? 1.0 : 0.5;
      const double2* xc = r.Xprev + ((size_t)p * a.S + (e + 1)) * N;
      const double2 x0 = xc[nn];
      MX = make_double2(cnn * x0.x, cnn * x0.y);
      if (nn + 2 < N) {
        const double2 x2 = xc[nn + 2];
        MX.x -= 0.5 * x2.x;
        MX.y -= 0.5 * x2.y;
      }
      B = make_double2(r.c1 * Ft.x - r.a1 * MX.x, r.c1 * Ft.y - r.a1 * MX.y);
      if (r.has_hist) {
        const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
        const double2 Fo = r.hist_old[ho], Mo = r.hist_old[ho + (size_t)ne * N];
        B.x += r.c2 * Fo.x - r.a2 * Mo.x;
        B.y += r.c2 * Fo.y - r.a2 * Mo.y;
      }
    }
    const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
    r.hist_cur[ho] = Ft;
    r.hist_cur[ho + (size_t)ne * N] = MX;
    out[o] = B;
  }
}

// ---------------------------------------------------------------------------
// launchers (N a multiple of 32 and N <= 256: M = 3N/2 a multiple of 16)
// ---------------------------------------------------------------------------
bool mm_supported(int N) { return N % 32 == 0 && N >= 32 && N <= 256; }

hipError_t launch_zb_mm(const XformArgs& a, const FieldList& fl, const void* X, void* G,
                        const double* Bfrag, hipStream_t st) {
  dim3 grid((a.P + 15) / 16, fl.nf);
  const size_t lds = (size_t)a.N * 32 * sizeof(double);
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)zb_mm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(zb_mm_kernel, grid, dim3(256), lds, st, a, fl, (const double2*)X, (double2*)G,
                     Bfrag);
  return hipGetLastError();
}

hipError_t launch_zf_mm(const XformArgs& a, const void* H, void* out, const RhsArgs& r,
                        const double* Ffrag, hipStream_t st) {
  if (!mm_supported(a.N)) return hipErrorInvalidValue;
  dim3 grid((a.P + 15) / 16, a.ne);
  size_t lds = (size_t)a.M * 32 * sizeof(double);
  const size_t lds2 = (size_t)32 * (a.N + 1) * sizeof(double);
  if (lds2 > lds) lds = lds2;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)zf_mm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(zf_mm_kernel, grid, dim3(256), lds, st, a, (const double2*)H, (double2*)out, r,
                     Ffrag);
  return hipGetLastError();
}

}  // namespace stau
