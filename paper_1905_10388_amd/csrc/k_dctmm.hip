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
// SBDF right-hand side from F~ (Ffrag = P^L Fz) and writes the history, mode 2
// the right-hand side of a Runge-Kutta stage.
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
      if (r.mode == 2) {
        rk_rhs(r.rk, o, Ft, MX, out);
        continue;
      }
      B = make_double2(r.c1 * Ft.x - r.a1 * MX.x, r.c1 * Ft.y - r.a1 * MX.y);
      if (r.has_hist) {
        const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
        const double2 Fo = r.hist_old[ho], Mo = r.hist_old[ho + (size_t)ne * N];
        B.x += r.c2 * Fo.x - r.a2 * Mo.x;
        B.y += r.c2 * Fo.y - r.a2 * Mo.y;
      }
    }
    if (r.mode == 2) {  // inactive pencil or row N - 1
      out[o] = B;
      continue;
    }
    const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
    r.hist_cur[ho] = Ft;
    r.hist_cur[ho + (size_t)ne * N] = MX;
    out[o] = B;
  }
}

// ---------------------------------------------------------------------------
// Mixed precision: the same products as split-BF16 matrix-core MFMAs with
// FP32 accumulation (v_mfma_f32_16x16x32_bf16).  Every operand x is split
// x = h + m + l into three BF16 terms (h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m), 24 significant bits in all); the product keeps the six
// terms above 2^-24 relative:
//   A B ~ Al Bh + Am Bm + Ah Bl + Am Bh + Ah Bm + Ah Bh   (small terms first).
// Fragment layout, lane l: A[i][k] at i = l mod 16, k = 8 (l / 16) + e
// (element e of the lane's 8 BF16); B[k][j] at j = l mod 16, same k;
// D[i][j] in lane j + 16 (i / 4), register i mod 4.  The tables are stored
// split in that order, A3[((rb * KS + ks) * 3 + term) * 64 + l] (8 BF16 per
// lane, KS = K / 32).  The data operand is split once per block into LDS in
// the same order, Bs[((ks * 2 + c) * 3 + term) * 64 + l] for the column
// blocks c = 0, 1 (16 pencils, real and imaginary columns interleaved).  A
// block covers 4 * RPW row blocks (blockIdx.z selects which), so that the
// grid has enough blocks where pencils are few.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kRPW = 2;  // row blocks per wave

// split 8 values into their three BF16 terms and store them as lane `ln` of
// the fragments at Bs + base (term stride 64)
__device__ __forceinline__ void split_store(const float (&x)[8], bf16x8* Bs, int base, int ln) {
  bf16x8 h, m, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 bh = (__bf16)x[e];
    const float r1 = x[e] - (float)bh;
    const __bf16 bm = (__bf16)r1;
    h[e] = bh;
    m[e] = bm;
    l[e] = (__bf16)(r1 - (float)bm);
  }
  Bs[base + ln] = h;
  Bs[base + 64 + ln] = m;
  Bs[base + 128 + ln] = l;
}

// acc0/acc1 += A(row block rb) x B(column blocks 0, 1)
__device__ __forceinline__ void mm3_tile2(const bf16x8* __restrict__ A3, const bf16x8* Bs, int rb,
                                          int KS, int lane, f32x4& acc0, f32x4& acc1) {
  const bf16x8* Ap = A3 + (size_t)rb * KS * 192 + lane;
  const bf16x8* Bp = Bs + lane;
  for (int ks = 0; ks < KS; ++ks) {
    const bf16x8 ah = Ap[ks * 192], am = Ap[ks * 192 + 64], al = Ap[ks * 192 + 128];
    const bf16x8 bh0 = Bp[ks * 384], bm0 = Bp[ks * 384 + 64], bl0 = Bp[ks * 384 + 128];
    const bf16x8 bh1 = Bp[ks * 384 + 192], bm1 = Bp[ks * 384 + 256], bl1 = Bp[ks * 384 + 320];
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh1, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm1, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl1, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh1, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm1, acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh1, acc1, 0, 0, 0);
  }
}
}  // namespace

// Backward z transform, mixed path: G[f][j][p] (FP32 complex) from the FP64
// state, derivative flags as in zb_kernel.
__global__ void __launch_bounds__(256) zb_bf16_kernel(XformArgs a, FieldList fl,
                                                      const double2* __restrict__ X,
                                                      float2* __restrict__ G,
                                                      const bf16x8* __restrict__ B3) {
  extern __shared__ bf16x8 sB[];
  const int f = blockIdx.y, p0 = blockIdx.x * 16, rb0 = blockIdx.z * 4 * kRPW;
  const int M = a.M, N = a.N, S = fl.src_S ? fl.src_S : a.S;
  const int var = fl.var[f], der = fl.deriv[f];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int RB = M / 16, KS = N / 32, NG = N / 8;
  const bool any = __syncthreads_or(tid < 16 && mm_active(a, p0 + tid));
  if (any) {
    for (int it = tid; it < 16 * NG; it += 256) {
      const int s = it / NG, g = it - s * NG;  // pencil s, coefficients 8g .. 8g+7
      const int p = p0 + s;
      float re[8], im[8];
      if (mm_active(a, p)) {
        const double2* xp = X + ((size_t)p * S + var) * N + 8 * g;
        const double kk = der ? mm_k(a, p, der) : 0.0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double2 c = xp[e];
          re[e] = (float)(der ? -kk * c.y : c.x);  // i k c
          im[e] = (float)(der ? kk * c.x : c.y);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) re[e] = im[e] = 0.f;
      }
      const int base = ((g >> 2) * 2 + (s >> 3)) * 192, ln = (g & 3) * 16 + ((2 * s) & 15);
      split_store(re, sB, base, ln);
      split_store(im, sB, base, ln + 1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kRPW; ++q) {
    const int rb = rb0 + wv + 4 * q;
    if (rb >= RB) break;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    if (any) mm3_tile2(B3, sB, rb, KS, lane, acc0, acc1);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = c * 16 + (lane & 15);
      const int p = p0 + (col >> 1), part = col & 1;
      if (p < a.P) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb * 16 + 4 * (lane >> 4) + r;
          ((float*)(G + ((size_t)f * M + row) * a.P + p))[part] = c == 0 ? acc0[r] : acc1[r];
        }
      }
    }
  }
}

// Forward z transform, mixed path, from H[e][j][p] (FP32 complex), with the
// FP64 epilogue of zf_kernel (mode 0: c with the Fz table; modes 1 and 2: the
// SBDF or Runge-Kutta stage right-hand side from F~ with the P^L Fz table) for
// the block's rows.
__global__ void __launch_bounds__(256) zf_bf16_kernel(XformArgs a, const float2* __restrict__ H,
                                                      double2* __restrict__ out, RhsArgs r,
                                                      const bf16x8* __restrict__ F3) {
  extern __shared__ bf16x8 sB[];
  const int e = blockIdx.y, p0 = blockIdx.x * 16, rb0 = blockIdx.z * 4 * kRPW;
  const int M = a.M, N = a.N, ne = a.ne;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int RB = N / 16, KS = M / 32, MG = M / 8;
  const bool any = __syncthreads_or(tid < 16 && (r.mode == 0 ? p0 + tid < a.P : mm_active(a, p0 + tid)));
  if (any) {
    for (int it = tid; it < 16 * MG; it += 256) {
      const int g = it >> 4, s = it & 15;  // rows 8g .. 8g+7 of pencil s (coalesced along p)
      const int p = p0 + s;
      float re[8], im[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        float2 v = make_float2(0.f, 0.f);
        if (p < a.P) v = H[((size_t)e * M + 8 * g + k) * a.P + p];
        re[k] = v.x;
        im[k] = v.y;
      }
      const int base = ((g >> 2) * 2 + (s >> 3)) * 192, ln = (g & 3) * 16 + ((2 * s) & 15);
      split_store(re, sB, base, ln);
      split_store(im, sB, base, ln + 1);
    }
    __syncthreads();
  }
  f32x4 acc[kRPW][2];
#pragma unroll
  for (int q = 0; q < kRPW; ++q) {
    const int rb = rb0 + wv + 4 * q;
    acc[q][0] = f32x4{0.f, 0.f, 0.f, 0.f};
    acc[q][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (any && rb < RB) mm3_tile2(F3, sB, rb, KS, lane, acc[q][0], acc[q][1]);
  }
  __syncthreads();
  // stage C[n][col] for the block's rows as Ct[col][n - 16 rb0]
  constexpr int NR = 4 * kRPW * 16;
  constexpr int ld = NR + 1;
  float* Ct = (float*)sB;
#pragma unroll
  for (int q = 0; q < kRPW; ++q) {
    const int rbl = wv + 4 * q;
    if (rb0 + rbl >= RB) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = c * 16 + (lane & 15);
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) Ct[col * ld + rbl * 16 + 4 * (lane >> 4) + rr] = acc[q][c][rr];
    }
  }
  __syncthreads();
  const int n0 = rb0 * 16, nr = min(NR, N - n0);
  for (int idx = tid; idx < 16 * nr; idx += 256) {
    const int s = idx / nr, nl = idx - s * nr, nn = n0 + nl;
    const int p = p0 + s;
    if (p >= a.P) continue;
    const size_t o = ((size_t)p * ne + e) * N + nn;
    const double2 v = make_double2((double)Ct[(2 * s) * ld + nl], (double)Ct[(2 * s + 1) * ld + nl]);
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
      if (r.mode == 2) {
        rk_rhs(r.rk, o, Ft, MX, out);
        continue;
      }
      B = make_double2(r.c1 * Ft.x - r.a1 * MX.x, r.c1 * Ft.y - r.a1 * MX.y);
      if (r.has_hist) {
        const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
        const double2 Fo = r.hist_old[ho], Mo = r.hist_old[ho + (size_t)ne * N];
        B.x += r.c2 * Fo.x - r.a2 * Mo.x;
        B.y += r.c2 * Fo.y - r.a2 * Mo.y;
      }
    }
    if (r.mode == 2) {  // inactive pencil or row N - 1
      out[o] = B;
      continue;
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

bool mm_bf16_supported(int N) { return N == 64 || N == 128 || N == 256; }

hipError_t launch_zb_bf16(const XformArgs& a, const FieldList& fl, const void* X, void* G,
                          const void* B3, hipStream_t st) {
  if (!mm_bf16_supported(a.N)) return hipErrorInvalidValue;
  const int RB = a.M / 16;
  dim3 grid((a.P + 15) / 16, fl.nf, (RB + 4 * kRPW - 1) / (4 * kRPW));
  const size_t lds = (size_t)(a.N / 32) * 384 * sizeof(bf16x8);
  hipLaunchKernelGGL(zb_bf16_kernel, grid, dim3(256), lds, st, a, fl, (const double2*)X, (float2*)G,
                     (const bf16x8*)B3);
  return hipGetLastError();
}

hipError_t launch_zf_bf16(const XformArgs& a, const void* H, void* out, const RhsArgs& r,
                          const void* F3, hipStream_t st) {
  if (!mm_bf16_supported(a.N)) return hipErrorInvalidValue;
  const int RB = a.N / 16;
  dim3 grid((a.P + 15) / 16, a.ne, (RB + 4 * kRPW - 1) / (4 * kRPW));
  size_t lds = (size_t)(a.M / 32) * 384 * sizeof(bf16x8);
  const size_t lds2 = (size_t)32 * (4 * kRPW * 16 + 1) * sizeof(float);
  if (lds2 > lds) lds = lds2;
  hipLaunchKernelGGL(zf_bf16_kernel, grid, dim3(256), lds, st, a, (const float2*)H, (double2*)out, r,
                     (const bf16x8*)F3);
  return hipGetLastError();
}

}  // namespace stau
