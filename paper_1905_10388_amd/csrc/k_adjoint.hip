// Adjoint transform kernels of the discrete adjoint step: the transposes of
// the z transforms, of the fused x pass and of the kinetic-energy and
// initial-state maps.
#include "xform.h"

namespace stau {

// ===========================================================================
// Adjoint kernels.  Complex coefficients are pairs of independent reals; the
// adjoint of z is dJ/dRe z + i dJ/dIm z.  Real-grid adjoints are real.
// ===========================================================================

// Adjoint of the backward z transform (c -> g_j = sum_n c_n T_n(z_j), with
// c optionally multiplied by i k): c_bar_n += conj(i k) sum_j T_n(z_j) g_bar_j,
// i.e. an unweighted DCT-II per source field, summed per target variable and
// accumulated into Xbar[p][var][n].
template <int MAXBF, int MAXIT, typename T, int EPT = kZEpt>
__global__ void __launch_bounds__(kZThreads) zadj_kernel(XformArgs a, AccList al,
                                                         const typename V2<T>::type* __restrict__ Gb,
                                                         double2* __restrict__ Xb, int TP) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  const int M = a.M, N = a.N, S = a.S;
  cT* buf = (cT*)smem;
  cT* twl = buf + EPT * kZThreads;  // FFT twiddles after the EPT * kZThreads tile points
  cT* dcl = twl + M;
  const int ti = blockIdx.y;
  const int p0 = blockIdx.x * TP;
  const int tid = threadIdx.x, nt = kZThreads;
  stage_z_tables<T>(a, twl, dcl, M, tid);
  cd acc[MAXIT];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) acc[it] = mk(0.0, 0.0);
  for (int q = 0; q < al.nsrc[ti]; ++q) {
    const int f = al.src[ti][q], der = al.deriv[ti][q];
    {
      cT hv[EPT];
#pragma unroll
      for (int it = 0; it < EPT; ++it) {
        const int idx = tid + it * nt;
        const int jz = idx / TP, s = idx - jz * TP;
        const int p = p0 + s;
        hv[it] = mk<T>(0, 0);
        if (p < a.P) hv[it] = ldv<T>(Gb + ((size_t)f * M + jz) * a.P + p);
      }
#pragma unroll
      for (int it = 0; it < EPT; ++it) {
        const int idx = tid + it * nt;
        const int jz = idx / TP, s = idx - jz * TP;
        const int dst = (jz & 1) ? (M - 1 - (jz >> 1)) : (jz >> 1);
        buf[s * M + dst] = hv[it];
      }
    }
    __syncthreads();
    fft_lds<-1, MAXBF>(buf, M, TP, (const cT*)twl, tid, nt);
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      const int idx = tid + it * nt;
      if (idx < TP * N) {
        const int s = idx / N, nn = idx - s * N;
        const int p = p0 + s;
        const cT V = buf[s * M + nn];
        const cT Vm = buf[s * M + (nn == 0 ? 0 : M - nn)];
        const cT w = conj(dcl[nn]);
        const cT P = cmul(w, V), Q = cmul(w, conj(Vm));
        cd Y = mk((double)((T)0.5 * (P.x + Q.x)), (double)((T)0.5 * (P.y - Q.y)));
        if (nn & 1) Y = mk(-Y.x, -Y.y);
        if (der && p < a.P) {
          const double kk = der == 1 ? kx_of(a, p) : ky_of(a, p);
          Y = mk(kk * Y.y, -kk * Y.x);  // conj(i k) Y = -i k Y
        }
        acc[it] = acc[it] + Y;
      }
    }
    __syncthreads();
  }
  const int var = al.target[ti];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int idx = tid + it * nt;
    if (idx < TP * N) {
      const int s = idx / N, nn = idx - s * N;
      const int p = p0 + s;
      if (active(a, p)) {
        double2* o = Xb + ((size_t)p * S + var) * N + nn;
        const double2 old = *o;
        *o = make_double2(old.x + acc[it].x, old.y + acc[it].y);
      }
    }
  }
}

// Adjoint of the fused x pass for one dealiased z row.  Recomputes the eight
// forward grid fields from G, maps the explicit-term adjoints H_bar to the
// grid (adjoint of the truncated real-to-complex transform:
// g_bar_i = (1/L) [Re c_0 + Re sum_{k>=1} c_k e^{2 pi i k i / L}]), applies the
// product rule, and maps the eight grid adjoints back to spectra (adjoint of
// the complex-to-real synthesis: c_bar_k = w_k sum_i g_bar_i e^{-2 pi i k i/L},
// w_0 = 1, w_k = 2).  SPLIT: two blocks per row (blockIdx.y 0: the (u, w)
// outputs, 1: the derivative outputs), for launches with fewer rows than
// compute units; each block synthesises the fields its outputs need.
template <int MAXBF, int PTS, int NT, bool TWL, typename T, bool SPLIT>
__global__ void __launch_bounds__(NT) xpass_adj_kernel(XformArgs a,
                                                       const typename V2<T>::type* __restrict__ G,
                                                       const typename V2<T>::type* __restrict__ Hb,
                                                       typename V2<T>::type* __restrict__ Gb) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  using S2 = typename V2<T>::type;
  constexpr int KPT = (PTS + 2) / 3;  // half-spectrum entries per thread (Pa = L / 3)
  cT* buf = (cT*)smem;
  const int jz = blockIdx.x;
  const int M = a.M, L = a.L, Pa = a.Pa, P = a.P;
  const int tid = threadIdx.x;
  const cT* twg = (const cT*)(sizeof(T) == 8 ? (const void*)a.twx : (const void*)a.twx32);
  cT* twl = buf + L;
  if constexpr (TWL) {
    for (int i = tid; i < L; i += NT) twl[i] = twg[i];
  }
  const cT* tw = TWL ? (const cT*)twl : twg;
  auto row = [&](const S2* base, int f) { return base + ((size_t)f * M + jz) * P; };
  // complex-to-real pairs: 0..3 the forward fields (G 0..7), 4 (Hb 0, Hb 1)
  // and 5 (Hb 2, -); hs scales k >= 1 (1 for synthesis, 0.5 for the adjoint
  // of the truncated forward transform)
  cT sa[KPT], sb[KPT];
  auto fetch = [&](int k) {
    const S2* A = k < 4 ? row(G, 2 * k) : row(Hb, 2 * (k - 4));
    const S2* B = k < 4 ? row(G, 2 * k + 1) : (k == 4 ? row(Hb, 1) : nullptr);
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      sa[q] = mk<T>(0, 0);
      sb[q] = mk<T>(0, 0);
      if (kk < Pa) {
        sa[q] = ldv<T>(A + kk);
        if (B) sb[q] = ldv<T>(B + kk);
      }
    }
  };
  auto scatter = [&](T hs) {
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      if (kk < Pa) {
        cT Ak = sa[q], Bk = sb[q];
        if (kk == 0) {
          Ak.y = 0;
          Bk.y = 0;
        } else {
          Ak = scale(Ak, hs);
          Bk = scale(Bk, hs);
        }
        buf[kk] = mk<T>(Ak.x - Bk.y, Ak.y + Bk.x);
        if (kk > 0) buf[L - kk] = mk<T>(Ak.x + Bk.y, -Ak.y + Bk.x);
      }
    }
    for (int k = Pa + tid; k <= L - Pa; k += NT) buf[k] = mk<T>(0, 0);
  };
  // adjoint of a synthesis pair: spectra of two real grid rows, weights w_k
  auto r2c_adj_pair = [&](const T* ga, const T* gb, int fa, int fb) {
#pragma unroll
    for (int q = 0; q < PTS; ++q) {
      const int i = tid + q * NT;
      if (i < L) buf[i] = mk<T>(ga[q], gb[q]);
    }
    __syncthreads();
    fft_lds<-1, MAXBF, T, true>(buf, L, 1, tw, tid, NT);
    S2* Oa = Gb + ((size_t)fa * M + jz) * P;
    S2* Ob = Gb + ((size_t)fb * M + jz) * P;
    for (int k = tid; k < P; k += NT) {
      cT A = mk<T>(0, 0), Bv = mk<T>(0, 0);
      if (k < Pa) {
        const cT Zk = buf[k], Zm = buf[k == 0 ? 0 : L - k];
        const T wk = k == 0 ? (T)1 : (T)2;
        A = mk<T>((T)0.5 * (Zk.x + Zm.x) * wk, (T)0.5 * (Zk.y - Zm.y) * wk);
        Bv = mk<T>((T)0.5 * (Zk.y + Zm.y) * wk, (T)-0.5 * (Zk.x - Zm.x) * wk);
      }
      stv<T>(Oa + k, A);
      stv<T>(Ob + k, Bv);
    }
    __syncthreads();
  };

  // The grid fields are consumed as they are synthesised: the explicit-term
  // adjoints first (n_b, n_u, n_w), then the derivative pairs accumulate the
  // (u, w) adjoints t1 = -(n . grad_x), t2 = -(n . grad_z), and (u, w) feeds
  // the derivative adjoints -n_q (u, w).  Part 1 computes the (u, w) outputs,
  // part 2 the six derivative outputs (blocks of a split launch), part 0 both.
  auto body = [&](auto part_c) {
    constexpr int PART = decltype(part_c)::value;
    constexpr int NS = PART == 1 ? 5 : PART == 2 ? 3 : 6;
    // synthesis order: 4, 5 (H_bar), then part 1: 1, 2, 3; part 2: 0; part 0: 1, 2, 3, 0
    auto seq = [](int i) { return i == 0 ? 4 : i == 1 ? 5 : PART == 2 ? 0 : i < 5 ? i - 1 : 0; };
    T u[PTS], w[PTS], nb[PTS], nu[PTS], nw[PTS], t1[PTS], t2[PTS];
    const T invL = (T)1 / (T)L;
    fetch(seq(0));
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int k = seq(i);
      scatter(k < 4 ? (T)1 : (T)0.5);
      if (i + 1 < NS) fetch(seq(i + 1));
      __syncthreads();
      fft_lds<+1, MAXBF, T, true>(buf, L, 1, tw, tid, NT);
#pragma unroll
      for (int q = 0; q < PTS; ++q) {
        const int ii = tid + q * NT;
        if (ii < L) {
          const T x = buf[ii].x, y = buf[ii].y;
          if (k == 4) {
            nb[q] = x * invL;
            nu[q] = y * invL;
          } else if (k == 5) {
            nw[q] = x * invL;
          } else if (k == 0) {
            u[q] = x;
            w[q] = y;
          } else if (k == 1) {
            t1[q] = -(nb[q] * x);
            t2[q] = -(nb[q] * y);
          } else {
            const T n = k == 2 ? nu[q] : nw[q];
            t1[q] -= n * x;
            t2[q] -= n * y;
          }
        }
      }
      __syncthreads();
    }
    if constexpr (PART != 2) r2c_adj_pair(t1, t2, 0, 1);
    if constexpr (PART != 1) {
#pragma unroll
      for (int q = 0; q < PTS; ++q) {
        t1[q] = -nb[q] * u[q];
        t2[q] = -nb[q] * w[q];
      }
      r2c_adj_pair(t1, t2, 2, 3);
#pragma unroll
      for (int q = 0; q < PTS; ++q) {
        t1[q] = -nu[q] * u[q];
        t2[q] = -nu[q] * w[q];
      }
      r2c_adj_pair(t1, t2, 4, 5);
#pragma unroll
      for (int q = 0; q < PTS; ++q) {
        t1[q] = -nw[q] * u[q];
        t2[q] = -nw[q] * w[q];
      }
      r2c_adj_pair(t1, t2, 6, 7);
    }
  };
  if constexpr (SPLIT) {
    if (blockIdx.y == 0)
      body(std::integral_constant<int, 1>{});
    else
      body(std::integral_constant<int, 2>{});
  } else {
    body(std::integral_constant<int, 0>{});
  }
}

// Kinetic-energy adjoint for one row: u_bar = e_bar_j u, w_bar = e_bar_j w with
// e_bar_j = (1/L) sum_m w_m (2 - delta)/M T_m(z_j) (precomputed in ebar).
template <int MAXBF, int PTS, int NT>
__global__ void __launch_bounds__(NT) ke_row_adj_kernel(XformArgs a, const double2* __restrict__ G,
                                                        const double2* __restrict__ ebar,
                                                        double2* __restrict__ Gb) {
  extern __shared__ double2 smem[];
  cd* buf = (cd*)smem;
  const int jz = blockIdx.x;
  const int M = a.M, L = a.L, Pa = a.Pa, P = a.P;
  const int tid = threadIdx.x;
  constexpr int nt = NT;
  const cd* tw = (const cd*)a.twx;
  const double2* A = G + ((size_t)0 * M + jz) * P;
  const double2* B = G + ((size_t)1 * M + jz) * P;
  for (int k = tid; k < L; k += nt) {
    cd z = mk(0.0, 0.0);
    if (k < Pa) {
      cd Ak = ld2(A + k), Bk = ld2(B + k);
      if (k == 0) {
        Ak.y = 0.0;
        Bk.y = 0.0;
      }
      z = mk(Ak.x - Bk.y, Ak.y + Bk.x);
    } else if (k > L - Pa) {
      cd Ak = ld2(A + (L - k)), Bk = ld2(B + (L - k));
      z = mk(Ak.x + Bk.y, -Ak.y + Bk.x);
    }
    buf[k] = z;
  }
  __syncthreads();
  fft_lds<+1, MAXBF>(buf, L, 1, tw, tid, nt);
  const double e = ebar[jz].x / (double)L;
  double gu[PTS], gw[PTS];
#pragma unroll
  for (int q = 0; q < PTS; ++q) {
    const int i = tid + q * nt;
    if (i < L) {
      gu[q] = e * buf[i].x;
      gw[q] = e * buf[i].y;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PTS; ++q) {
    const int i = tid + q * nt;
    if (i < L) buf[i] = mk(gu[q], gw[q]);
  }
  __syncthreads();
  fft_lds<-1, MAXBF>(buf, L, 1, tw, tid, nt);
  double2* Oa = Gb + ((size_t)0 * M + jz) * P;
  double2* Ob = Gb + ((size_t)1 * M + jz) * P;
  for (int k = tid; k < P; k += nt) {
    cd Av = mk(0.0, 0.0), Bv = mk(0.0, 0.0);
    if (k < Pa) {
      cd Zk = buf[k], Zm = buf[k == 0 ? 0 : L - k];
      const double wk = k == 0 ? 1.0 : 2.0;
      Av = mk(0.5 * (Zk.x + Zm.x) * wk, 0.5 * (Zk.y - Zm.y) * wk);
      Bv = mk(0.5 * (Zk.y + Zm.y) * wk, -0.5 * (Zk.x - Zm.x) * wk);
    }
    st2(Oa + k, Av);
    st2(Ob + k, Bv);
  }
}

// Initial-state adjoint, step 1 (per pencil): c_bar = X_bar_b + D^T X_bar_bz
// for bz = D b, D_nm = 4 m / (1 + delta_n0) for n < m, m - n odd (d/dz on
// [0, 1] of the T-to-T derivative).
__global__ void ic_adj_coef_kernel(XformArgs a, const double2* __restrict__ Xb,
                                   double2* __restrict__ C, int vb, int vbz) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  const int N = a.N, S = a.S;
  const double2* xb = Xb + ((size_t)p * S + vb) * N;
  const double2* xz = Xb + ((size_t)p * S + vbz) * N;
  double2* c = C + (size_t)p * N;
  double se_r = 0.0, se_i = 0.0, so_r = 0.0, so_i = 0.0;  // running sums over even / odd n
  for (int m = 0; m < N; ++m) {
    double vr = xb[m].x, vi = xb[m].y;
    if (m & 1) {
      vr += 4.0 * m * se_r;
      vi += 4.0 * m * se_i;
    } else {
      vr += 4.0 * m * so_r;
      vi += 4.0 * m * so_i;
    }
    c[m] = make_double2(vr, vi);
    const double f = m == 0 ? 0.5 : 1.0;
    if (m & 1) {
      so_r += xz[m].x;
      so_i += xz[m].y;
    } else {
      se_r += f * xz[m].x;
      se_i += f * xz[m].y;
    }
  }
}

// Initial-state adjoint, step 3 (per z level): g_bar_i = (1/Nx) [Re H_0 +
// Re sum_{k>=1} H_k e^{2 pi i k i / Nx}] (adjoint of the truncated forward x
// transform at scale 1), written to gbar[ix][jz].
template <int MAXBF>
__global__ void __launch_bounds__(256) ic_adj_x_kernel(XformArgs a, const double2* __restrict__ H1,
                                                       double* __restrict__ gbar) {
  extern __shared__ double2 smem[];
  cd* buf = (cd*)smem;
  const int jz = blockIdx.x;
  const int Nx = a.Nx, N = a.N, Pa = a.Pa;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double2* h = H1 + (size_t)jz * a.P;
  for (int k = tid; k < Nx; k += nt) {
    cd z = mk(0.0, 0.0);
    if (k == 0)
      z = mk(h[0].x, 0.0);
    else if (k < Pa)
      z = scale(ld2(h + k), 0.5);
    else if (k > Nx - Pa)
      z = scale(conj(ld2(h + (Nx - k))), 0.5);
    buf[k] = z;
  }
  __syncthreads();
  fft_lds<+1, MAXBF>(buf, Nx, 1, (const cd*)a.twx, tid, nt);
  const double inv = 1.0 / (double)Nx;
  for (int i = tid; i < Nx; i += nt) gbar[(size_t)i * N + jz] = buf[i].x * inv;
}

hipError_t launch_zadj(const XformArgs& a, const AccList& al, const void* Gbar, void* Xbar,
                       hipStream_t st, bool fp32) {
  int TP = z_tile(a.M);
  if (TP * a.M != kZPts || TP * a.N > 12 * kZThreads) return hipErrorInvalidValue;
  // half-size tiles when the full-size grid has fewer blocks than compute
  // units (512x128: 102 -> 198 blocks, adjoint step 146 -> 139 us; at 4096x64,
  // 390 -> 774 blocks, half tiles measured 7 us slower)
  const int dv = z_split((a.P + TP - 1) / TP * al.nt, a.M, 1);
  TP /= dv;
  const int pts = kZPts / dv;
  dim3 grid((a.P + TP - 1) / TP, al.nt);
  auto go = [&](auto kern, auto g) {
    const size_t lds = (size_t)(pts + 2 * a.M) * sizeof(*g);
    allow_lds((const void*)kern, lds);
    hipLaunchKernelGGL(kern, grid, dim3(kZThreads), lds, st, a, al, g, (double2*)Xbar, TP);
  };
  if (fp32) {
    if (dv == 2) go(zadj_kernel<3, 12, float, kZEpt / 2>, (const float2*)Gbar);
    else go(zadj_kernel<3, 12, float>, (const float2*)Gbar);
  } else {
    if (dv == 2) go(zadj_kernel<3, 12, double, kZEpt / 2>, (const double2*)Gbar);
    else go(zadj_kernel<3, 12, double>, (const double2*)Gbar);
  }
  return hipGetLastError();
}

template <int NT, int PTS, int MAXBF, typename T>
static hipError_t launch_xpass_adj_t(const XformArgs& a, const void* G, const void* Hb, void* Gb,
                                     hipStream_t st) {
  using S2 = typename V2<T>::type;
  const bool twl = (size_t)a.L * sizeof(S2) <= 32768;
  const size_t lds = (size_t)a.L * sizeof(S2) * (twl ? 2 : 1);
  int dev = 0, cus = 0;
  const bool split = hipGetDevice(&dev) == hipSuccess &&
                     hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                     a.M < cus;
  auto go = [&](auto fn) {
    allow_lds((const void*)fn, lds);
    hipLaunchKernelGGL(fn, dim3(a.M, split ? 2 : 1), dim3(NT), lds, st, a, (const S2*)G,
                       (const S2*)Hb, (S2*)Gb);
  };
  if (twl) {
    if (split)
      go(xpass_adj_kernel<MAXBF, PTS, NT, true, T, true>);
    else
      go(xpass_adj_kernel<MAXBF, PTS, NT, true, T, false>);
  } else {
    if (split)
      go(xpass_adj_kernel<MAXBF, PTS, NT, false, T, true>);
    else
      go(xpass_adj_kernel<MAXBF, PTS, NT, false, T, false>);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_xpass_adj_T(const XformArgs& a, const void* G, const void* Hb, void* Gb,
                                     hipStream_t st) {
  const int L = a.L;
  if (L <= 64) return launch_xpass_adj_t<64, 1, 1, T>(a, G, Hb, Gb, st);
  if (L <= 128) return launch_xpass_adj_t<64, 2, 1, T>(a, G, Hb, Gb, st);
  if (L <= 192) return launch_xpass_adj_t<64, 3, 1, T>(a, G, Hb, Gb, st);
  if (L <= 384) return launch_xpass_adj_t<128, 3, 1, T>(a, G, Hb, Gb, st);
  if (L <= 768) return launch_xpass_adj_t<256, 3, 1, T>(a, G, Hb, Gb, st);
  if (L <= 1536) return launch_xpass_adj_t<512, 3, 1, T>(a, G, Hb, Gb, st);
  if (L <= 3072) return launch_xpass_adj_t<1024, 3, 1, T>(a, G, Hb, Gb, st);
  if (L <= 6144) return launch_xpass_adj_t<1024, 6, 2, T>(a, G, Hb, Gb, st);
  return hipErrorInvalidValue;
}

hipError_t launch_xpass_adj(const XformArgs& a, const void* G, const void* Hbar, void* Gbar,
                            hipStream_t st, bool fp32) {
  return fp32 ? launch_xpass_adj_T<float>(a, G, Hbar, Gbar, st)
              : launch_xpass_adj_T<double>(a, G, Hbar, Gbar, st);
}

template <int NT>
static hipError_t launch_ke_row_adj_t(const XformArgs& a, const void* G, const void* ebar,
                                      void* Gb, hipStream_t st) {
  size_t lds = (size_t)a.L * sizeof(double2);
  allow_lds((const void*)ke_row_adj_kernel<2, 6, NT>, lds);
  hipLaunchKernelGGL((ke_row_adj_kernel<2, 6, NT>), dim3(a.M), dim3(NT), lds, st, a,
                     (const double2*)G, (const double2*)ebar, (double2*)Gb);
  return hipGetLastError();
}

hipError_t launch_ke_adjoint(const XformArgs& a, const void* X, void* G, void* Gbar,
                             const void* wvec, void* ebar, void* Xbar, hipStream_t st) {
  // e_bar_j: weighted DCT-III of the integration weights (one "pencil")
  XformArgs aw = a;
  aw.P = 1;
  aw.Pa = 1;
  aw.dim = 2;
  FieldList fw{};
  fw.nf = 1;
  fw.var[0] = 0;
  fw.src_S = 1;
  fw.wmode = 1;
  launch_zb(aw, fw, wvec, ebar, st);
  FieldList fl{};
  fl.nf = 2;
  fl.var[0] = 2;                   // u
  fl.var[1] = a.dim == 2 ? 3 : 4;  // w
  launch_zb(a, fl, X, G, st);
  hipError_t e;
  switch (x_threads(a.L)) {
    case 64: e = launch_ke_row_adj_t<64>(a, G, ebar, Gbar, st); break;
    case 128: e = launch_ke_row_adj_t<128>(a, G, ebar, Gbar, st); break;
    case 256: e = launch_ke_row_adj_t<256>(a, G, ebar, Gbar, st); break;
    case 512: e = launch_ke_row_adj_t<512>(a, G, ebar, Gbar, st); break;
    case 1024: e = launch_ke_row_adj_t<1024>(a, G, ebar, Gbar, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(Xbar, 0, (size_t)a.P * a.S * a.N * sizeof(double2), st);
  if (e != hipSuccess) return e;
  AccList al{};
  al.nt = 2;
  al.target[0] = 2;
  al.nsrc[0] = 1;
  al.src[0][0] = 0;
  al.target[1] = a.dim == 2 ? 3 : 4;
  al.nsrc[1] = 1;
  al.src[1][0] = 1;
  return launch_zadj(a, al, Gbar, Xbar, st);
}

hipError_t launch_initial_state_adjoint(const XformArgs& a1, const void* Xbar, double* gbar,
                                        void* work, hipStream_t st) {
  double2* C = (double2*)work;              // [P][1][N]
  double2* H1 = C + (size_t)a1.P * a1.N;    // [N][P]
  const int vb = 1, vbz = a1.dim == 2 ? 4 : 5;
  hipLaunchKernelGGL(ic_adj_coef_kernel, dim3((a1.P + 63) / 64), dim3(64), 0, st, a1,
                     (const double2*)Xbar, C, vb, vbz);
  FieldList fl{};
  fl.nf = 1;
  fl.var[0] = 0;
  fl.src_S = 1;
  fl.wmode = 1;
  launch_zb(a1, fl, C, H1, st);
  allow_lds((const void*)ic_adj_x_kernel<8>, (size_t)a1.Nx * sizeof(double2));
  hipLaunchKernelGGL((ic_adj_x_kernel<8>), dim3(a1.N), dim3(256), (size_t)a1.Nx * sizeof(double2),
                     st, a1, (const double2*)H1, gbar);
  return hipGetLastError();
}

}  // namespace stau
