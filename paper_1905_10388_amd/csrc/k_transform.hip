// Spectral transform kernels (Sec. IV): Chebyshev z transforms as DCT-III /
// DCT-II through one complex FFT of the dealiased length M per column (the
// Gauss grid is ascending, so T_n(z_j) = (-1)^n cos(pi n (2j+1) / (2M))), the
// complex y transforms of 3-D domains, and the initial-state, boundary-value
// right-hand side and kinetic-energy kernels.  The fused x pass is in
// k_xpass.hip, the adjoint kernels in k_adjoint.hip.
//
// Layouts (2-D; P = Nx/2 + 1 pencil slots, Pa = Nx/2 active):
//   state X[p][var][n]          complex, n < N
//   G[f][jz][p]                 complex, after the z backward transform
//   H[e][jz][p]                 complex, explicit term before the z forward
//   F / Bev[p][e][n]            complex

#include "xform.h"

namespace stau {

// ---------------------------------------------------------------------------
// Backward z (DCT-III with padding N -> M): g_j = sum_{n<N} c_n T_n(z_j)
// for every field of `fl` and TP pencils per block.
// ---------------------------------------------------------------------------
// MC > 0: M = MC fixed at compile time (constant divisors in the index math).
template <int MAXBF, typename T, int EPT = kZEpt, int MC = 0>
__global__ void __launch_bounds__(kZThreads) zb_kernel(XformArgs a, FieldList fl,
                                                       const double2* __restrict__ X,
                                                       typename V2<T>::type* __restrict__ G, int TPr) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  const int M = MC > 0 ? MC : a.M, N = a.N, S = fl.src_S ? fl.src_S : a.S;
  const int TP = MC > 0 ? EPT * kZThreads / MC : TPr;
  cT* buf = (cT*)smem;
  cT* twl = buf + EPT * kZThreads;  // FFT twiddles
  cT* dcl = twl + M;      // DCT twiddles
  const int f = blockIdx.y;
  const int p0 = blockIdx.x * TP;
  const int var = fl.var[f], der = fl.deriv[f];
  const double wfac = fl.wmode ? 2.0 / (double)M : 1.0;  // (2 - delta_n0) / M, n > 0
  const int tid = threadIdx.x;
  const PencilBase pb = pencil_base(a, p0);
  stage_z_tables<T>(a, twl, dcl, M, tid);
  // c_n and c_{M-n} of each owned point (zero outside the stored modes)
  double2 ya[EPT], yb[EPT];
#pragma unroll
  for (int it = 0; it < EPT; ++it) {
    const int idx = tid + it * kZThreads;
    const int s = idx / M, nn = idx - s * M;
    const int p = p0 + s;
    ya[it] = make_double2(0.0, 0.0);
    yb[it] = make_double2(0.0, 0.0);
    if (active_at(a, pb, s)) {
      const double2* col = X + ((size_t)p * S + var) * N;
      if (nn < N) ya[it] = col[nn];
      if (nn > 0 && M - nn < N) yb[it] = col[M - nn];
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < EPT; ++it) {
    const int idx = tid + it * kZThreads;
    const int s = idx / M, nn = idx - s * M;
    cT z = mk<T>(0, 0);
    if (active_at(a, pb, s)) {
      double kk = 0.0;
      if (der == 1) kk = kx_at(a, pb, s);
      if (der == 2) kk = ky_at(a, pb, s);
      auto Yp = [&](double2 v, int m) -> cd {
        cd c = mk(v.x, v.y);
        if (der) c = mk(-kk * c.y, kk * c.x);  // i k c
        double s1 = (m & 1) ? -1.0 : 1.0;      // T_n on the ascending grid
        if (m > 0) s1 *= 0.5 * wfac;
        else if (fl.wmode) s1 = 1.0 / (double)M;
        return scale(c, s1);
      };
      const cd yn = Yp(ya[it], nn);
      const cd ym = nn == 0 ? mk(0.0, 0.0) : Yp(yb[it], M - nn);
      const cd t = mk(yn.x + ym.y, yn.y - ym.x);  // Y_n - i Y_{M-n}
      if constexpr (sizeof(T) == 8) {
        z = cmul(dcl[nn], t);
      } else {
        z = cmul(dcl[nn], mk<T>((T)t.x, (T)t.y));
      }
    }
    buf[idx] = z;
  }
  __syncthreads();
  fft_lds_c<MC, +1, MAXBF, T, true, MC == 384>(buf, M, TP, (const cT*)twl, tid, kZThreads);
#pragma unroll
  for (int it = 0; it < EPT; ++it) {
    const int idx = tid + it * kZThreads;
    const int jz = idx / TP, s = idx - jz * TP;
    const int p = p0 + s;
    if (p < a.P) {
      const int src = (jz & 1) ? (M - 1 - (jz >> 1)) : (jz >> 1);
      stv<T>(G + ((size_t)f * M + jz) * a.P + p, buf[s * M + src]);
    }
  }
}

// ---------------------------------------------------------------------------
// Forward z (DCT-II with truncation M -> N): c_n = (2 - d_n0)/M sum_j g_j T_n(z_j).
// mode 0: F[p][e][n] = c_n.
// mode 1: SBDF right-hand side of the evolved-equation U-rows:
//   F~_n = P^L c (n <= N-2), MX_n = P^L X^{n-1}_e,
//   B_n = c1 F~_n - a1 MX_n + [c2 F~old_n - a2 MXold_n],
//   history hist_cur[p][0][e][n] = F~_n, hist_cur[p][1][e][n] = MX_n.
// mode 2: right-hand side of a Runge-Kutta stage from F~_n and MX_n (rk_rhs).
// ---------------------------------------------------------------------------
// MC, NC > 0: M and N fixed at compile time (constant divisors).
template <int MAXBF, int MAXIT, typename T, bool RK = false, int EPT = kZEpt, int MC = 0, int NC = 0>
__global__ void __launch_bounds__(kZThreads) zf_kernel(XformArgs a,
                                                       const typename V2<T>::type* __restrict__ H,
                                                       double2* __restrict__ out, RhsArgs r, int TPr) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  const int M = MC > 0 ? MC : a.M, N = NC > 0 ? NC : a.N, ne = a.ne;
  const int TP = MC > 0 ? EPT * kZThreads / MC : TPr;
  cT* buf = (cT*)smem;
  cT* twl = buf + EPT * kZThreads;
  cT* dcl = twl + M;
  const int e = blockIdx.y;
  const int p0 = blockIdx.x * TP;
  const int tid = threadIdx.x, nt = kZThreads;
  const PencilBase pb = pencil_base(a, p0);
  if (r.mode >= 1 && a.dim == 2 && blockIdx.x == 0) {
    // pencils beyond the grid (2-D, p >= Pa): inactive, zero right-hand side
    // (and history)
    for (int p = a.Pa; p < a.P; ++p)
      for (int nn = tid; nn < N; nn += nt) {
        const size_t o = ((size_t)p * ne + e) * N + nn;
        out[o] = make_double2(0.0, 0.0);
        if (r.mode == 1) {
          const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
          r.hist_cur[ho] = make_double2(0.0, 0.0);
          r.hist_cur[ho + (size_t)ne * N] = make_double2(0.0, 0.0);
        }
      }
  }
  stage_z_tables<T>(a, twl, dcl, M, tid);
  // epilogue in groups of four points per thread: a group's state and
  // history loads are issued together
  constexpr int GE = 4;
  static_assert(MAXIT % GE == 0, "epilogue groups");
  auto load_group = [&](int g0, double2* x0, double2* x2, double2* fo, double2* mo, RkRow* rv) {
#pragma unroll
    for (int u = 0; u < GE; ++u) {
      const int idx = tid + (g0 + u) * nt;
      x0[u] = x2[u] = fo[u] = mo[u] = make_double2(0.0, 0.0);
      if (r.mode >= 1 && idx < TP * N) {
        const int s = idx / N, nn = idx - s * N;
        const int p = p0 + s;
        if (active_at(a, pb, s) && nn <= N - 2) {
          const double2* xc = r.Xprev + ((size_t)p * a.S + (e + 1)) * N;
          x0[u] = xc[nn];
          if (nn + 2 < N) x2[u] = xc[nn + 2];
          if constexpr (RK) rk_load(r.rk, ((size_t)p * ne + e) * N + nn, rv[u]);
          if (r.mode == 1 && r.has_hist) {
            const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
            fo[u] = r.hist_old[ho];
            mo[u] = r.hist_old[ho + (size_t)ne * N];
          }
        }
      }
    }
  };
  {
    cT hv[EPT];
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
      const int idx = tid + it * nt;
      const int jz = idx / TP, s = idx - jz * TP;
      const int p = p0 + s;
      hv[it] = mk<T>(0, 0);
      if (p < a.P) hv[it] = ldv<T>(H + ((size_t)e * M + jz) * a.P + p);
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
  fft_lds_c<MC, -1, MAXBF, T, true, MC == 384>(buf, M, TP, (const cT*)twl, tid, nt);
  cT c[MAXIT];
  const T invM = (T)1 / (T)M;
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int idx = tid + it * nt;
    if (idx < TP * N) {
      const int s = idx / N, nn = idx - s * N;
      cT V = buf[s * M + nn];
      cT Vm = buf[s * M + (nn == 0 ? 0 : M - nn)];
      cT w = conj(dcl[nn]);
      cT P = cmul(w, V), Q = cmul(w, conj(Vm));
      cT Y = mk<T>((T)0.5 * (P.x + Q.x), (T)0.5 * (P.y - Q.y));
      T sc = (nn == 0 ? (T)1 : (T)2) * invM;
      if (nn & 1) sc = -sc;
      c[it] = scale(Y, sc);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int idx = tid + it * nt;
    if (idx < TP * N) {
      const int s = idx / N, nn = idx - s * N;
      buf[s * M + nn] = c[it];
    }
  }
  __syncthreads();
#pragma unroll
  for (int g0 = 0; g0 < MAXIT; g0 += GE) {
    double2 x0[GE], x2[GE], fo[GE], mo[GE];
    RkRow rv[RK ? GE : 1];
    load_group(g0, x0, x2, fo, mo, rv);
#pragma unroll
    for (int u = 0; u < GE; ++u) {
      const int idx = tid + (g0 + u) * nt;
      if (idx >= TP * N) continue;
      const int s = idx / N, nn = idx - s * N;
      const int p = p0 + s;
      if (p >= a.P) continue;
      const size_t o = ((size_t)p * ne + e) * N + nn;
      auto cget = [&](int m) -> cd {
        const cT v = buf[s * M + m];
        return mk((double)v.x, (double)v.y);
      };
      if (r.mode == 0) {
        st2(out + o, cget(nn));
        continue;
      }
      cd Ft = mk(0.0, 0.0), MX = mk(0.0, 0.0), B = mk(0.0, 0.0);
      if (active_at(a, pb, s) && nn <= N - 2) {
        const double cnn = nn == 0 ? 1.0 : 0.5;
        Ft = scale(cget(nn), cnn);
        if (nn + 2 < N) Ft = Ft - scale(cget(nn + 2), 0.5);
        MX = scale(mk(x0[u].x, x0[u].y), cnn) - scale(mk(x2[u].x, x2[u].y), 0.5);
        if constexpr (RK) {
          rk_finish(r.rk, o, rv[u], make_double2(Ft.x, Ft.y), make_double2(MX.x, MX.y), out);
          continue;
        }
        B = scale(Ft, r.c1) - scale(MX, r.a1);
        if (r.has_hist) B = B + scale(mk(fo[u].x, fo[u].y), r.c2) - scale(mk(mo[u].x, mo[u].y), r.a2);
      }
      if constexpr (RK) {  // inactive pencil or row N - 1
        st2(out + o, B);
        continue;
      }
      const size_t ho = (((size_t)p * 2) * ne + e) * N + nn;
      st2(r.hist_cur + ho, Ft);
      st2(r.hist_cur + ho + (size_t)ne * N, MX);
      st2(out + o, B);
    }
  }
}

// ---------------------------------------------------------------------------
// y pass (3-D): complex transforms along y of TK consecutive kx columns per
// block, one (field, z level) per (blockIdx.z, blockIdx.y).  Stored y slots
// iy hold the signed wavenumbers 0..Ny/2-1, [Nyquist, held zero],
// -Ny/2+1..-1; on the padded grid of Ngy points they sit at position k
// (k >= 0) or Ngy + k (k < 0).
//   dir +1 (backward): In[f][jz][iy][kx] -> Out[f][jz][l][kx] = sum_k c_k e^{+2 pi i k l / Ngy}
//   dir -1 (forward):  In[f][jz][l][kx]  -> Out[f][jz][iy][kx] = (1/Ngy) sum_l g_l e^{-2 pi i k l / Ngy},
//                      truncated to the stored slots; Nyquist slots (iy = Ny/2 or kx >= Pa) zero.
// ---------------------------------------------------------------------------
// ys (0: the default above) replaces the output scale: 1 / Ngy of the forward
// transform, 1 of the backward one (the adjoint grid transforms use the
// other's).
// NGC > 0: Ngy = NGC fixed at compile time, TK = PB / NGC (PB points per
// block, PB / 256 per thread).
// ym (backward pass): output field f from input field ym.src[f], times i ky
// where ym.der[f] (y derivatives formed here, after the z transform).
template <int DIR, int MAXBF, typename T, int NGC = 0, int PB = 3072>
__global__ void __launch_bounds__(256) ypass_kernel(XformArgs a,
                                                    const typename V2<T>::type* __restrict__ In,
                                                    typename V2<T>::type* __restrict__ Out, int TKr,
                                                    double ys, YMap ym) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  cT* buf = (cT*)smem;
  const int TK = NGC > 0 ? PB / NGC : TKr;
  // Blocks go to the eight XCDs (each with its own L2) in turn by linear
  // index; the neighbouring kx tiles of a row share the cache lines at their
  // ends (rows of Px values are not line-aligned), so the linear index is
  // remapped to give each XCD a contiguous range of tiles.
  int bx = blockIdx.x, jz = blockIdx.y, f = blockIdx.z;
  {
    const int nbx = gridDim.x, nby = gridDim.y, total = nbx * nby * gridDim.z;
    if (total % 8 == 0) {
      int lin = bx + nbx * (jz + nby * f);
      lin = (lin & 7) * (total >> 3) + (lin >> 3);
      bx = lin % nbx;
      lin /= nbx;
      jz = lin % nby;
      f = lin / nby;
    }
  }
  const int k0 = bx * TK;
  const int Ny = a.Ny, Ng = NGC > 0 ? NGC : a.Ngy, Px = a.Px, M = a.M, half = Ny / 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t inRows = DIR > 0 ? Ny : Ng, outRows = DIR > 0 ? Ng : Ny;
  const int fin = ym.n ? ym.src[f] : f;
  const bool dy = DIR > 0 && ym.n && ym.der[f];
  const typename V2<T>::type* src = In + ((size_t)fin * M + jz) * inRows * Px;
  typename V2<T>::type* dst = Out + ((size_t)f * M + jz) * outRows * Px;
  // padded position -> stored slot (-1: padding or Nyquist)
  auto slot_of = [&](int pos) -> int {
    if (pos < half) return pos;
    if (pos > Ng - half) return Ny + (pos - Ng);
    return -1;
  };
  auto load = [&](int idx) -> cT {
    const int pos = idx / TK, s = idx - pos * TK;  // consecutive threads: consecutive kx
    const int kx = k0 + s;
    cT v = mk<T>(0, 0);
    if (kx < Px) {
      if (DIR > 0) {
        const int iy = slot_of(pos);
        if (iy >= 0) {
          v = ldv<T>(src + (size_t)iy * Px + kx);
          if (dy) {  // i ky v
            const T ky = (T)(a.two_pi_over_Ly * (double)(iy < half ? iy : iy - Ny));
            v = mk<T>(-ky * v.y, ky * v.x);
          }
        }
      } else {
        v = ldv<T>(src + (size_t)pos * Px + kx);
      }
    }
    return v;
  };
  if constexpr (NGC > 0) {
    // TK * Ng = PB points, PB / 256 per thread: every load issued before
    // the first LDS store, so that their latencies overlap
    constexpr int EPT = PB / 256;
    cT v[EPT];
#pragma unroll
    for (int it = 0; it < EPT; ++it) v[it] = load(tid + it * 256);
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
      const int idx = tid + it * 256, pos = idx / TK, s = idx - pos * TK;
      buf[s * Ng + pos] = v[it];
    }
  } else {
    for (int idx = tid; idx < TK * Ng; idx += nt) {
      const int pos = idx / TK, s = idx - pos * TK;
      buf[s * Ng + pos] = load(idx);
    }
  }
  __syncthreads();
  if constexpr (sizeof(T) == 8)
    fft_lds_c<NGC, DIR, MAXBF, T, true, true>(buf, Ng, TK, (const cT*)a.twy, tid, nt);
  else
    fft_lds_c<NGC, DIR, MAXBF, T, true, true>(buf, Ng, TK, (const cT*)a.twy32, tid, nt);
  if (DIR > 0) {
    for (int idx = tid; idx < TK * Ng; idx += nt) {
      const int l = idx / TK, s = idx - l * TK;
      const int kx = k0 + s;
      if (kx < Px) stv<T>(dst + (size_t)l * Px + kx, ys != 0.0 ? scale(buf[s * Ng + l], (T)ys) : buf[s * Ng + l]);
    }
  } else {
    const T inv = ys != 0.0 ? (T)ys : (T)1 / (T)Ng;
    for (int idx = tid; idx < TK * Ny; idx += nt) {
      const int iy = idx / TK, s = idx - iy * TK;
      const int kx = k0 + s;
      if (kx >= Px) continue;
      cT v = mk<T>(0, 0);
      if (iy != half && kx < a.Pa) {
        const int pos = iy < half ? iy : Ng + (iy - Ny);
        v = scale(buf[s * Ng + pos], inv);
      }
      stv<T>(dst + (size_t)iy * Px + kx, v);
    }
  }
}

// ---------------------------------------------------------------------------
// Initial state: scale-1 forward x transform of the b grid (one z level per
// block), then the z forward transform (zf_kernel, mode 0) and the fill below.
// ---------------------------------------------------------------------------
template <int MAXBF>
__global__ void __launch_bounds__(256) ic_x_kernel(XformArgs a, const double* __restrict__ bgrid,
                                                   double2* __restrict__ H1) {
  // one (z level jz, y level l) row per block; b grid [ix][l][jz] (Ny = 1 in 2-D);
  // output H1[jz][l][kx] with Px slots per row
  extern __shared__ double2 smem[];
  cd* buf = (cd*)smem;
  const int jz = blockIdx.x, l = blockIdx.y;
  const int Nx = a.Nx, N = a.N, Ny = a.dim == 2 ? 1 : a.Ny;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < Nx; i += nt) buf[i] = mk(bgrid[((size_t)i * Ny + l) * N + jz], 0.0);
  __syncthreads();
  fft_lds<-1, MAXBF>(buf, Nx, 1, (const cd*)a.twx, tid, nt);
  const double inv = 1.0 / (double)Nx;
  double2* out = H1 + ((size_t)jz * Ny + l) * a.Px;
  for (int k = tid; k < a.Px; k += nt) st2(out + k, k < a.Pa ? scale(buf[k], inv) : mk(0.0, 0.0));
}

// Right-hand side of the linear boundary value solve on the evolved-equation
// U-rows: Bev[p][e][n] = (P^L F)_n = c_n F_n - F_{n+2} / 2 (c_0 = 1, else 1/2)
// for n <= N - 2 of an active pencil, zero otherwise (T-to-U conversion,
// Appendix A).
__global__ void lbvp_rhs_kernel(XformArgs a, const double2* __restrict__ F, double2* __restrict__ Bev) {
  const int N = a.N, ne = a.ne;
  const size_t total = (size_t)a.P * ne * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int nn = (int)(i % N);
    const int p = (int)(i / ((size_t)ne * N));
    double2 v = make_double2(0.0, 0.0);
    if (active(a, p) && nn <= N - 2) {
      const double c = nn == 0 ? 1.0 : 0.5;
      const double2 f0 = F[i];
      v = make_double2(c * f0.x, c * f0.y);
      if (nn + 2 < N) {
        const double2 f2 = F[i + 2];
        v.x -= 0.5 * f2.x;
        v.y -= 0.5 * f2.y;
      }
    }
    Bev[i] = v;
  }
}

hipError_t launch_lbvp_rhs(const XformArgs& a, const void* F, void* Bev, hipStream_t st) {
  const size_t total = (size_t)a.P * a.ne * a.N;
  const int blocks = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  hipLaunchKernelGGL(lbvp_rhs_kernel, dim3(blocks), dim3(256), 0, st, a, (const double2*)F,
                     (double2*)Bev);
  return hipGetLastError();
}

// X[p][b] = c, X[p][bz] = d_z c (Chebyshev derivative recursion on [0, 1]),
// all other variables zero.
__global__ void ic_fill_kernel(XformArgs a, const double2* __restrict__ C, double2* __restrict__ X,
                               int vb, int vbz) {
  const int p = blockIdx.x;
  const int N = a.N, S = a.S;
  double2* Xp = X + (size_t)p * S * N;
  const double2* c = C + (size_t)p * N;
  for (int i = threadIdx.x; i < S * N; i += blockDim.x) {
    const int v = i / N;
    if (v == vbz) continue;
    Xp[i] = v == vb ? c[i - v * N] : make_double2(0.0, 0.0);
  }
  if (threadIdx.x == 0) {
    double2* dz = Xp + (size_t)vbz * N;
    double2 dn2 = make_double2(0.0, 0.0), dn1 = make_double2(0.0, 0.0);  // d_{n+2}, d_{n+1}
    for (int n = N - 1; n >= 0; --n) {
      double2 dn = make_double2(0.0, 0.0);
      if (n <= N - 2) {
        const double2 cn1 = c[n + 1];
        dn = make_double2(dn2.x + 2.0 * (n + 1) * cn1.x, dn2.y + 2.0 * (n + 1) * cn1.y);
      }
      if (n == 0) dn = make_double2(0.5 * dn.x, 0.5 * dn.y);
      dz[n] = make_double2(2.0 * dn.x, 2.0 * dn.y);  // d/dz = 2 d/dzeta
      dn2 = dn1;
      dn1 = dn;
    }
  }
}

// ---------------------------------------------------------------------------
// Kinetic energy: per dealiased row r (z level, and y level in 3-D), mean
// over x of |u|^2 / 2 from complex-to-real transforms of the velocity
// components (u, w in 2-D; u, v, w in 3-D).  Field f of row r at
// G + (f * R + r) * Px, R = M * Ngy.
// ---------------------------------------------------------------------------
template <int MAXBF, int PTS>
__global__ void __launch_bounds__(1024) ke_row_kernel(XformArgs a, const double2* __restrict__ G,
                                                      int nf, double* __restrict__ rowmean) {
  extern __shared__ double2 smem[];
  cd* buf = (cd*)smem;
  __shared__ double red[1024];
  const int r = blockIdx.x;
  const int L = a.L, Pa = a.Pa, Px = a.Px;
  const size_t R = (size_t)a.M * a.Ngy;
  const int tid = threadIdx.x, nt = blockDim.x;
  double acc = 0.0;
  for (int f0 = 0; f0 < nf; f0 += 2) {
    const double2* A = G + ((size_t)f0 * R + r) * Px;
    const double2* B = f0 + 1 < nf ? G + ((size_t)(f0 + 1) * R + r) * Px : nullptr;
    for (int k = tid; k < L; k += nt) {
      cd z = mk(0.0, 0.0);
      const int kk = k < Pa ? k : (k > L - Pa ? L - k : -1);
      if (kk >= 0) {
        cd Ak = ld2(A + kk), Bk = B ? ld2(B + kk) : mk(0.0, 0.0);
        if (kk == 0) {
          Ak.y = 0.0;
          Bk.y = 0.0;
        }
        z = k < Pa ? mk(Ak.x - Bk.y, Ak.y + Bk.x) : mk(Ak.x + Bk.y, -Ak.y + Bk.x);
      }
      buf[k] = z;
    }
    __syncthreads();
    fft_lds<+1, MAXBF>(buf, L, 1, (const cd*)a.twx, tid, nt);
    for (int i = tid; i < L; i += nt) acc += 0.5 * (buf[i].x * buf[i].x + buf[i].y * buf[i].y);
    __syncthreads();
  }
  red[tid] = acc;
  __syncthreads();
  for (int s = nt / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) rowmean[r] = red[0] / (double)L;
}

// mean over the Ngy y levels of each z level (3-D), as complex values for the
// z forward transform
__global__ void ke_ymean_kernel(const double* __restrict__ rowmean, double2* __restrict__ h, int M,
                                int Ngy) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int l = 0; l < Ngy; ++l) acc += rowmean[(size_t)j * Ngy + l];
    h[j] = make_double2(acc / (double)Ngy, 0.0);
  }
}

// J = sum_{m even < N} c_m / (1 - m^2) from the Chebyshev coefficients c of
// the x-mean (integration over z in [0, 1]: half the [-1, 1] integral).
__global__ void ke_sum_kernel(const double2* __restrict__ c, int N, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int m = threadIdx.x; m < N; m += blockDim.x)
    if ((m & 1) == 0) acc += c[m].x / (1.0 - (double)m * (double)m);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_zb(const XformArgs& a, const FieldList& fl, const void* X, void* G,
                     hipStream_t st, bool fp32, bool active_only) {
  int TP = z_tile(a.M);
  if (TP * a.M != kZPts) return hipErrorInvalidValue;
  const int plaunch = active_only && a.dim == 2 ? a.Pa : a.P;
  const int dv = z_split((plaunch + TP - 1) / TP * fl.nf, a.M);
  TP /= dv;
  const int pts = kZPts / dv;
  dim3 grid((plaunch + TP - 1) / TP, fl.nf);
  auto go = [&](auto kern, auto g) {
    const size_t lds = (size_t)(pts + 2 * a.M) * sizeof(*g);
    allow_lds((const void*)kern, lds);
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, a, fl, (const double2*)X, g, TP);
  };
  // the workloads' dealiased lengths (Nz = 64, 128, 256) with M fixed at compile time
  auto pick = [&](auto tc, auto g) {
    using TT = typename decltype(tc)::type;
    if (a.M == 192) {
      if (dv == 2) go(zb_kernel<3, TT, kZEpt / 2, 192>, g);
      else go(zb_kernel<3, TT, kZEpt, 192>, g);
    } else if (a.M == 384) {
      if (dv == 2) go(zb_kernel<3, TT, kZEpt / 2, 384>, g);
      else go(zb_kernel<3, TT, kZEpt, 384>, g);
    } else if (a.M == 96) {
      if (dv == 2) go(zb_kernel<3, TT, kZEpt / 2, 96>, g);
      else go(zb_kernel<3, TT, kZEpt, 96>, g);
    } else {
      if (dv == 2) go(zb_kernel<3, TT, kZEpt / 2>, g);
      else go(zb_kernel<3, TT>, g);
    }
  };
  if (fp32) pick(std::common_type<float>(), (float2*)G);
  else pick(std::common_type<double>(), (double2*)G);
  return hipGetLastError();
}

hipError_t launch_zf(const XformArgs& a, const void* H, void* out, const RhsArgs& r,
                     hipStream_t st, bool fp32) {
  int TP = z_tile(a.M);
  if (TP * a.M != kZPts || TP * a.N > 12 * kZThreads) return hipErrorInvalidValue;
  const int plaunch = (a.dim == 2 && r.mode >= 1) ? a.Pa : a.P;
  const int dv = z_split((plaunch + TP - 1) / TP * a.ne, a.M);
  TP /= dv;
  const int pts = kZPts / dv;
  dim3 grid((plaunch + TP - 1) / TP, a.ne);
  // the Runge-Kutta stage epilogue is a separate instantiation, so the SBDF
  // kernel carries none of its code
  auto go = [&](auto kern, auto h) {
    const size_t lds = (size_t)(pts + 2 * a.M) * sizeof(*h);
    allow_lds((const void*)kern, lds);
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, a, h, (double2*)out, r, TP);
  };
  const float2* h32 = (const float2*)H;
  const double2* h64 = (const double2*)H;
  // the workloads' (M, N) = (96, 64), (192, 128), (384, 256) fixed at compile
  // time, with the epilogue's points per thread (TP N / threads: 8 for full
  // tiles at M = 3N/2, 4 for half tiles); other lengths (the scale-1
  // transforms, M = N) up to 12 and 8
  auto pick = [&](auto tc, auto rk, auto h) {
    using TT = typename decltype(tc)::type;
    constexpr bool RKv = decltype(rk)::value;
    if (a.M == 192 && a.N == 128) {
      if (dv == 2) go(zf_kernel<3, 4, TT, RKv, kZEpt / 2, 192, 128>, h);
      else go(zf_kernel<3, 8, TT, RKv, kZEpt, 192, 128>, h);
    } else if (a.M == 384 && a.N == 256) {
      if (dv == 2) go(zf_kernel<3, 4, TT, RKv, kZEpt / 2, 384, 256>, h);
      else go(zf_kernel<3, 8, TT, RKv, kZEpt, 384, 256>, h);
    } else if (a.M == 96 && a.N == 64) {
      if (dv == 2) go(zf_kernel<3, 4, TT, RKv, kZEpt / 2, 96, 64>, h);
      else go(zf_kernel<3, 8, TT, RKv, kZEpt, 96, 64>, h);
    } else {
      if (dv == 2) go(zf_kernel<3, 8, TT, RKv, kZEpt / 2>, h);
      else go(zf_kernel<3, 12, TT, RKv>, h);
    }
  };
  using tf = std::common_type<float>;
  using td = std::common_type<double>;
  if (fp32) {
    if (r.mode == 2) pick(tf(), std::true_type(), h32);
    else pick(tf(), std::false_type(), h32);
  } else {
    if (r.mode == 2) pick(td(), std::true_type(), h64);
    else pick(td(), std::false_type(), h64);
  }
  return hipGetLastError();
}


hipError_t launch_ypass(const XformArgs& a, int dir, int nf, const void* In, void* Out,
                        hipStream_t st, bool fp32, double ys, const YMap* map) {
  YMap ym{};
  if (map) ym = *map;
  // Ny = 256 (384 padded points) with the length fixed at compile time; FP64
  // tiles of 4 kx (1536 points, 24 KB of LDS: six blocks per compute unit
  // instead of three with tiles of 8)
  const bool c384 = a.Ngy == 384;
  const int pb = c384 && !fp32 ? 1536 : 3072;
  const int TK = a.Ngy >= pb ? 1 : pb / a.Ngy;
  dim3 grid((a.Px + TK - 1) / TK, a.M, nf);
  const size_t lds = (size_t)TK * a.Ngy * (fp32 ? sizeof(float2) : sizeof(double2));
  auto go = [&](auto kern, auto in, auto out) {
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, a, in, out, TK, ys, ym);
  };
  auto pick = [&](auto tc) {
    using TT = typename decltype(tc)::type;
    using S2 = typename V2<TT>::type;
    const S2* in = (const S2*)In;
    S2* out = (S2*)Out;
    if (c384) {
      if constexpr (sizeof(TT) == 8) {
        if (dir > 0) go(ypass_kernel<+1, 2, TT, 384, 1536>, in, out);
        else go(ypass_kernel<-1, 2, TT, 384, 1536>, in, out);
      } else {
        if (dir > 0) go(ypass_kernel<+1, 3, TT, 384>, in, out);
        else go(ypass_kernel<-1, 3, TT, 384>, in, out);
      }
    } else {
      if (dir > 0) go(ypass_kernel<+1, 3, TT>, in, out);
      else go(ypass_kernel<-1, 3, TT>, in, out);
    }
  };
  if (fp32) pick(std::common_type<float>());
  else pick(std::common_type<double>());
  return hipGetLastError();
}

// x-pass launch shape for an L-point row: NT ~ L/3 threads (one radix-4
// butterfly per thread per pass, MAXBF = 1), PTS = ceil(L / NT) points each;
// L = 6144 uses 1024 threads, 6 points, MAXBF = 2.  The twiddle table goes
// to LDS when it fits in 32 KB.
hipError_t launch_initial_state(const XformArgs& a1, const double* bgrid, void* X, void* work,
                                hipStream_t st) {
  // a1 describes the scale-1 transforms: M = N (z), twx of length Nx, L = Nx,
  // and in 3-D Ngy = Ny with the y table of length Ny.
  const int Ny = a1.dim == 2 ? 1 : a1.Ny;
  double2* H1 = (double2*)work;                           // [N][Ny][Px]
  double2* Hy = H1 + (size_t)a1.N * Ny * a1.Px;           // [N][P] (3-D)
  double2* C = Hy + (size_t)a1.N * a1.P;                  // [P][1][N]
  allow_lds((const void*)ic_x_kernel<8>, (size_t)a1.Nx * sizeof(double2));
  hipLaunchKernelGGL((ic_x_kernel<8>), dim3(a1.N, Ny), dim3(256), (size_t)a1.Nx * sizeof(double2),
                     st, a1, bgrid, H1);
  const double2* Hz = H1;
  if (a1.dim == 3) {
    hipError_t e = launch_ypass(a1, -1, 1, H1, Hy, st);
    if (e != hipSuccess) return e;
    Hz = Hy;
  }
  XformArgs az = a1;
  az.ne = 1;
  RhsArgs r{};
  r.mode = 0;
  hipError_t e = launch_zf(az, Hz, C, r, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ic_fill_kernel, dim3(a1.P), dim3(256), 0, st, a1, (const double2*)C,
                     (double2*)X, 1, a1.dim == 2 ? 4 : 5);
  return hipGetLastError();
}

hipError_t launch_ke(const XformArgs& a, const void* X, void* G, void* G2, double* rowmean,
                     double* out, hipStream_t st) {
  const int nf = a.dim == 2 ? 2 : 3;
  FieldList fl{};
  fl.nf = nf;
  fl.var[0] = 2;                    // u
  fl.var[1] = 3;                    // w (2-D) / v (3-D)
  fl.var[2] = 4;                    // w (3-D)
  launch_zb(a, fl, X, G, st);
  const void* Gr = G;
  if (a.dim == 3) {
    hipError_t e = launch_ypass(a, +1, nf, G, G2, st);
    if (e != hipSuccess) return e;
    Gr = G2;
  }
  const int nt = x_threads(a.L);
  const int rows = a.M * (a.dim == 2 ? 1 : a.Ngy);
  allow_lds((const void*)ke_row_kernel<2, 6>, (size_t)a.L * sizeof(double2) + 8192);
  hipLaunchKernelGGL((ke_row_kernel<2, 6>), dim3(rows), dim3(nt), (size_t)a.L * sizeof(double2),
                     st, a, (const double2*)Gr, nf, rowmean);
  // z forward of the (real) x[y]-means: one pencil, one field
  XformArgs az = a;
  az.P = 1;
  az.ne = 1;
  az.dim = 2;
  az.Pa = 1;
  double2* H = (double2*)G;            // reuse: [1][M][1]
  double2* C = H + a.M;                // [1][1][N]
  hipLaunchKernelGGL(ke_ymean_kernel, dim3(1), dim3(256), 0, st, (const double*)rowmean, H, a.M,
                     a.dim == 2 ? 1 : a.Ngy);
  RhsArgs r{};
  r.mode = 0;
  hipError_t e = launch_zf(az, H, C, r, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ke_sum_kernel, dim3(1), dim3(256), 0, st, (const double2*)C, a.N, out);
  return hipGetLastError();
}

}  // namespace stau
