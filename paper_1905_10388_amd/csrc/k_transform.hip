// Spectral transform kernels (Sec. IV): Chebyshev z transforms as DCT-III /
// DCT-II through one complex FFT of the dealiased length M per column (the
// Gauss grid is ascending, so T_n(z_j) = (-1)^n cos(pi n (2j+1) / (2M))), and
// the fused x pass (complex-to-real, grid products, real-to-complex) with two
// real rows packed into each complex FFT.
//
// Layouts (2-D; P = Nx/2 + 1 pencil slots, Pa = Nx/2 active):
//   state X[p][var][n]          complex, n < N
//   G[f][jz][p]                 complex, after the z backward transform
//   H[e][jz][p]                 complex, explicit term before the z forward
//   F / Bev[p][e][n]            complex
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
constexpr int kZBlocksPerCU = 3;  // half-size tiles below this many full-size blocks per CU

template <typename T>
__device__ __forceinline__ void stage_z_tables(const XformArgs& a, cpx<T>* twl, cpx<T>* dcl, int M,
                                               int tid) {
  for (int i = tid; i < M; i += kZThreads) {
    twl[i] = tw_of<T>(a, a.twz, a.twz32, i);
    dcl[i] = tw_of<T>(a, a.dctz, a.dctz32, i);
  }
}

// ---------------------------------------------------------------------------
// Backward z (DCT-III with padding N -> M): g_j = sum_{n<N} c_n T_n(z_j)
// for every field of `fl` and TP pencils per block.
// ---------------------------------------------------------------------------
template <int MAXBF, typename T, int EPT = kZEpt>
__global__ void __launch_bounds__(kZThreads) zb_kernel(XformArgs a, FieldList fl,
                                                       const double2* __restrict__ X,
                                                       typename V2<T>::type* __restrict__ G, int TP) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  const int M = a.M, N = a.N, S = fl.src_S ? fl.src_S : a.S;
  cT* buf = (cT*)smem;
  cT* twl = buf + EPT * kZThreads;  // FFT twiddles
  cT* dcl = twl + M;      // DCT twiddles
  const int f = blockIdx.y;
  const int p0 = blockIdx.x * TP;
  const int var = fl.var[f], der = fl.deriv[f];
  const double wfac = fl.wmode ? 2.0 / (double)M : 1.0;  // (2 - delta_n0) / M, n > 0
  const int tid = threadIdx.x;
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
    if (active(a, p)) {
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
    const int p = p0 + s;
    cT z = mk<T>(0, 0);
    if (active(a, p)) {
      double kk = 0.0;
      if (der == 1) kk = kx_of(a, p);
      if (der == 2) kk = ky_of(a, p);
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
  fft_lds<+1, MAXBF>(buf, M, TP, (const cT*)twl, tid, kZThreads);
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
template <int MAXBF, int MAXIT, typename T, bool RK = false, int EPT = kZEpt>
__global__ void __launch_bounds__(kZThreads) zf_kernel(XformArgs a,
                                                       const typename V2<T>::type* __restrict__ H,
                                                       double2* __restrict__ out, RhsArgs r, int TP) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  const int M = a.M, N = a.N, ne = a.ne;
  cT* buf = (cT*)smem;
  cT* twl = buf + EPT * kZThreads;
  cT* dcl = twl + M;
  const int e = blockIdx.y;
  const int p0 = blockIdx.x * TP;
  const int tid = threadIdx.x, nt = kZThreads;
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
  fft_lds<-1, MAXBF>(buf, M, TP, (const cT*)twl, tid, nt);
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
  // epilogue in groups of four points per thread: the group's loads first
  constexpr int GE = 4;
  static_assert(MAXIT % GE == 0, "epilogue groups");
#pragma unroll
  for (int g0 = 0; g0 < MAXIT; g0 += GE) {
    double2 x0[GE], x2[GE], fo[GE], mo[GE];
    RkRow rv[RK ? GE : 1];
#pragma unroll
    for (int u = 0; u < GE; ++u) {
      const int idx = tid + (g0 + u) * nt;
      x0[u] = x2[u] = fo[u] = mo[u] = make_double2(0.0, 0.0);
      if (r.mode >= 1 && idx < TP * N) {
        const int s = idx / N, nn = idx - s * N;
        const int p = p0 + s;
        if (active(a, p) && nn <= N - 2) {
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
      if (active(a, p) && nn <= N - 2) {
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
template <int DIR, int MAXBF, typename T>
__global__ void __launch_bounds__(256) ypass_kernel(XformArgs a,
                                                    const typename V2<T>::type* __restrict__ In,
                                                    typename V2<T>::type* __restrict__ Out, int TK) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  cT* buf = (cT*)smem;
  const int f = blockIdx.z, jz = blockIdx.y, k0 = blockIdx.x * TK;
  const int Ny = a.Ny, Ng = a.Ngy, Px = a.Px, M = a.M, half = Ny / 2;
  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t inRows = DIR > 0 ? Ny : Ng, outRows = DIR > 0 ? Ng : Ny;
  const typename V2<T>::type* src = In + ((size_t)f * M + jz) * inRows * Px;
  typename V2<T>::type* dst = Out + ((size_t)f * M + jz) * outRows * Px;
  // padded position -> stored slot (-1: padding or Nyquist)
  auto slot_of = [&](int pos) -> int {
    if (pos < half) return pos;
    if (pos > Ng - half) return Ny + (pos - Ng);
    return -1;
  };
  for (int idx = tid; idx < TK * Ng; idx += nt) {
    const int pos = idx / TK, s = idx - pos * TK;  // consecutive threads: consecutive kx
    const int kx = k0 + s;
    cT v = mk<T>(0, 0);
    if (kx < Px) {
      if (DIR > 0) {
        const int iy = slot_of(pos);
        if (iy >= 0) v = ldv<T>(src + (size_t)iy * Px + kx);
      } else {
        v = ldv<T>(src + (size_t)pos * Px + kx);
      }
    }
    buf[s * Ng + pos] = v;
  }
  __syncthreads();
  if constexpr (sizeof(T) == 8)
    fft_lds<DIR, MAXBF>(buf, Ng, TK, (const cT*)a.twy, tid, nt);
  else
    fft_lds<DIR, MAXBF>(buf, Ng, TK, (const cT*)a.twy32, tid, nt);
  if (DIR > 0) {
    for (int idx = tid; idx < TK * Ng; idx += nt) {
      const int l = idx / TK, s = idx - l * TK;
      const int kx = k0 + s;
      if (kx < Px) stv<T>(dst + (size_t)l * Px + kx, buf[s * Ng + l]);
    }
  } else {
    const T inv = (T)1 / (T)Ng;
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
// Fused x pass for one dealiased row r (a z level; in 3-D a (z, y) level):
// packed complex-to-real transforms of field pairs, the grid products
//   N_q = -(u q_x [+ v q_y] + w q_z),
// and packed real-to-complex transforms truncated to k < Nx/2 and scaled 1/L.
// Field f of row r sits at G + (f R + r) Px with R = M Ngy (Ngy = 1 in 2-D).
//   2-D fields: u, w, b_x, b_z, u_x, u_z, w_x, w_z           -> N_b, N_u, N_w
//   3-D fields: u, v, w, b_x, b_y, b_z, u_x, u_y, u_z, v_x, v_y, v_z, w_x,
//               w_y, w_z                                     -> N_b, N_u, N_v, N_w
// Each pair's half spectrum is loaded into registers one pair ahead of its
// transform; with TWL the twiddle table is staged in LDS once per block.
// Thread t owns grid points t + q NT, q < PTS.  SPLIT (2-D, for launches with
// fewer rows than compute units): two blocks per row, blockIdx.y = 0 forms
// N_b and N_u from the pairs (u, w), (b_x, b_z), (u_x, u_z), blockIdx.y = 1
// forms N_w from (u, w), (w_x, w_z).
// ---------------------------------------------------------------------------
template <int DIM, int NT, int PTS, int MAXBF, bool TWL, typename T, bool SPLIT = false>
__global__ void __launch_bounds__(NT) xrow_kernel(XformArgs a,
                                                  const typename V2<T>::type* __restrict__ G,
                                                  typename V2<T>::type* __restrict__ H) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  using S2 = typename V2<T>::type;
  constexpr int KPT = (PTS + 2) / 3;  // half-spectrum entries per thread (Pa = L / 3)
  constexpr int NP = DIM == 2 ? 4 : 8;
  cT* buf = (cT*)smem;
  const int r = blockIdx.x;
  const int L = a.L, Pa = a.Pa, Px = a.Px;
  const size_t R = (size_t)a.M * a.Ngy;
  const int tid = threadIdx.x;
  const cT* twg = (const cT*)(sizeof(T) == 8 ? (const void*)a.twx : (const void*)a.twx32);
  cT* twl = buf + L;
  if constexpr (TWL) {
    for (int i = tid; i < L; i += NT) twl[i] = twg[i];
  }
  const cT* tw = TWL ? (const cT*)twl : twg;

  // pair k: fields (fa, fb); fb < 0 means zero
  auto pair_fields = [](int k, int& fa, int& fb) {
    fa = 2 * k;
    fb = 2 * k + 1;
    if (DIM == 3 && k == 7) fb = -1;
  };
  cT sa[KPT], sb[KPT];
  auto fetch = [&](int k) {
    int fa, fb;
    pair_fields(k, fa, fb);
    const S2* A = G + ((size_t)fa * R + r) * Px;
    const S2* B = G + ((size_t)(fb < 0 ? fa : fb) * R + r) * Px;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      sa[q] = mk<T>(0, 0);
      sb[q] = mk<T>(0, 0);
      if (kk < Pa) {
        sa[q] = ldv<T>(A + kk);
        if (fb >= 0) sb[q] = ldv<T>(B + kk);
      }
    }
  };
  // Hermitian extension of the packed pair A + i B onto the L-point grid
  auto scatter = [&]() {
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      if (kk < Pa) {
        cT Ak = sa[q], Bk = sb[q];
        if (kk == 0) {
          Ak.y = 0;
          Bk.y = 0;
        }
        buf[kk] = mk<T>(Ak.x - Bk.y, Ak.y + Bk.x);
        if (kk > 0) buf[L - kk] = mk<T>(Ak.x + Bk.y, -Ak.y + Bk.x);
      }
    }
    for (int k = Pa + tid; k <= L - Pa; k += NT) buf[k] = mk<T>(0, 0);
  };

  T u[PTS], v[PTS], w[PTS], nb[PTS], nu[PTS], nv[PTS], nw[PTS];
  // pairs of this block: all NP, or for SPLIT (0, 1, 2) / (0, 3)
  const int part = SPLIT ? (int)blockIdx.y : 0;
  const int npr = SPLIT ? (part == 0 ? 3 : 2) : NP;
  auto pair_of = [&](int k) { return SPLIT && part == 1 && k == 1 ? 3 : k; };
  fetch(0);
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (k >= npr) break;
    const int pk = pair_of(k);
    scatter();
    if (k + 1 < npr) fetch(pair_of(k + 1));
    __syncthreads();
    fft_lds<+1, MAXBF, T, DIM == 2>(buf, L, 1, tw, tid, NT);
#pragma unroll
    for (int q = 0; q < PTS; ++q) {
      const int i = tid + q * NT;
      if (i < L) {
        const T x = buf[i].x, y = buf[i].y;  // the pair's two real fields at point i
        if constexpr (DIM == 2) {
          if (pk == 0) { u[q] = x; w[q] = y; }
          if (pk == 1) nb[q] = -(u[q] * x + w[q] * y);
          if (pk == 2) nu[q] = -(u[q] * x + w[q] * y);
          if (pk == 3) nw[q] = -(u[q] * x + w[q] * y);
        } else {
          if (k == 0) { u[q] = x; v[q] = y; }
          if (k == 1) { w[q] = x; nb[q] = -(u[q] * y); }
          if (k == 2) nb[q] -= v[q] * x + w[q] * y;
          if (k == 3) nu[q] = -(u[q] * x + v[q] * y);
          if (k == 4) { nu[q] -= w[q] * x; nv[q] = -(u[q] * y); }
          if (k == 5) nv[q] -= v[q] * x + w[q] * y;
          if (k == 6) nw[q] = -(u[q] * x + v[q] * y);
          if (k == 7) nw[q] -= w[q] * x;
        }
      }
    }
    __syncthreads();
  }

  const T invL = (T)1 / (T)L;
  const T hf = (T)0.5;
  // packed real-to-complex: ra + i rb (rb null: a single real field)
  auto r2c = [&](const T* ra, const T* rb, int ea, int eb) {
#pragma unroll
    for (int q = 0; q < PTS; ++q) {
      const int i = tid + q * NT;
      if (i < L) buf[i] = mk<T>(ra[q], rb ? rb[q] : (T)0);
    }
    __syncthreads();
    fft_lds<-1, MAXBF, T, DIM == 2>(buf, L, 1, tw, tid, NT);
    S2* Ha = H + ((size_t)ea * R + r) * Px;
    S2* Hb = H + ((size_t)(eb < 0 ? ea : eb) * R + r) * Px;
    for (int k = tid; k < Px; k += NT) {
      cT A = mk<T>(0, 0), Bv = mk<T>(0, 0);
      if (k < Pa) {
        const cT Zk = buf[k];
        if (eb < 0) {
          A = scale(Zk, invL);
        } else {
          const cT Zm = buf[k == 0 ? 0 : L - k];
          A = mk<T>(hf * (Zk.x + Zm.x) * invL, hf * (Zk.y - Zm.y) * invL);
          Bv = mk<T>(hf * (Zk.y + Zm.y) * invL, -hf * (Zk.x - Zm.x) * invL);
        }
      }
      stv<T>(Ha + k, A);
      if (eb >= 0) stv<T>(Hb + k, Bv);
    }
    __syncthreads();
  };
  if constexpr (DIM == 2) {
    if (!SPLIT || part == 0) r2c(nb, nu, 0, 1);
    if (!SPLIT || part == 1) r2c(nw, nullptr, 2, -1);
  } else {
    r2c(nb, nu, 0, 1);
    r2c(nv, nw, 2, 3);
  }
}

// ---------------------------------------------------------------------------
// 2-D x pass with the field pairs transformed two at a time: the backward
// transforms of pairs (0, 1) and (2, 3), and the forward ones of (N_b, N_u)
// and N_w, each run as one batch of two sequences, so a row takes half the
// radix passes and barriers of one pair at a time (the passes are latency
// bound: a radix-8 pass of one 1536-point sequence keeps 192 of 512 threads
// busy).  Data [2][L] and twiddles [L] in LDS.  Same products and outputs as
// xrow_kernel<2>; SPLIT as there (part 0: pairs (0, 1), (2) and N_b, N_u;
// part 1: pairs (0, 3) and N_w).
// ---------------------------------------------------------------------------
template <int NT, int PTS, int MAXBF, typename T, bool SPLIT>
__global__ void __launch_bounds__(NT) xrow2_kernel(XformArgs a,
                                                   const typename V2<T>::type* __restrict__ G,
                                                   typename V2<T>::type* __restrict__ H) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  using S2 = typename V2<T>::type;
  constexpr int KPT = (PTS + 2) / 3;  // half-spectrum entries per thread (Pa = L / 3)
  cT* buf = (cT*)smem;                // two sequences of L points
  const int r = blockIdx.x;
  const int L = a.L, Pa = a.Pa, Px = a.Px;
  const size_t R = (size_t)a.M;
  const int tid = threadIdx.x;
  const cT* twg = (const cT*)(sizeof(T) == 8 ? (const void*)a.twx : (const void*)a.twx32);
  cT* twl = buf + 2 * L;
  for (int i = tid; i < L; i += NT) twl[i] = twg[i];
  const int part = SPLIT ? (int)blockIdx.y : 0;
  // the block's batches of pairs (-1: none): (0, 1), (2, 3); SPLIT part 0
  // (0, 1), (2); part 1 (0, 3)
  const bool p1 = SPLIT && part == 1;
  const int b01 = p1 ? 3 : 1, b10 = p1 ? -1 : 2, b11 = SPLIT ? -1 : 3;
  const int nbatch = p1 ? 1 : 2;
  cT sa[2][KPT], sb[2][KPT];
  auto fetch = [&](int slot, int k) {
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      sa[slot][q] = mk<T>(0, 0);
      sb[slot][q] = mk<T>(0, 0);
    }
    if (k < 0) return;
    const S2* A = G + ((size_t)(2 * k) * R + r) * Px;
    const S2* B = G + ((size_t)(2 * k + 1) * R + r) * Px;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      if (kk < Pa) {
        sa[slot][q] = ldv<T>(A + kk);
        sb[slot][q] = ldv<T>(B + kk);
      }
    }
  };
  // Hermitian extension of the packed pair A + i B onto sequence `slot`
  auto scatter = [&](int slot) {
    cT* bb = buf + slot * L;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      if (kk < Pa) {
        cT Ak = sa[slot][q], Bk = sb[slot][q];
        if (kk == 0) {
          Ak.y = 0;
          Bk.y = 0;
        }
        bb[kk] = mk<T>(Ak.x - Bk.y, Ak.y + Bk.x);
        if (kk > 0) bb[L - kk] = mk<T>(Ak.x + Bk.y, -Ak.y + Bk.x);
      }
    }
    for (int k = Pa + tid; k <= L - Pa; k += NT) bb[k] = mk<T>(0, 0);
  };

  T u[PTS], w[PTS], nb[PTS], nu[PTS], nw[PTS];
  auto take = [&](int pk, int q, T x, T y) {  // the pair's two real fields at point q
    if (pk == 0) {
      u[q] = x;
      w[q] = y;
    }
    if (pk == 1) nb[q] = -(u[q] * x + w[q] * y);
    if (pk == 2) nu[q] = -(u[q] * x + w[q] * y);
    if (pk == 3) nw[q] = -(u[q] * x + w[q] * y);
  };
  fetch(0, 0);
  fetch(1, b01);
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    if (bi >= nbatch) break;
    const int k0 = bi == 0 ? 0 : b10, k1 = bi == 0 ? b01 : b11;
    scatter(0);
    if (k1 >= 0) scatter(1);
    if (bi == 0 && nbatch == 2) {
      fetch(0, b10);
      fetch(1, b11);
    }
    __syncthreads();
    fft_lds<+1, MAXBF, T, true>(buf, L, k1 >= 0 ? 2 : 1, twl, tid, NT);
#pragma unroll
    for (int q = 0; q < PTS; ++q) {
      const int i = tid + q * NT;
      if (i < L) {
        const cT x0 = buf[i];
        take(k0, q, x0.x, x0.y);
        if (k1 >= 0) {
          const cT x1 = buf[L + i];
          take(k1, q, x1.x, x1.y);
        }
      }
    }
    __syncthreads();
  }

  // forward: sequence 0 = N_b + i N_u (part 0), sequence 1 (or 0) = N_w
  const bool f0 = !SPLIT || part == 0, f1 = !SPLIT || part == 1;
  const int s1 = f0 ? 1 : 0;
#pragma unroll
  for (int q = 0; q < PTS; ++q) {
    const int i = tid + q * NT;
    if (i < L) {
      if (f0) buf[i] = mk<T>(nb[q], nu[q]);
      if (f1) buf[s1 * L + i] = mk<T>(nw[q], (T)0);
    }
  }
  __syncthreads();
  fft_lds<-1, MAXBF, T, true>(buf, L, (f0 && f1) ? 2 : 1, twl, tid, NT);
  const T invL = (T)1 / (T)L;
  const T hf = (T)0.5;
  S2* H0 = H + (size_t)r * Px;
  S2* H1 = H + (R + r) * Px;
  S2* H2 = H + (2 * R + r) * Px;
  for (int k = tid; k < Px; k += NT) {
    cT A = mk<T>(0, 0), Bv = mk<T>(0, 0), Wv = mk<T>(0, 0);
    if (k < Pa) {
      if (f0) {
        const cT Zk = buf[k], Zm = buf[k == 0 ? 0 : L - k];
        A = mk<T>(hf * (Zk.x + Zm.x) * invL, hf * (Zk.y - Zm.y) * invL);
        Bv = mk<T>(hf * (Zk.y + Zm.y) * invL, -hf * (Zk.x - Zm.x) * invL);
      }
      if (f1) Wv = scale(buf[s1 * L + k], invL);
    }
    if (f0) {
      stv<T>(H0 + k, A);
      stv<T>(H1 + k, Bv);
    }
    if (f1) stv<T>(H2 + k, Wv);
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static int z_tile(int M) { return M >= 3072 ? 1 : 3072 / M; }
static int x_threads(int L) {
  int nt = (L + 5) / 6;
  nt = (nt + 63) / 64 * 64;
  if (nt < 64) nt = 64;
  if (nt > 1024) nt = 1024;
  return nt;
}

// Half-size z tiles (kZPts / 2 points, 6 per thread) when the full-size grid
// has fewer than kZBlocksPerCU blocks per compute unit: more, smaller blocks
// keep every unit busy (1024x256: z backward 28.2 -> 24.9 us, z forward 30.8 ->
// 25.7 us; quarter tiles measured no better).  Returns the divisor (1 or 2).
static int z_split(int blocks, int M, int per_cu = kZBlocksPerCU) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1;
  int d = 1;
  if (M <= kZPts / 2 && blocks < per_cu * cus) d = 2;
  return d;
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
  if (fp32) {
    if (dv == 2) go(zb_kernel<3, float, kZEpt / 2>, (float2*)G);
    else go(zb_kernel<3, float>, (float2*)G);
  } else {
    if (dv == 2) go(zb_kernel<3, double, kZEpt / 2>, (double2*)G);
    else go(zb_kernel<3, double>, (double2*)G);
  }
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
  auto pick = [&](auto tc, auto rk, auto h) {
    using TT = typename decltype(tc)::type;
    constexpr bool RKv = decltype(rk)::value;
    if (dv == 2) go(zf_kernel<3, 12, TT, RKv, kZEpt / 2>, h);
    else go(zf_kernel<3, 12, TT, RKv>, h);
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
                        hipStream_t st, bool fp32) {
  const int TK = a.Ngy >= 3072 ? 1 : 3072 / a.Ngy;
  dim3 grid((a.Px + TK - 1) / TK, a.M, nf);
  const size_t lds = (size_t)TK * a.Ngy * (fp32 ? sizeof(float2) : sizeof(double2));
  if (fp32) {
    if (dir > 0)
      hipLaunchKernelGGL((ypass_kernel<+1, 3, float>), grid, dim3(256), lds, st, a,
                         (const float2*)In, (float2*)Out, TK);
    else
      hipLaunchKernelGGL((ypass_kernel<-1, 3, float>), grid, dim3(256), lds, st, a,
                         (const float2*)In, (float2*)Out, TK);
  } else {
    if (dir > 0)
      hipLaunchKernelGGL((ypass_kernel<+1, 3, double>), grid, dim3(256), lds, st, a,
                         (const double2*)In, (double2*)Out, TK);
    else
      hipLaunchKernelGGL((ypass_kernel<-1, 3, double>), grid, dim3(256), lds, st, a,
                         (const double2*)In, (double2*)Out, TK);
  }
  return hipGetLastError();
}

// x-pass launch shape for an L-point row: NT ~ L/3 threads (one radix-4
// butterfly per thread per pass, MAXBF = 1), PTS = ceil(L / NT) points each;
// L = 6144 uses 1024 threads, 6 points, MAXBF = 2.  The twiddle table goes
// to LDS when it fits in 32 KB.
template <int DIM, int NT, int PTS, int MAXBF, typename T>
static hipError_t launch_xrow_t(const XformArgs& a, const void* G, void* H, hipStream_t st) {
  using S2 = typename V2<T>::type;
  const int rows = a.M * (DIM == 2 ? 1 : a.Ngy);
  const bool twl = (size_t)a.L * sizeof(S2) <= 32768;
  const size_t lds = (size_t)a.L * sizeof(S2) * (twl ? 2 : 1);
  // 2-D rows fewer than compute units (FP32: fewer than twice as many): two
  // blocks per row.  (Measured at 1536 x 384 points: FP32 27.8 -> 21.6 us
  // split; FP64 37.8 -> 41.3 us, so FP64 keeps one block per row there.)
  int dev = 0, cus = 0;
  const bool split = DIM == 2 && hipGetDevice(&dev) == hipSuccess &&
                     hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                     rows < (sizeof(T) == 4 ? 2 * cus : cus);
  const dim3 grid(rows, split ? 2 : 1);
  // 2-D: pairs two at a time when two sequences and the twiddles fit 80 KB
  if constexpr (DIM == 2) {
    const size_t lds2 = (size_t)3 * a.L * sizeof(S2);
    if (lds2 <= 80 * 1024) {
      auto fn = split ? xrow2_kernel<NT, PTS, 2 * MAXBF, T, true> : xrow2_kernel<NT, PTS, 2 * MAXBF, T, false>;
      allow_lds((const void*)fn, lds2);
      hipLaunchKernelGGL(fn, grid, dim3(NT), lds2, st, a, (const S2*)G, (S2*)H);
      return hipGetLastError();
    }
  }
  if (twl) {
    auto fn = split ? xrow_kernel<DIM, NT, PTS, MAXBF, true, T, true> : xrow_kernel<DIM, NT, PTS, MAXBF, true, T, false>;
    allow_lds((const void*)fn, lds);
    hipLaunchKernelGGL(fn, grid, dim3(NT), lds, st, a, (const S2*)G, (S2*)H);
  } else {
    auto fn = split ? xrow_kernel<DIM, NT, PTS, MAXBF, false, T, true> : xrow_kernel<DIM, NT, PTS, MAXBF, false, T, false>;
    allow_lds((const void*)fn, lds);
    hipLaunchKernelGGL(fn, grid, dim3(NT), lds, st, a, (const S2*)G, (S2*)H);
  }
  return hipGetLastError();
}

template <int DIM, typename T>
static hipError_t launch_xrow_T(const XformArgs& a, const void* G, void* H, hipStream_t st) {
  const int L = a.L;
  if (L <= 64) return launch_xrow_t<DIM, 64, 1, 1, T>(a, G, H, st);
  if (L <= 128) return launch_xrow_t<DIM, 64, 2, 1, T>(a, G, H, st);
  if (L <= 192) return launch_xrow_t<DIM, 64, 3, 1, T>(a, G, H, st);
  if (L <= 384) return launch_xrow_t<DIM, 128, 3, 1, T>(a, G, H, st);
  if (L <= 768) return launch_xrow_t<DIM, 256, 3, 1, T>(a, G, H, st);
  if (L <= 1536) return launch_xrow_t<DIM, 512, 3, 1, T>(a, G, H, st);
  if (L <= 3072) return launch_xrow_t<DIM, 1024, 3, 1, T>(a, G, H, st);
  if (L <= 6144) return launch_xrow_t<DIM, 1024, 6, 2, T>(a, G, H, st);
  return hipErrorInvalidValue;
}

hipError_t launch_xpass(const XformArgs& a, const void* G, void* H, hipStream_t st, bool fp32) {
  return fp32 ? launch_xrow_T<2, float>(a, G, H, st) : launch_xrow_T<2, double>(a, G, H, st);
}

hipError_t launch_xpass3(const XformArgs& a, const void* G2, void* H2, hipStream_t st, bool fp32) {
  return fp32 ? launch_xrow_T<3, float>(a, G2, H2, st) : launch_xrow_T<3, double>(a, G2, H2, st);
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
  launch_zf(az, Hz, C, r, st);
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
  launch_zf(az, H, C, r, st);
  hipLaunchKernelGGL(ke_sum_kernel, dim3(1), dim3(256), 0, st, (const double2*)C, a.N, out);
  return hipGetLastError();
}

}  // namespace stau
