// Fused x pass of the explicit term (Sec. IV "Scaled transforms &
// dealiasing", Sec. VII "Arithmetic operators"): per dealiased row, packed
// complex-to-real transforms of the grid fields, the products, and packed
// real-to-complex transforms truncated to the stored modes (2-D and 3-D).
#include "xform.h"

namespace stau {

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
// The grid fields of pair k as (source field of G, x-derivative flag) for
// its real and imaginary parts.  G holds the z (and y) transforms of the
// state fields without their x derivatives (2-D: u, w, b, bz, uz, wz; 3-D: u,
// v, w, b, b_y, bz, u_y, uz, v_y, vz, w_y, wz): q_x is i kx times q's row,
// formed here, since the x derivative commutes with the z and y transforms.
//   2-D pairs: (u, w), (b_x, bz), (u_x, uz), (w_x, wz)
//   3-D pairs: (u, v), (w, b_x), (b_y, bz), (u_x, u_y), (uz, v_x), (v_y, vz),
//              (w_x, w_y), (wz, -)
template <int DIM>
__device__ __forceinline__ void pair_src(int k, int& fa, int& da, int& fb, int& db) {
  if constexpr (DIM == 2) {
    constexpr int A[4] = {0, 2, 0, 1}, DA[4] = {0, 1, 1, 1}, B[4] = {1, 3, 4, 5};
    fa = A[k];
    da = DA[k];
    fb = B[k];
    db = 0;
  } else {
    constexpr int A[8] = {0, 2, 4, 0, 7, 8, 2, 11}, DA[8] = {0, 0, 0, 1, 0, 0, 1, 0};
    constexpr int B[8] = {1, 3, 5, 6, 1, 9, 10, -1}, DB[8] = {0, 1, 0, 0, 1, 0, 0, 0};
    fa = A[k];
    da = DA[k];
    fb = B[k];
    db = DB[k];
  }
}

// i kx c for the half-spectrum entry kk of a row (kx = 2 pi kk / Lx)
template <typename T>
__device__ __forceinline__ cpx<T> ikx(const XformArgs& a, int kk, cpx<T> c) {
  const T k = (T)(a.two_pi_over_Lx * (double)kk);
  return mk<T>(-k * c.y, k * c.x);
}

template <int DIM, int NT, int PTS, int MAXBF, bool TWL, typename T, bool SPLIT = false, int LC = 0>
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
  const int L = LC > 0 ? LC : a.L, Pa = a.Pa, Px = a.Px;
  const size_t R = (size_t)a.M * a.Ngy;
  const int tid = threadIdx.x;
  const cT* twg = (const cT*)(sizeof(T) == 8 ? (const void*)a.twx : (const void*)a.twx32);
  cT* twl = buf + L;
  if constexpr (TWL) {
    for (int i = tid; i < L; i += NT) twl[i] = twg[i];
  }
  const cT* tw = TWL ? (const cT*)twl : twg;

  cT sa[KPT], sb[KPT];
  auto fetch = [&](int k) {
    int fa, da, fb, db;
    pair_src<DIM>(k, fa, da, fb, db);
    const S2* A = G + ((size_t)fa * R + r) * Px;
    const S2* B = G + ((size_t)(fb < 0 ? fa : fb) * R + r) * Px;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      sa[q] = mk<T>(0, 0);
      sb[q] = mk<T>(0, 0);
      if (kk < Pa) {
        sa[q] = ldv<T>(A + kk);
        if (da) sa[q] = ikx<T>(a, kk, sa[q]);
        if (fb >= 0) {
          sb[q] = ldv<T>(B + kk);
          if (db) sb[q] = ikx<T>(a, kk, sb[q]);
        }
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
    fft_lds_c<LC, +1, MAXBF, T, DIM == 2>(buf, L, 1, tw, tid, NT);
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
    fft_lds_c<LC, -1, MAXBF, T, DIM == 2>(buf, L, 1, tw, tid, NT);
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
template <int NT, int PTS, int MAXBF, typename T, bool SPLIT, int LC = 0>
__global__ void __launch_bounds__(NT) xrow2_kernel(XformArgs a,
                                                   const typename V2<T>::type* __restrict__ G,
                                                   typename V2<T>::type* __restrict__ H) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  using S2 = typename V2<T>::type;
  constexpr int KPT = (PTS + 2) / 3;  // half-spectrum entries per thread (Pa = L / 3)
  cT* buf = (cT*)smem;                // two sequences of L points
  const int r = blockIdx.x;
  const int L = LC > 0 ? LC : a.L, Pa = a.Pa, Px = a.Px;
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
    int fa, da, fb, db;
    pair_src<2>(k, fa, da, fb, db);
    const S2* A = G + ((size_t)fa * R + r) * Px;
    const S2* B = G + ((size_t)fb * R + r) * Px;
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int kk = tid + q * NT;
      if (kk < Pa) {
        sa[slot][q] = ldv<T>(A + kk);
        if (da) sa[slot][q] = ikx<T>(a, kk, sa[slot][q]);
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
    fft_lds_c<LC, +1, MAXBF, T, true>(buf, L, k1 >= 0 ? 2 : 1, twl, tid, NT);
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
  fft_lds_c<LC, -1, MAXBF, T, true>(buf, L, (f0 && f1) ? 2 : 1, twl, tid, NT);
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
// 3-D x pass with the eight field pairs transformed four at a time (two
// batches of four sequences) and the two forward pairs as one batch: three
// batched transforms per row instead of ten one-sequence transforms, a
// quarter of the radix passes and barriers, with twice the threads per row.
// Batch A holds (u, v), (w, b_x), (b_y, bz), (u_x, u_y): N_b completes and
// N_u starts; batch B holds (uz, v_x), (v_y, vz), (w_x, w_y), (wz, -): N_u,
// N_v and N_w complete.  Data [4][L] and twiddles [L] in LDS.  The lower
// half of the threads loads the spectra of batch A and the upper half those
// of batch B, both at the start (one entry per thread and sequence: the
// launch has Pa <= NT / 2); each batch goes onto LDS from its own half while
// the other half writes the zero padding.  Same products and outputs as
// xrow_kernel<3>.
// ---------------------------------------------------------------------------
template <int NT, int PTS, int MAXBF, typename T, int LC>
__global__ void __launch_bounds__(NT) xrow3_kernel(XformArgs a,
                                                   const typename V2<T>::type* __restrict__ G,
                                                   typename V2<T>::type* __restrict__ H) {
  extern __shared__ double2 smem[];
  using cT = cpx<T>;
  using S2 = typename V2<T>::type;
  constexpr int HT = NT / 2;          // threads per batch (whole wavefronts)
  cT* buf = (cT*)smem;                // four sequences of L points
  const int r = blockIdx.x;
  const int L = LC > 0 ? LC : a.L, Pa = a.Pa, Px = a.Px;
  const size_t R = (size_t)a.M * a.Ngy;
  const int tid = threadIdx.x;
  const int upper = tid >= HT, j = tid - upper * HT;
  const cT* twg = (const cT*)(sizeof(T) == 8 ? (const void*)a.twx : (const void*)a.twx32);
  // the twiddles the passes read: indices below L / R of the smallest radix
  // (the compile-time 384-point plan is 6 x 8 x 8: the first 64 entries)
  constexpr int TWC = LC == 384 ? 64 : 0;
  const int tn = TWC > 0 ? TWC : L;
  cT* twl = buf + 4 * L;
  for (int i = tid; i < tn; i += NT) twl[i] = twg[i];
  cT sa[4], sb[4];
  auto fetch = [&](int slot, int k) {
    int fa, da, fb, db;
    pair_src<3>(k, fa, da, fb, db);
    const S2* A = G + ((size_t)fa * R + r) * Px;
    const S2* B = G + ((size_t)(fb < 0 ? fa : fb) * R + r) * Px;
    sa[slot] = mk<T>(0, 0);
    sb[slot] = mk<T>(0, 0);
    if (j < Pa) {
      sa[slot] = ldv<T>(A + j);
      if (da) sa[slot] = ikx<T>(a, j, sa[slot]);
      if (fb >= 0) {
        sb[slot] = ldv<T>(B + j);
        if (db) sb[slot] = ikx<T>(a, j, sb[slot]);
      }
    }
  };
  // Hermitian extension of the packed pairs A + i B onto the four sequences
  // (the half holding the batch), or the zero padding between the two ends
  // of the spectrum (the other half)
  auto scatter = [&](bool mine) {
#pragma unroll
    for (int slot = 0; slot < 4; ++slot) {
      cT* bb = buf + slot * L;
      if (mine) {
        if (j < Pa) {
          cT Ak = sa[slot], Bk = sb[slot];
          if (j == 0) {
            Ak.y = 0;
            Bk.y = 0;
          }
          bb[j] = mk<T>(Ak.x - Bk.y, Ak.y + Bk.x);
          if (j > 0) bb[L - j] = mk<T>(Ak.x + Bk.y, -Ak.y + Bk.x);
        }
      } else {
        for (int k = Pa + j; k <= L - Pa; k += HT) bb[k] = mk<T>(0, 0);
      }
    }
  };

  T u[PTS], v[PTS], w[PTS], nb[PTS], nu[PTS], nv[PTS], nw[PTS];
  if (!upper) {
#pragma unroll
    for (int s = 0; s < 4; ++s) fetch(s, s);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) fetch(s, 4 + s);
  }
  scatter(!upper);
  __syncthreads();
  fft_lds_c<LC, +1, MAXBF, T, true, true>(buf, L, 4, twl, tid, NT);
#pragma unroll
  for (int q = 0; q < PTS; ++q) {
    const int i = tid + q * NT;
    if (i < L) {
      const cT p0 = buf[i], p1 = buf[L + i], p2 = buf[2 * L + i], p3 = buf[3 * L + i];
      u[q] = p0.x;
      v[q] = p0.y;
      w[q] = p1.x;
      nb[q] = -(u[q] * p1.y + v[q] * p2.x + w[q] * p2.y);
      nu[q] = -(u[q] * p3.x + v[q] * p3.y);
    }
  }
  __syncthreads();
  scatter(upper);
  __syncthreads();
  fft_lds_c<LC, +1, MAXBF, T, true, true>(buf, L, 4, twl, tid, NT);
#pragma unroll
  for (int q = 0; q < PTS; ++q) {
    const int i = tid + q * NT;
    if (i < L) {
      const cT p4 = buf[i], p5 = buf[L + i], p6 = buf[2 * L + i], p7 = buf[3 * L + i];
      nu[q] -= w[q] * p4.x;
      nv[q] = -(u[q] * p4.y + v[q] * p5.x + w[q] * p5.y);
      nw[q] = -(u[q] * p6.x + v[q] * p6.y + w[q] * p7.x);
    }
  }
  __syncthreads();
  // forward: sequence 0 = N_b + i N_u, sequence 1 = N_v + i N_w
#pragma unroll
  for (int q = 0; q < PTS; ++q) {
    const int i = tid + q * NT;
    if (i < L) {
      buf[i] = mk<T>(nb[q], nu[q]);
      buf[L + i] = mk<T>(nv[q], nw[q]);
    }
  }
  __syncthreads();
  fft_lds_c<LC, -1, MAXBF, T, true, true>(buf, L, 2, twl, tid, NT);
  const T invL = (T)1 / (T)L;
  const T hf = (T)0.5;
  for (int k = tid; k < Px; k += NT) {
#pragma unroll
    for (int sq = 0; sq < 2; ++sq) {
      cT A = mk<T>(0, 0), Bv = mk<T>(0, 0);
      if (k < Pa) {
        const cT Zk = buf[sq * L + k], Zm = buf[sq * L + (k == 0 ? 0 : L - k)];
        A = mk<T>(hf * (Zk.x + Zm.x) * invL, hf * (Zk.y - Zm.y) * invL);
        Bv = mk<T>(hf * (Zk.y + Zm.y) * invL, -hf * (Zk.x - Zm.x) * invL);
      }
      stv<T>(H + ((size_t)(2 * sq) * R + r) * Px + k, A);
      stv<T>(H + ((size_t)(2 * sq + 1) * R + r) * Px + k, Bv);
    }
  }
}

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
      // 1536-point rows (Nx = 1024) with the length fixed at compile time
      constexpr bool k1536 = NT * PTS >= 1536 && NT * PTS < 3072;
      auto fn = split ? xrow2_kernel<NT, PTS, 2 * MAXBF, T, true> : xrow2_kernel<NT, PTS, 2 * MAXBF, T, false>;
      if constexpr (k1536) {
        if (a.L == 1536)
          fn = split ? xrow2_kernel<NT, PTS, 2 * MAXBF, T, true, 1536> : xrow2_kernel<NT, PTS, 2 * MAXBF, T, false, 1536>;
      }
      allow_lds((const void*)fn, lds2);
      hipLaunchKernelGGL(fn, grid, dim3(NT), lds2, st, a, (const S2*)G, (S2*)H);
      return hipGetLastError();
    }
  }
  // 3-D: pairs four at a time, with twice the threads (each thread half the
  // points), when four sequences and the twiddles fit 64 KB
  if constexpr (DIM == 3 && NT <= 512) {
    constexpr int PTS3 = (PTS + 1) / 2;
    const bool c384 = a.L == 384 && 2 * NT * PTS3 >= 384;
    const size_t lds3 = ((size_t)4 * a.L + (c384 ? 64 : a.L)) * sizeof(S2);
    if (lds3 <= 64 * 1024 && a.L <= 2 * NT * PTS3 && a.Pa <= NT) {
      // the 256 x 256 workload's 384-point rows with their length fixed
      // (and 64 twiddles in LDS: 25 KB per block, six blocks per unit)
      auto fn = c384 ? xrow3_kernel<2 * NT, PTS3, 2 * MAXBF, T, 384>
                     : xrow3_kernel<2 * NT, PTS3, 2 * MAXBF, T, 0>;
      allow_lds((const void*)fn, lds3);
      hipLaunchKernelGGL(fn, grid, dim3(2 * NT), lds3, st, a, (const S2*)G, (S2*)H);
      return hipGetLastError();
    }
  }
  // 2-D 6144-point rows (Nx = 4096) with the length fixed at compile time
  if constexpr (DIM == 2 && NT * PTS >= 6144) {
    if (a.L == 6144 && !twl) {
      auto fn = split ? xrow_kernel<DIM, NT, PTS, MAXBF, false, T, true, 6144>
                      : xrow_kernel<DIM, NT, PTS, MAXBF, false, T, false, 6144>;
      allow_lds((const void*)fn, lds);
      hipLaunchKernelGGL(fn, grid, dim3(NT), lds, st, a, (const S2*)G, (S2*)H);
      return hipGetLastError();
    }
    if (a.L == 6144 && twl) {
      auto fn = split ? xrow_kernel<DIM, NT, PTS, MAXBF, true, T, true, 6144>
                      : xrow_kernel<DIM, NT, PTS, MAXBF, true, T, false, 6144>;
      allow_lds((const void*)fn, lds);
      hipLaunchKernelGGL(fn, grid, dim3(NT), lds, st, a, (const S2*)G, (S2*)H);
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

}  // namespace stau
