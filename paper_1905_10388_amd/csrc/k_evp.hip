// Linear stability of the conduction state (Sec. IX "Eigenvalue solver"): the
// eigenvalues sigma of  sigma M~ x + (L~ + L~') x = 0  nearest a real shift
// tau, for every pencil, by shift-invert Krylov-Schur iteration (the sparse
// route of Sec. IX: a Krylov eigensolver applied to the shift-inverted
// operator, with the banded LU of its pencil).
//
// With A = tau M~ + L~ + L~' factored, the operator T = A^{-1} M~ has the
// eigenvalues theta = 1 / (tau - sigma); those of largest modulus belong to
// the sigma nearest tau.  One wavefront per pencil keeps an orthonormal basis
// V_0..V_m of a Krylov subspace of T (in global memory, vector-major) and the
// projected matrix G = V^T T V (m x m, in LDS), with T V = V G + beta
// V_m e_{m-1}^T after each cycle of Arnoldi steps:
//   * an Arnoldi step applies T (M~ x from the operator templates, then the
//     two sweeps of the banded solve) and orthogonalises the result against
//     the basis with classical Gram-Schmidt and one reorthogonalisation;
//   * after the basis reaches m vectors, one thread computes the eigenvalues
//     of G (Householder-Hessenberg reduction and double-shift QR), the
//     eigenvectors of the `keep` eigenvalues of largest modulus (inverse
//     iteration; the real invariant subspace of a complex pair), and the
//     residual |beta y_{m-1}| / |theta| of each wanted Ritz pair;
//   * unless the nev wanted pairs have converged (residual <= tol) or the
//     operator count reached max_ops, the basis is contracted to the
//     orthonormalised kept vectors Q (V <- V Q, G <- Q^T G Q, the new row
//     beta Q_{m-1,:} coupling them to V_m, which becomes basis vector `keep`)
//     and the Arnoldi steps resume from there (a thick restart).
// Output per pencil: the nev values sigma = tau - 1 / theta (complex, nearest
// tau first), their residuals, the number converged, the operator count and
// optionally the eigenvectors X = P^R x (state layout, unit 2-norm of the
// real-scaled vector x, u-type variables scaled by -i).
#include "smalleig.h"
#include "sweeps.h"

namespace stau {

namespace {

constexpr int kM = small::kMaxM;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// LDS doubles beyond the solve vector and the basis vector: G, H, W, Y
// (kM x kM each) and the short vectors wr, wi, tv (2 kM), key, res
constexpr int kSmallDoubles = 4 * kM * kM + 6 * kM;
constexpr int kSmallInts = 2 * kM + 4;

// Rayleigh-Ritz step and restart data, run by one thread.  mc: basis size,
// betaL: coefficient of V_mc in T V_{mc-1}.  Returns the number of kept
// vectors (columns of Y) and sets *done; with *done the final Ritz values,
// residuals and (complex) eigenvectors of the nev wanted pairs are written
// (sigma, resid, nconv; eigenvectors as column pairs 2q, 2q+1 of H).
__device__ __forceinline__ int ritz(double* G, double* H, double* W, double* Y, double* wr,
                                    double* wi, double* tv, double* key, double* res, int* piv,
                                    int* ord, int mc, double betaL, int nev, double tau, double tol,
                                    bool stop, bool* done, double2* sigma, double* resid,
                                    int* nconv) {
  using namespace small;
  for (int i = 0; i < mc; ++i)
    for (int j = 0; j < mc; ++j) H[i * kM + j] = G[i * kM + j];
  hessenberg(H, mc, kM, tv);
  if (!hess_eigvals(H, mc, kM, wr, wi)) {
    for (int q = 0; q < nev; ++q) {
      sigma[q] = make_double2(__builtin_nan(""), 0.0);
      resid[q] = __builtin_inf();
    }
    *nconv = 0;
    *done = true;
    return 0;
  }
  // positions by |theta| descending (stable: a complex pair stays adjacent,
  // the member with wi > 0 first)
  for (int i = 0; i < mc; ++i) {
    key[i] = wr[i] * wr[i] + wi[i] * wi[i];
    int k = i;
    while (k > 0 && key[ord[k - 1]] < key[i]) {
      ord[k] = ord[k - 1];
      --k;
    }
    ord[k] = i;
  }
  double scale = 0.0;
  for (int i = 0; i < mc; ++i)
    for (int j = 0; j < mc; ++j) scale += dabs(G[i * kM + j]);
  // vectors kept by a restart: nev plus half of the rest (at least two basis
  // vectors are then added per cycle); a complex pair is kept whole
  int target = nev + (mc - nev) / 2;
  if (target > mc - 2) target = mc - 2;
  if (target < nev) target = nev < mc ? nev : mc;
  int q = 0;
  while (q < target) {
    const int e = ord[q];
    const double mod = __builtin_sqrt(key[e]);
    const double rm = mod > 0.0 ? 1.0 / mod : 0.0;
    if (wi[e] == 0.0) {
      eigvec_real(G, mc, kM, wr[e], scale, W, piv, Y, kM, q, tv);
      res[q] = mod > 0.0 ? dabs(betaL * Y[(mc - 1) * kM + q]) * rm : __builtin_inf();
      ++q;
    } else {
      if (q + 1 >= mc) break;
      eigspace_pair(G, mc, kM, wr[e], wi[e], scale, W, piv, Y, kM, q, tv);
      const double y0 = Y[(mc - 1) * kM + q], y1 = Y[(mc - 1) * kM + q + 1];
      res[q] = res[q + 1] =
          mod > 0.0 ? dabs(betaL) * __builtin_sqrt(y0 * y0 + y1 * y1) * rm : __builtin_inf();
      q += 2;
    }
  }
  int keep = q;
  int nc = 0;
  for (int i = 0; i < nev && i < keep; ++i) nc += res[i] <= tol;
  *done = stop || nc == nev || betaL == 0.0;
  if (*done) {
    for (int i = 0; i < nev; ++i) {
      if (i >= keep || key[ord[i]] == 0.0) {
        sigma[i] = make_double2(__builtin_nan(""), 0.0);
        resid[i] = __builtin_inf();
        continue;
      }
      const int e = ord[i];
      const double k2 = key[e];
      sigma[i] = make_double2(tau - wr[e] / k2, wi[e] / k2);  // tau - 1 / theta
      resid[i] = res[i];
      if (wi[e] == 0.0) {
        for (int r = 0; r < mc; ++r) {
          H[r * kM + 2 * i] = Y[r * kM + i];
          H[r * kM + 2 * i + 1] = 0.0;
        }
      } else {
        // eigenvector in the pair's basis B = Y[:, c..c+1]: the eigenvector
        // c of the 2 x 2 matrix B^T G B for wr + i |wi|, conjugated for the
        // member with wi < 0
        const int c = wi[e] > 0.0 ? i : i - 1;
        double bm[4];
        for (int s = 0; s < 2; ++s)
          for (int t = 0; t < 2; ++t) {
            double acc = 0.0;
            for (int r = 0; r < mc; ++r) {
              double gy = 0.0;
              for (int k = 0; k < mc; ++k) gy += G[r * kM + k] * Y[k * kM + c + t];
              acc += Y[r * kM + c + s] * gy;
            }
            bm[2 * s + t] = acc;
          }
        const double lr = wr[e], li = dabs(wi[e]);
        double c0r, c0i, c1r, c1i;  // c = (c0, c1), (B - lambda) c = 0
        if (dabs(bm[1]) >= dabs(bm[2])) {
          c0r = bm[1];
          c0i = 0.0;
          c1r = lr - bm[0];
          c1i = li;
        } else {
          c0r = lr - bm[3];
          c0i = li;
          c1r = bm[2];
          c1i = 0.0;
        }
        double nrm = 0.0;
        for (int r = 0; r < mc; ++r) {
          const double yr = Y[r * kM + c] * c0r + Y[r * kM + c + 1] * c1r;
          const double yi = Y[r * kM + c] * c0i + Y[r * kM + c + 1] * c1i;
          nrm += yr * yr + yi * yi;
        }
        const double rn = nrm > 0.0 ? 1.0 / __builtin_sqrt(nrm) : 0.0;
        const double sgn = wi[e] > 0.0 ? 1.0 : -1.0;
        for (int r = 0; r < mc; ++r) {
          H[r * kM + 2 * i] = (Y[r * kM + c] * c0r + Y[r * kM + c + 1] * c1r) * rn;
          H[r * kM + 2 * i + 1] = sgn * (Y[r * kM + c] * c0i + Y[r * kM + c + 1] * c1i) * rn;
        }
      }
    }
    *nconv = nc;
    return keep;
  }
  // restart data: Q = orthonormalised Y[:, 0..keep), G <- Q^T G Q bordered
  // by the row beta Q_{mc-1,:}
  for (int c = 0; c < keep; ++c)
    if (orthonormalize_col(Y, mc, kM, c) < 1e-8) {
      keep = c;  // (a kept vector in the span of the others: drop the rest)
      break;
    }
  for (int r = 0; r < mc; ++r)
    for (int c = 0; c < keep; ++c) {
      double acc = 0.0;
      for (int k = 0; k < mc; ++k) acc += G[r * kM + k] * Y[k * kM + c];
      H[r * kM + c] = acc;  // G Q
    }
  for (int i = 0; i < keep; ++i)
    for (int c = 0; c < keep; ++c) {
      double acc = 0.0;
      for (int r = 0; r < mc; ++r) acc += Y[r * kM + i] * H[r * kM + c];
      W[i * kM + c] = acc;  // Q^T G Q
    }
  for (int i = 0; i < kM * kM; ++i) G[i] = 0.0;
  for (int i = 0; i < keep; ++i)
    for (int c = 0; c < keep; ++c) G[i * kM + c] = W[i * kM + c];
  for (int c = 0; c < keep; ++c) G[keep * kM + c] = betaL * Y[(mc - 1) * kM + c];
  return keep;
}

template <int FW, int BW>
__global__ void __launch_bounds__(kWave) evp_kernel(PencilArgs a, double tau, int nev, int m,
                                                    int max_ops, double tol,
                                                    const double* __restrict__ Lf,
                                                    const uint8_t* __restrict__ sl,
                                                    const double* __restrict__ Uf,
                                                    double* __restrict__ V, EvpOut o) {
  extern __shared__ double lds[];
  const int p = blockIdx.x, lane = threadIdx.x;
  const SysDesc& d = a.desc;
  const int n = a.n, N = d.N, S = d.S, npad = a.nst, nch = npad / kCH;
  const int span = BW + npad + FW;
  const size_t ss = (size_t)S * N;
  double* b = lds + BW;    // T x: rows [-BW, npad + FW)
  double* x = lds + span;  // basis vector being applied, rows [0, npad)
  double* G = x + npad;
  double* H = G + kM * kM;
  double* W = H + kM * kM;
  double* Y = W + kM * kM;
  double* wr = Y + kM * kM;
  double* wi = wr + kM;
  double* tv = wi + kM;
  double* key = tv + 2 * kM;
  double* res = key + kM;
  int* piv = (int*)(res + kM);
  int* ord = piv + kM;
  int* flags = ord + kM;  // [0] done, [1] kept vectors
  if (!pencil_active(a, p)) {
    for (int q = lane; q < nev; q += kWave) {
      o.sigma[(size_t)p * nev + q] = make_double2(0.0, 0.0);
      o.resid[(size_t)p * nev + q] = 0.0;
    }
    if (lane == 0) {
      o.nconv[p] = 0;
      if (o.nops) o.nops[p] = 0;
    }
    if (o.X)
      for (int q = 0; q < nev; ++q)
        for (size_t i = lane; i < ss; i += kWave) o.X[((size_t)q * a.P + p) * ss + i] = make_double2(0.0, 0.0);
    return;
  }
  const PencilCoef pm = pencil_coef(a, p, 1.0, 0.0);  // M~
  const double* Lp = Lf + (size_t)p * npad * FW;
  const uint32_t* swp = (const uint32_t*)(sl + (size_t)p * npad);
  const double* Up = Uf + (size_t)p * npad * BW;
  const size_t nV = (size_t)n;
  double* Vp = V + (size_t)p * (m + 1) * nV;

  // b <- A^{-1} M~ x
  auto apply_T = [&]() {
    __syncthreads();
    for (int r = lane - BW; r < npad + FW; r += kWave)
      b[r] = (r >= 0 && r < n) ? apply_row(d, pm, r, [&](int mm, int var) { return x[mm * S + d.var_pos[var]]; })
                               : 0.0;
    __syncthreads();
    sweeps<double, FW, BW>(b, Lp, swp, Up, nch, lane);
    __syncthreads();
  };
  auto norm_b = [&]() {
    double s2 = 0.0;
    for (int r = lane; r < n; r += kWave) s2 += b[r] * b[r];
    return __builtin_sqrt(wave_sum(s2));
  };
  // V_j <- b / beta, x <- V_j
  auto store_basis = [&](int j, double beta) {
    const double inv = 1.0 / beta;
    for (int r = lane; r < n; r += kWave) {
      const double v = b[r] * inv;
      Vp[(size_t)j * nV + r] = v;
      x[r] = v;
    }
  };

  // start: T applied to a fixed vector without symmetry (which also removes
  // the components in the null space of M~, the infinite eigenvalues)
  for (int r = lane; r < npad; r += kWave) x[r] = r < n ? small::start_entry(r, 0) : 0.0;
  for (int i = lane; i < kM * kM; i += kWave) G[i] = 0.0;
  apply_T();
  int ops = 1;
  store_basis(0, norm_b());
  int j0 = 0;
  for (;;) {
    int mc = m;
    double betaL = 0.0;
    for (int j = j0; j < m; ++j) {
      apply_T();
      ++ops;
      const double tn = norm_b();
      // classical Gram-Schmidt against V_0..V_j with one reorthogonalisation;
      // column j of G accumulates both passes
      for (int pass = 0; pass < 2; ++pass) {
        double h[kM];
#pragma unroll
        for (int i = 0; i < kM; ++i) h[i] = 0.0;
        for (int r = lane; r < n; r += kWave) {
          const double w = b[r];
#pragma unroll
          for (int i = 0; i < kM; ++i)
            if (i <= j) h[i] += Vp[(size_t)i * nV + r] * w;
        }
#pragma unroll
        for (int i = 0; i < kM; ++i)
          if (i <= j) h[i] = wave_sum(h[i]);
        for (int r = lane; r < n; r += kWave) {
          double w = b[r];
#pragma unroll
          for (int i = 0; i < kM; ++i)
            if (i <= j) w -= Vp[(size_t)i * nV + r] * h[i];
          b[r] = w;
        }
        if (lane == 0) {
#pragma unroll
          for (int i = 0; i < kM; ++i)
            if (i <= j) G[i * kM + j] = pass == 0 ? h[i] : G[i * kM + j] + h[i];
        }
      }
      const double beta = norm_b();
      if (!(beta > 1e-12 * tn)) {  // the basis spans an invariant subspace of T
        mc = j + 1;
        break;
      }
      store_basis(j + 1, beta);
      if (j + 1 < m) {
        if (lane == 0) G[(j + 1) * kM + j] = beta;
      } else {
        betaL = beta;
      }
    }
    __syncthreads();
    if (lane == 0) {
      bool done = false;
      const int keep = ritz(G, H, W, Y, wr, wi, tv, key, res, piv, ord, mc, betaL, nev, tau, tol,
                            ops >= max_ops, &done, o.sigma + (size_t)p * nev, o.resid + (size_t)p * nev,
                            o.nconv + p);
      flags[0] = done;
      flags[1] = keep;
      if (done && o.nops) o.nops[p] = ops;
    }
    __syncthreads();
    const int keep = flags[1];
    if (flags[0]) {
      // eigenvectors V H[:, 2q] + i V H[:, 2q+1] of the wanted pairs
      if (o.X)
        for (int q = 0; q < nev; ++q) {
          double2* Xq = o.X + ((size_t)q * a.P + p) * ss;
          if (q >= keep) {
            for (size_t i = lane; i < ss; i += kWave) Xq[i] = make_double2(0.0, 0.0);
            continue;
          }
          __syncthreads();
          for (int r = lane; r < n; r += kWave) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int l = 0; l < kM; ++l)
              if (l < mc) {
                const double v = Vp[(size_t)l * nV + r];
                re += v * H[l * kM + 2 * q];
                im += v * H[l * kM + 2 * q + 1];
              }
            b[r] = re;
            x[r] = im;
          }
          __syncthreads();
          for (size_t i = lane; i < ss; i += kWave) {
            const int vabi = (int)(i / N), mm = (int)(i - (size_t)vabi * N);
            const int var = a.var_of_abi[vabi];
            const int pos = d.var_pos[var];
            double xr = b[mm * S + pos], xi = x[mm * S + pos];
            if (mm + 2 < N) {
              xr -= b[(mm + 2) * S + pos];
              xi -= x[(mm + 2) * S + pos];
            }
            Xq[i] = (var == VU || var == VUZ || var == VV || var == VVZ) ? make_double2(xi, -xr)  // u = -i u~
                                                                         : make_double2(xr, xi);
          }
        }
      return;
    }
    // thick restart: V_0..V_{keep-1} <- V Q, V_keep <- V_m
    for (int r = lane; r < n; r += kWave) {
      double vals[kM];
#pragma unroll
      for (int l = 0; l < kM; ++l) vals[l] = l < mc ? Vp[(size_t)l * nV + r] : 0.0;
      const double vlast = Vp[(size_t)mc * nV + r];
      for (int i = 0; i < keep; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < kM; ++l)
          if (l < mc) acc += vals[l] * Y[l * kM + i];
        Vp[(size_t)i * nV + r] = acc;
      }
      Vp[(size_t)keep * nV + r] = vlast;
      x[r] = vlast;
    }
    j0 = keep;
  }
}

template <int FW, int BW>
hipError_t launch_evp_t(const PencilArgs& a, double tau, int nev, int ncv, int max_ops, double tol,
                        const double* Lf, const uint8_t* sl, const double* Uf, double* V, const EvpOut& o,
                        hipStream_t st) {
  const int span = BW + a.nst + FW;
  const size_t lds = (size_t)(span + a.nst + kSmallDoubles) * sizeof(double) + (size_t)kSmallInts * sizeof(int);
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)evp_kernel<FW, BW>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((evp_kernel<FW, BW>), dim3(a.P), dim3(kWave), lds, st, a, tau, nev, ncv, max_ops, tol,
                     Lf, sl, Uf, V, o);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_evp(const PencilArgs& a, double tau, int nev, int ncv, int max_ops, double tol,
                      const double* Lf, const uint8_t* sl, const double* Uf, double* V,
                      const EvpOut& o, hipStream_t st) {
  if (nev < 1 || ncv < nev + 2 || ncv > kM || 2 * nev > kM || ncv > a.n) return hipErrorInvalidValue;
#define STAU_CASE(F, B) \
  if (a.FW == F && a.BW == B) return launch_evp_t<F, B>(a, tau, nev, ncv, max_ops, tol, Lf, sl, Uf, V, o, st);
  STAU_SWEEP_VARIANTS(STAU_CASE)
#undef STAU_CASE
  return hipErrorInvalidValue;
}

}  // namespace stau
