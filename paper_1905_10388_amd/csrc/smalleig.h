// Small dense eigenproblems of the Krylov-Schur stability solver (the
// projected m x m matrix of the shift-inverted operator, m <= kMaxM): Householder
// reduction to Hessenberg form, implicit double-shift QR for the eigenvalues,
// inverse iteration for eigenvectors (a real eigenvalue) and for the real
// two-dimensional invariant subspace of a complex-conjugate pair, and
// modified Gram-Schmidt.  Serial code for one thread; every matrix is
// row-major with leading dimension ld, in memory the caller provides (LDS in
// the kernel), so no private arrays are indexed at run time.  All loops are
// bounded (the QR iteration by 30 m steps).
#pragma once

namespace stau {
namespace small {

constexpr int kMaxM = 32;
constexpr double kEps = 2.220446049250313e-16;

__host__ __device__ inline double dabs(double x) { return x < 0.0 ? -x : x; }

// A <- P A P (Householder reflectors P = I - f v v^T) until A is upper
// Hessenberg; the reflectors are not kept.  v: workspace of m doubles.
__host__ __device__ inline void hessenberg(double* A, int m, int ld, double* v) {
  for (int k = 0; k + 2 < m; ++k) {
    double s = 0.0;
    for (int i = k + 1; i < m; ++i) s += A[i * ld + k] * A[i * ld + k];
    const double x0 = A[(k + 1) * ld + k];
    if (s == 0.0 || s == x0 * x0) continue;  // already zero below the subdiagonal
    const double alpha = x0 > 0.0 ? -__builtin_sqrt(s) : __builtin_sqrt(s);
    for (int i = k + 1; i < m; ++i) v[i] = A[i * ld + k];
    v[k + 1] = x0 - alpha;
    const double f = 2.0 / (s - x0 * x0 + v[k + 1] * v[k + 1]);
    for (int j = k + 1; j < m; ++j) {  // rows k+1.. from the left (column k set below)
      double d = 0.0;
      for (int i = k + 1; i < m; ++i) d += v[i] * A[i * ld + j];
      d *= f;
      for (int i = k + 1; i < m; ++i) A[i * ld + j] -= d * v[i];
    }
    for (int i = 0; i < m; ++i) {  // columns k+1.. from the right
      double d = 0.0;
      for (int j = k + 1; j < m; ++j) d += A[i * ld + j] * v[j];
      d *= f;
      for (int j = k + 1; j < m; ++j) A[i * ld + j] -= d * v[j];
    }
    A[(k + 1) * ld + k] = alpha;
    for (int i = k + 2; i < m; ++i) A[i * ld + k] = 0.0;
  }
}

// Eigenvalues wr + i wi of the upper Hessenberg matrix H (overwritten):
// implicit double-shift (Francis) QR steps on the unreduced trailing window,
// deflating 1 x 1 and 2 x 2 blocks at negligible subdiagonal entries; the two
// eigenvalues of a 2 x 2 block are stored at consecutive indices (a complex
// pair with wi > 0 first).  Shifts: the eigenvalues of the window's trailing
// 2 x 2 block, replaced by ad hoc values after 10 and 20 steps without a
// deflation.  Returns false after 30 m steps in all.
__host__ __device__ inline bool hess_eigvals(double* H, int m, int ld, double* wr, double* wi) {
  double anorm = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = i > 0 ? i - 1 : 0; j < m; ++j) anorm += dabs(H[i * ld + j]);
  int hi = m - 1, its = 0, total = 0;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = dabs(H[(l - 1) * ld + l - 1]) + dabs(H[l * ld + l]);
      if (s == 0.0) s = anorm;
      if (dabs(H[l * ld + l - 1]) <= kEps * s) {
        H[l * ld + l - 1] = 0.0;
        break;
      }
    }
    if (l == hi) {
      wr[hi] = H[hi * ld + hi];
      wi[hi] = 0.0;
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {
      const double a = H[(hi - 1) * ld + hi - 1], b = H[(hi - 1) * ld + hi];
      const double c = H[hi * ld + hi - 1], d = H[hi * ld + hi];
      const double p = 0.5 * (a - d), q = p * p + b * c;
      if (q >= 0.0) {
        // z = p + sign(p) sqrt(q): eigenvalues d + z and d - b c / z
        const double sq = __builtin_sqrt(q);
        const double z = p >= 0.0 ? p + sq : p - sq;
        wr[hi - 1] = d + z;
        wr[hi] = z != 0.0 ? d - b * c / z : d;
        wi[hi - 1] = wi[hi] = 0.0;
      } else {
        const double y = __builtin_sqrt(-q);
        wr[hi - 1] = wr[hi] = d + p;
        wi[hi - 1] = y;
        wi[hi] = -y;
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (++total > 30 * m) return false;
    ++its;
    double s, t;  // sum and product of the two shifts
    if (its == 10 || its == 20) {
      const double x = dabs(H[hi * ld + hi - 1]) + dabs(H[(hi - 1) * ld + hi - 2]);
      s = 1.5 * x;
      t = x * x;
    } else {
      const double a = H[(hi - 1) * ld + hi - 1], b = H[(hi - 1) * ld + hi];
      const double c = H[hi * ld + hi - 1], d = H[hi * ld + hi];
      s = a + d;
      t = a * d - b * c;
    }
    // first column of H^2 - s H + t I on the window (rows l, l+1, l+2)
    const double h00 = H[l * ld + l], h01 = H[l * ld + l + 1], h10 = H[(l + 1) * ld + l];
    const double h11 = H[(l + 1) * ld + l + 1], h21 = H[(l + 2) * ld + l + 1];
    double x = h00 * h00 + h01 * h10 - s * h00 + t;
    double y = h10 * (h00 + h11 - s);
    double z = h10 * h21;
    for (int k = l; k < hi; ++k) {
      const bool three = k + 2 <= hi;
      const double nrm = __builtin_sqrt(x * x + y * y + (three ? z * z : 0.0));
      if (nrm != 0.0) {
        const double alpha = x > 0.0 ? -nrm : nrm;
        const double v0 = x - alpha, v1 = y, v2 = three ? z : 0.0;
        const double f = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
        for (int j = k > l ? k - 1 : l; j <= hi; ++j) {
          double d = v0 * H[k * ld + j] + v1 * H[(k + 1) * ld + j];
          if (three) d += v2 * H[(k + 2) * ld + j];
          d *= f;
          H[k * ld + j] -= d * v0;
          H[(k + 1) * ld + j] -= d * v1;
          if (three) H[(k + 2) * ld + j] -= d * v2;
        }
        const int ie = k + 3 < hi ? k + 3 : hi;
        for (int i = l; i <= ie; ++i) {
          double d = H[i * ld + k] * v0 + H[i * ld + k + 1] * v1;
          if (three) d += H[i * ld + k + 2] * v2;
          d *= f;
          H[i * ld + k] -= d * v0;
          H[i * ld + k + 1] -= d * v1;
          if (three) H[i * ld + k + 2] -= d * v2;
        }
        if (k > l) {  // the bulge column is now (alpha, 0, 0)
          H[k * ld + k - 1] = alpha;
          H[(k + 1) * ld + k - 1] = 0.0;
          if (three) H[(k + 2) * ld + k - 1] = 0.0;
        }
      }
      if (k + 1 < hi) {
        x = H[(k + 1) * ld + k];
        y = H[(k + 2) * ld + k];
        z = k + 3 <= hi ? H[(k + 3) * ld + k] : 0.0;
      }
    }
  }
  return true;
}

// LU factorisation with partial pivoting of the m x m matrix A (in place;
// piv[k] = the row swapped with row k).  A zero pivot is replaced by
// kEps * scale, so that inverse iteration at an exact eigenvalue still
// yields a (large) finite solution.
__host__ __device__ inline void lu_factor(double* A, int m, int ld, int* piv, double scale) {
  for (int k = 0; k < m; ++k) {
    int pr = k;
    double best = dabs(A[k * ld + k]);
    for (int i = k + 1; i < m; ++i)
      if (dabs(A[i * ld + k]) > best) {
        best = dabs(A[i * ld + k]);
        pr = i;
      }
    piv[k] = pr;
    if (pr != k)
      for (int j = 0; j < m; ++j) {
        const double q = A[k * ld + j];
        A[k * ld + j] = A[pr * ld + j];
        A[pr * ld + j] = q;
      }
    if (A[k * ld + k] == 0.0) A[k * ld + k] = kEps * (scale > 0.0 ? scale : 1.0);
    const double r = 1.0 / A[k * ld + k];
    for (int i = k + 1; i < m; ++i) {
      const double l = A[i * ld + k] * r;
      A[i * ld + k] = l;
      if (l != 0.0)
        for (int j = k + 1; j < m; ++j) A[i * ld + j] -= l * A[k * ld + j];
    }
  }
}

// x <- A^{-1} x with the factors of lu_factor.
__host__ __device__ inline void lu_solve(const double* A, int m, int ld, const int* piv, double* x) {
  for (int k = 0; k < m; ++k) {
    const int pr = piv[k];
    if (pr != k) {
      const double q = x[k];
      x[k] = x[pr];
      x[pr] = q;
    }
    for (int i = k + 1; i < m; ++i) x[i] -= A[i * ld + k] * x[k];
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < m; ++j) s -= A[i * ld + j] * x[j];
    x[i] = s / A[i * ld + i];
  }
}

// Column c of Y (m rows, leading dimension ld) scaled to unit 2-norm; returns
// the norm it had.
__host__ __device__ inline double normalize_col(double* Y, int m, int ld, int c) {
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += Y[i * ld + c] * Y[i * ld + c];
  const double nrm = __builtin_sqrt(s);
  if (nrm > 0.0)
    for (int i = 0; i < m; ++i) Y[i * ld + c] /= nrm;
  return nrm;
}

// Column c of Y made orthogonal to columns 0..c-1 (orthonormal) and
// normalised, with two Gram-Schmidt passes; returns its final norm relative
// to its norm on entry (small: c lay in the span of the others).
__host__ __device__ inline double orthonormalize_col(double* Y, int m, int ld, int c) {
  double s0 = 0.0;
  for (int i = 0; i < m; ++i) s0 += Y[i * ld + c] * Y[i * ld + c];
  if (s0 == 0.0) return 0.0;
  for (int pass = 0; pass < 2; ++pass)
    for (int q = 0; q < c; ++q) {
      double d = 0.0;
      for (int i = 0; i < m; ++i) d += Y[i * ld + q] * Y[i * ld + c];
      for (int i = 0; i < m; ++i) Y[i * ld + c] -= d * Y[i * ld + q];
    }
  return normalize_col(Y, m, ld, c) / __builtin_sqrt(s0);
}

// Start vector of inverse iteration: entries in [0.5, 1.5) from the
// golden-ratio sequence, offset by `seed` (no symmetry of the problem).
__host__ __device__ inline double start_entry(int i, int seed) {
  const double q = 0.6180339887498949 * (double)(i + 1 + 7 * seed);
  return 0.5 + (q - __builtin_floor(q));
}

// Column c of Y <- the eigenvector (unit norm) of G for the real eigenvalue
// t: two steps of inverse iteration with G - t I.  W: m x m workspace.
__host__ __device__ inline void eigvec_real(const double* G, int m, int ld, double t, double scale,
                                            double* W, int* piv, double* Y, int ldy, int c,
                                            double* x) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) W[i * ld + j] = G[i * ld + j] - (i == j ? t : 0.0);
  lu_factor(W, m, ld, piv, scale);
  for (int i = 0; i < m; ++i) x[i] = start_entry(i, c);
  for (int it = 0; it < 2; ++it) {
    lu_solve(W, m, ld, piv, x);
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += x[i] * x[i];
    const double r = s > 0.0 ? 1.0 / __builtin_sqrt(s) : 0.0;
    for (int i = 0; i < m; ++i) x[i] *= r;
  }
  for (int i = 0; i < m; ++i) Y[i * ldy + c] = x[i];
}

// Columns c, c+1 of Y <- an orthonormal basis of the real invariant subspace
// of G for the complex pair a +- i b: two steps of block inverse iteration
// with the real matrix G^2 - 2 a G + (a^2 + b^2) I, singular on that
// subspace.  W: m x m workspace; x: 2 m doubles.
__host__ __device__ inline void eigspace_pair(const double* G, int m, int ld, double a, double b,
                                              double scale, double* W, int* piv, double* Y,
                                              int ldy, int c, double* x) {
  const double s = 2.0 * a, t = a * a + b * b;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double g2 = 0.0;
      for (int k = 0; k < m; ++k) g2 += G[i * ld + k] * G[k * ld + j];
      W[i * ld + j] = g2 - s * G[i * ld + j] + (i == j ? t : 0.0);
    }
  lu_factor(W, m, ld, piv, scale * scale);
  double* x0 = x;
  double* x1 = x + m;
  for (int i = 0; i < m; ++i) {
    x0[i] = start_entry(i, c);
    x1[i] = start_entry(i, c + 1) * (i & 1 ? -1.0 : 1.0);
  }
  for (int it = 0; it < 2; ++it) {
    lu_solve(W, m, ld, piv, x0);
    lu_solve(W, m, ld, piv, x1);
    for (int i = 0; i < m; ++i) {
      Y[i * ldy + c] = x0[i];
      Y[i * ldy + c + 1] = x1[i];
    }
    // orthonormalise the pair in place (the columns before c are not involved)
    normalize_col(Y, m, ldy, c);
    double d = 0.0;
    for (int i = 0; i < m; ++i) d += Y[i * ldy + c] * Y[i * ldy + c + 1];
    for (int i = 0; i < m; ++i) Y[i * ldy + c + 1] -= d * Y[i * ldy + c];
    normalize_col(Y, m, ldy, c + 1);
    for (int i = 0; i < m; ++i) {
      x0[i] = Y[i * ldy + c];
      x1[i] = Y[i * ldy + c + 1];
    }
  }
}

}  // namespace small
}  // namespace stau
