// Host-side description of the per-pencil system (Sec. IX "Matrix
// construction"): the interleaved variable and equation order, the band
// widths found from the entries, and the band templates that the
// factorisation combines per pencil.  Host code only: the runtime and the
// host checks of the operator build from these functions.
#pragma once

#include <cstdint>
#include <cstring>

#include "common.h"

namespace stau {

// Interleaved order of one mode: 2-D (w, b, u, p, bz, uz, wz) columns and (w, b,
// u, continuity, uz, bz, wz) rows; 3-D adds v, vz and their equations.  The
// first kb rows are the boundary conditions (z = 0 then z = 1 on each evolved
// variable).  var_of_abi[i] is the variable at index i of the state layout
// (p, b, u, [v], w, bz, uz, [vz], wz).
inline void build_sysdesc(int dim, int N, SysDesc& d, int* var_of_abi) {
  std::memset(&d, 0, sizeof(d));
  d.dim = dim;
  d.N = N;
  for (int i = 0; i < 9; ++i) {
    d.var_pos[i] = -1;
    d.eq_pos[i] = -1;
    d.abi_index[i] = -1;
  }
  if (dim == 2) {
    const int va[7] = {VW, VB, VU, VP, VBZ, VUZ, VWZ};
    const int ea[7] = {EW, EB, EU, EC, EUZ, EBZ, EWZ};
    const int abi[7] = {VP, VB, VU, VW, VBZ, VUZ, VWZ};
    d.S = 7;
    d.ne = 3;
    d.kb = 6;
    for (int i = 0; i < 7; ++i) {
      d.var_at[i] = va[i];
      d.eq_at[i] = ea[i];
      var_of_abi[i] = abi[i];
    }
    const int bv[6] = {VB, VU, VW, VB, VU, VW};
    for (int i = 0; i < 6; ++i) {
      d.bc_var[i] = bv[i];
      d.bc_side[i] = i < 3 ? 0 : 1;
    }
    d.evolved[0] = VB;
    d.evolved[1] = VU;
    d.evolved[2] = VW;
  } else {
    const int va[9] = {VW, VB, VU, VV, VP, VBZ, VUZ, VVZ, VWZ};
    const int ea[9] = {EW, EB, EU, EV, EC, EUZ, EVZ, EBZ, EWZ};
    const int abi[9] = {VP, VB, VU, VV, VW, VBZ, VUZ, VVZ, VWZ};
    d.S = 9;
    d.ne = 4;
    d.kb = 8;
    for (int i = 0; i < 9; ++i) {
      d.var_at[i] = va[i];
      d.eq_at[i] = ea[i];
      var_of_abi[i] = abi[i];
    }
    const int bv[8] = {VB, VU, VV, VW, VB, VU, VV, VW};
    for (int i = 0; i < 8; ++i) {
      d.bc_var[i] = bv[i];
      d.bc_side[i] = i < 4 ? 0 : 1;
    }
    d.evolved[0] = VB;
    d.evolved[1] = VU;
    d.evolved[2] = VV;
    d.evolved[3] = VW;
  }
  for (int i = 0; i < d.S; ++i) {
    d.var_pos[d.var_at[i]] = i;
    d.eq_pos[d.eq_at[i]] = i;
    d.abi_index[var_of_abi[i]] = i;
  }
}

// Band widths of the interleaved system from its structure (generic
// coefficients, plus the mean pencil for the gauge row).  Entries couple
// modes at most six below and seven above a row's own mode, so only that
// window of columns is scanned.
inline void band_widths(const SysDesc& d, int64_t n, int nncc, int* kl, int* ku) {
  int l = 0, u = 0;
  for (int mean = 0; mean < 2; ++mean) {
    // the linear-stability term and the non-constant coefficient inside the band too
    PencilCoef pc{1.7, 1.3, 0.31, 0.67, 1.1, mean ? 0.0 : 0.93, (mean || d.dim == 2) ? 0.0 : 0.61,
                  mean, -0.83, nncc, {0.7, -0.4, 0.25, 0.1}};
    for (int64_t r = 0; r < n; ++r) {
      const int64_t c0 = r - 6 * d.S < 0 ? 0 : r - 6 * d.S;
      const int64_t c1 = r + 7 * d.S > n ? n : r + 7 * d.S;
      for (int64_t c = c0; c < c1; ++c) {
        if (sys_entry(d, pc, (int)r, (int)c) != 0.0) {
          if (r - c > l) l = (int)(r - c);
          if (c - r > u) u = (int)(c - r);
        }
      }
    }
  }
  *kl = l;
  *ku = u;
}

// Band templates of a0 M~ + b0 L~: seven planes of n x (kl + ku + 1) entries
// (row r, column c at r * tw + c - r + kl) such that every entry of the
// operator is
//   a0 T0 + b0 (T1 (T2 at the mean pencil) + k^2 T3 + kx T4 + ky T5 + lin T6)
// with k^2 = kx^2 + ky^2.  Each plane is an exact difference of operator
// entries at unit coefficients (the entries are affine in kx, ky and lin
// apart from the k^2 terms).  base supplies kappa, nu, the buoyancy and the
// non-constant coefficient; its a0, b0, kx, ky, mean and lin are ignored.
inline void band_templates(const SysDesc& d, const PencilCoef& base, int n, int kl, int ku, double* T) {
  const int tw = kl + ku + 1;
  const size_t plane = (size_t)n * tw;
  std::memset(T, 0, 7 * plane * sizeof(double));
  auto coef = [&](double a0, double b0, double kx, double ky, int mean, double lin, int ncc) {
    PencilCoef pc = base;
    pc.a0 = a0;
    pc.b0 = b0;
    pc.kx = kx;
    pc.ky = ky;
    pc.mean = mean;
    pc.lin = lin;
    pc.nncc = ncc ? base.nncc : 0;
    return pc;
  };
  const PencilCoef cM = coef(1, 0, 0, 0, 0, 0, 0), c1 = coef(0, 1, 0, 0, 0, 0, 1),
                   c1m = coef(0, 1, 0, 0, 1, 0, 1), cxp = coef(0, 1, 1, 0, 0, 0, 1),
                   cxm = coef(0, 1, -1, 0, 0, 0, 1), cyp = coef(0, 1, 0, 1, 0, 0, 1),
                   cym = coef(0, 1, 0, -1, 0, 0, 1), cl1 = coef(0, 1, 0, 0, 0, 1, 0),
                   cl0 = coef(0, 1, 0, 0, 0, 0, 0);
  for (int r = 0; r < n; ++r)
    for (int c = r - kl < 0 ? 0 : r - kl; c < n && c - r <= ku; ++c) {
      const size_t o = (size_t)r * tw + (c - r + kl);
      const double t1 = sys_entry(d, c1, r, c);
      const double xp = sys_entry(d, cxp, r, c), xm = sys_entry(d, cxm, r, c);
      T[o] = sys_entry(d, cM, r, c);
      T[plane + o] = t1;
      T[2 * plane + o] = sys_entry(d, c1m, r, c);
      T[3 * plane + o] = 0.5 * (xp + xm) - t1;
      T[4 * plane + o] = 0.5 * (xp - xm);
      if (d.dim == 3) T[5 * plane + o] = 0.5 * (sys_entry(d, cyp, r, c) - sys_entry(d, cym, r, c));
      T[6 * plane + o] = sys_entry(d, cl1, r, c) - sys_entry(d, cl0, r, c);
    }
}

}  // namespace stau
