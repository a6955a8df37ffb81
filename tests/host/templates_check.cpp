// Host check of the structured operator application used by the stability
// iteration (M~ x): apply_row (rows of a0 M~ + b0 L~) against the
// entry-by-entry matrix sys_entry, on random vectors, for 2-D and 3-D system
// descriptions, several N, mean and non-mean pencils.  Prints the worst
// relative error (scaled by the sum of |terms|) and exits 1 above 1e-14.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "common.h"

using namespace stau;

static void build(int dim, int N, SysDesc& d) {
  std::memset(&d, 0, sizeof(d));
  d.dim = dim;
  d.N = N;
  for (int i = 0; i < 9; ++i) {
    d.var_pos[i] = -1;
    d.eq_pos[i] = -1;
  }
  if (dim == 2) {
    const int va[7] = {VW, VB, VU, VP, VBZ, VUZ, VWZ}, ea[7] = {EW, EB, EU, EC, EUZ, EBZ, EWZ};
    d.S = 7;
    d.ne = 3;
    d.kb = 6;
    for (int i = 0; i < 7; ++i) {
      d.var_at[i] = va[i];
      d.eq_at[i] = ea[i];
    }
    const int bv[6] = {VB, VU, VW, VB, VU, VW};
    for (int i = 0; i < 6; ++i) {
      d.bc_var[i] = bv[i];
      d.bc_side[i] = i < 3 ? 0 : 1;
    }
  } else {
    const int va[9] = {VW, VB, VU, VV, VP, VBZ, VUZ, VVZ, VWZ};
    const int ea[9] = {EW, EB, EU, EV, EC, EUZ, EVZ, EBZ, EWZ};
    d.S = 9;
    d.ne = 4;
    d.kb = 8;
    for (int i = 0; i < 9; ++i) {
      d.var_at[i] = va[i];
      d.eq_at[i] = ea[i];
    }
    const int bv[8] = {VB, VU, VV, VW, VB, VU, VV, VW};
    for (int i = 0; i < 8; ++i) {
      d.bc_var[i] = bv[i];
      d.bc_side[i] = i < 4 ? 0 : 1;
    }
  }
  for (int i = 0; i < d.S; ++i) {
    d.var_pos[d.var_at[i]] = i;
    d.eq_pos[d.eq_at[i]] = i;
  }
}

int main() {
  std::mt19937_64 gen(7);
  std::normal_distribution<double> nd;
  double worst_row = 0;
  for (int dim = 2; dim <= 3; ++dim)
    for (int N : {4, 5, 16, 33})
      for (int mean = 0; mean < 2; ++mean)
      for (int nn = 0; nn <= kMaxNcc; nn += 2)
      for (double lin : {0.0, -1.0}) {
        SysDesc d;
        build(dim, N, d);
        PencilCoef pc{1.7e3, 1.0, 3e-4, 2e-4, 1.0, mean ? 0.0 : 3.3,
                      (mean || dim == 2) ? 0.0 : 1.9, mean, lin, nn, {0.7, -0.4, 0.25, 0.1}};
        if (nn == 0) pc.nncc = 0;
        if (nn == 2) pc.nncc = 3;
        const int n = d.S * N;  // kb + (N - 1) S + 1 with kb = S - 1
        std::vector<double> x(n);
        for (auto& v : x) v = nd(gen);
        for (int i = 0; i < n; ++i) {
          double rr = 0, rs = 0;
          for (int j = 0; j < n; ++j) {
            const double a = sys_entry(d, pc, i, j);  // A~(i, j)
            rr += a * x[j];
            rs += std::fabs(a * x[j]);
          }
          const double vr = apply_row(d, pc, i, [&](int m, int var) { return x[m * d.S + d.var_pos[var]]; });
          const double er = std::fabs(vr - rr) / (rs + 1e-300);
          if (er > worst_row) worst_row = er;
        }
      }
  std::printf("apply_row %.3e\n", worst_row);
  return worst_row > 1e-14 ? 1 : 0;
}
