// Host checks of the per-pencil operator of the runtime (the system
// description, band widths and band templates it builds, and the structured
// row application of the stability iteration), and a dump of the operator
// for comparison with the oracle's matrices.
//
//   templates_check          run the checks, print the worst errors, exit 1
//                            when one is above its bound:
//     * apply_row (rows of a0 M~ + b0 L~ from the templates) against the
//       entry-by-entry matrix sys_entry on random vectors;
//     * the band templates combined per pencil (as the factorisation does)
//       against sys_entry, entry by entry;
//     * every nonzero entry of sys_entry (full scan) inside the band widths
//       band_widths reports;
//   templates_check dump dim N mean a0 b0 kappa nu buoy kx ky lin nncc g0 g1 g2 g3
//                            print n, kl, ku, then the n x n matrix a0 M~ + b0 L~
//                            (row-major, one row per line, %.17g).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "system.h"

using namespace stau;

static int dump(int argc, char** argv) {
  if (argc != 18) {
    std::fprintf(stderr, "dump: expected 16 numbers\n");
    return 2;
  }
  auto f = [&](int i) { return std::atof(argv[i]); };
  const int dim = std::atoi(argv[2]), N = std::atoi(argv[3]);
  SysDesc d;
  int abi[9];
  build_sysdesc(dim, N, d, abi);
  PencilCoef pc{f(5), f(6), f(7), f(8), f(9), f(10), f(11), std::atoi(argv[4]), f(12), std::atoi(argv[13]),
                {f(14), f(15), f(16), f(17)}};
  const int n = d.S * N;
  int kl = 0, ku = 0;
  band_widths(d, n, pc.nncc, &kl, &ku);
  std::printf("%d %d %d\n", n, kl, ku);
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) std::printf(c ? " %.17g" : "%.17g", sys_entry(d, pc, r, c));
    std::printf("\n");
  }
  return 0;
}

int main(int argc, char** argv) {
  if (argc > 1 && std::strcmp(argv[1], "dump") == 0) return dump(argc, argv);
  std::mt19937_64 gen(7);
  std::normal_distribution<double> nd;
  std::uniform_real_distribution<double> ud(-3.0, 3.0);
  double worst_row = 0, worst_tpl = 0;
  int outside = 0;
  for (int dim = 2; dim <= 3; ++dim)
    for (int N : {4, 5, 16, 33})
      for (int mean = 0; mean < 2; ++mean)
        for (int nn = 0; nn <= kMaxNcc; nn += 2)
          for (double lin : {0.0, -1.0}) {
            SysDesc d;
            int abi[9];
            build_sysdesc(dim, N, d, abi);
            const int nncc = nn == 0 ? 0 : (nn == 2 ? 3 : nn);
            PencilCoef pc{1.7e3, 1.0, 3e-4, 2e-4, 1.0, mean ? 0.0 : 3.3,
                          (mean || dim == 2) ? 0.0 : 1.9, mean, lin, nncc, {0.7, -0.4, 0.25, 0.1}};
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
              const double vr =
                  apply_row(d, pc, i, [&](int m, int var) { return x[m * d.S + d.var_pos[var]]; });
              const double er = std::fabs(vr - rr) / (rs + 1e-300);
              if (er > worst_row) worst_row = er;
            }
            // band widths (heuristic scan window) against a full scan
            int kl = 0, ku = 0;
            band_widths(d, n, nncc, &kl, &ku);
            // band templates combined with random pencil coefficients
            const int tw = kl + ku + 1;
            const size_t plane = (size_t)n * tw;
            std::vector<double> T(7 * plane);
            band_templates(d, pc, n, kl, ku, T.data());
            for (int rep = 0; rep < 3; ++rep) {
              PencilCoef q = pc;
              q.a0 = ud(gen);
              q.b0 = ud(gen);
              q.kx = mean ? 0.0 : ud(gen);
              q.ky = (mean || dim == 2) ? 0.0 : ud(gen);
              q.lin = lin == 0.0 ? 0.0 : ud(gen);
              const double k2 = q.kx * q.kx + q.ky * q.ky;
              const double* t1 = T.data() + (mean ? 2 : 1) * plane;
              for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c) {
                  const double e = sys_entry(d, q, r, c);
                  if (c - r > ku || r - c > kl) {
                    if (e != 0.0) ++outside;
                    continue;
                  }
                  const size_t o = (size_t)r * tw + (c - r + kl);
                  const double terms[6] = {q.a0 * T[o], q.b0 * t1[o], q.b0 * k2 * T[3 * plane + o],
                                           q.b0 * q.kx * T[4 * plane + o], q.b0 * q.ky * T[5 * plane + o],
                                           q.b0 * q.lin * T[6 * plane + o]};
                  double v = 0, s = 0;
                  for (double t : terms) {
                    v += t;
                    s += std::fabs(t);
                  }
                  const double er = std::fabs(v - e) / (s + std::fabs(e) + 1e-300);
                  if (er > worst_tpl) worst_tpl = er;
                }
            }
          }
  std::printf("apply_row %.3e\nband templates %.3e\nentries outside the band %d\n", worst_row, worst_tpl,
              outside);
  return (worst_row > 1e-14 || worst_tpl > 1e-14 || outside) ? 1 : 0;
}
