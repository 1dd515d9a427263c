// The generated amplitude code of one process instantiated on the host in
// double precision: |M|^2 per event for events read from stdin.
//   stdin:  n alpha_s m_t, then n lines of npart x 4 momenta (E px py pz)
//   stdout: n values of |M|^2 (averaged, summed over every kept helicity)
// With the argument "hel": first a line "NGOOD NSUM HELW", then per event the
// kept helicities' bit patterns and colour-summed |M_h|^2 (not averaged), in
// the kernels' order (the first NSUM are the ones they evaluate).
// Built by tests/test_generated_host.py with -DGEN_HEADER=<header> -DGEN_NS=<namespace>.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include GEN_HEADER

using namespace rwgt;

int main(int argc, char** argv) {
  const bool per_hel = argc > 1 && argv[1][0] == 'h';
  int n = 0;
  double as = 0.0, mt = 0.0;
  if (std::scanf("%d %lf %lf", &n, &as, &mt) != 3) return 1;
  Card<double, double> cd{};
  const double gs = std::sqrt(4.0 * M_PI * as);
  cd.gqq = gs;
  cd.g3 = gs;
  cd.g4 = gs * gs;
  cd.mt = mt;
  constexpr int NP = GEN_NS::NPART;
  if (per_hel) std::printf("%d %d %.17g\n", GEN_NS::NGOOD, GEN_NS::NSUM, GEN_NS::HELW);
  for (int e = 0; e < n; ++e) {
    double P[NP][4];
    for (int a = 0; a < NP; ++a)
      for (int m = 0; m < 4; ++m)
        if (std::scanf("%lf", &P[a][m]) != 1) return 2;
    double me = 0.0;
    for (int h = 0; h < GEN_NS::NGOOD; ++h) {
      cx<double> j[GEN_NS::NCOL];
      GEN_NS::jamps<double, double>(P, GEN_NS::GOOD_HOST[h], cd, j);
      const double mh = GEN_NS::colour_sum<double>(j);
      if (per_hel) std::printf("%d %.17g\n", GEN_NS::GOOD_HOST[h], mh);
      me += mh;
    }
    if (!per_hel) std::printf("%.17g\n", me * GEN_NS::AVERAGE);
  }
  return 0;
}
