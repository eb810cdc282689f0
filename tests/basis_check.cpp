// Host check of the reduced-basis table: for random unit vectors, every dependent
// monomial equals its combination of kept monomials (built with -D__host__= -D__device__=).
#include <cmath>
#include <cstdio>
#include <random>

#include "basis.hpp"

static double mono(int a, int b, int c, const double* r) { return std::pow(r[0], a) * std::pow(r[1], b) * std::pow(r[2], c); }

int main() {
  // exponents of the 22 monomials in the library order
  const int E[22][3] = {{0, 0, 0}, {2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}, {4, 0, 0},
                        {3, 1, 0}, {3, 0, 1}, {2, 2, 0}, {2, 1, 1}, {2, 0, 2}, {1, 3, 0}, {1, 2, 1}, {1, 1, 2},
                        {1, 0, 3}, {0, 4, 0}, {0, 3, 1}, {0, 2, 2}, {0, 1, 3}, {0, 0, 4}};
  std::mt19937_64 g(1505);
  std::normal_distribution<double> n(0.0, 1.0);
  double worst = 0.0;
  int bad = 0;
  for (int j = 0; j < pk::kept_count(4); ++j)
    if (E[pk::kept_monomial(j)][2] > 1) ++bad;  // kept ones have c <= 1
  for (int d = 0; d < pk::dep_count(4); ++d)
    if (E[pk::dep_monomial(d)][2] < 2) ++bad;   // dependent ones have c >= 2
  if (pk::kept_count(2) != 6 || pk::dep_count(2) != 1 || pk::dep_monomial(0) != 6) ++bad;
  for (int it = 0; it < 1000; ++it) {
    double r[3] = {n(g), n(g), n(g)};
    const double s = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (double& v : r) v /= s;
    for (int d = 0; d < pk::dep_count(4); ++d) {
      const int* e = E[pk::dep_monomial(d)];
      double sum = 0.0;
      for (int t = 0; t < pk::dep_terms(d); ++t) {
        const int* k = E[pk::kept_monomial(pk::dep_kept(d, t))];
        sum += pk::dep_coef(d, t) * mono(k[0], k[1], k[2], r);
      }
      const double err = std::fabs(sum - mono(e[0], e[1], e[2], r));
      if (err > worst) worst = err;
    }
  }
  std::printf("bad=%d worst=%.3e\n", bad, worst);
  return (bad == 0 && worst < 1e-13) ? 0 : 1;
}
