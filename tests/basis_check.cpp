// Host check of the reduced-basis header: the gathered monomials have a power of rhat_z of
// at most 1, kept_monomials evaluates them, for random unit vectors every dependent
// monomial equals its combination of gathered ones, and the factored sums of the x pass
// (monomial_sums.hpp) add w times each gathered monomial at its index (built with
// -D__host__= -D__device__=).
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "basis.hpp"
#include "monomial_sums.hpp"

struct E3 { int a, b, c; };

int main() {
  // exponents of the 50 monomials in the library order: degree 0, 2, 4, 6; x power
  // descending, then y power descending
  std::vector<E3> E;
  for (int n = 0; n <= 6; n += 2)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) E.push_back({a, b, n - a - b});
  int bad = 0;
  if (E.size() != 50) ++bad;
  const int ells[4] = {0, 2, 4, 6}, total[4] = {1, 7, 22, 50};
  for (int i = 0; i < 4; ++i) {
    const int l = ells[i];
    if (pk::kept_count(l) + pk::dep_count(l) != total[i]) ++bad;
    for (int j = 0; j < pk::kept_count(l); ++j)
      if (E[pk::kept_monomial(j)].c > 1 || E[pk::kept_monomial(j)].a + E[pk::kept_monomial(j)].b + E[pk::kept_monomial(j)].c > l) ++bad;
    for (int d = 0; d < pk::dep_count(l); ++d)
      if (E[pk::dep_monomial(d)].c < 2) ++bad;
  }
  std::mt19937_64 g(1505);
  std::normal_distribution<double> nd(0.0, 1.0);
  double worst = 0.0, worst_m = 0.0, worst_s = 0.0;
  for (int it = 0; it < 1000; ++it) {
    double r[3] = {nd(g), nd(g), nd(g)};
    const double s = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (double& v : r) v /= s;
    auto mono = [&](const E3& e) { return std::pow(r[0], e.a) * std::pow(r[1], e.b) * std::pow(r[2], e.c); };
    float m[28];
    pk::kept_monomials<28>((float)r[0], (float)r[1], (float)r[2], m);
    for (int j = 0; j < 28; ++j) worst_m = std::fmax(worst_m, std::fabs(m[j] - mono(E[pk::kept_monomial(j)])));
    // the factored sums for each ell_max, with a weight of either sign, on top of a prior sum
    const double w = nd(g);
    auto check_sums = [&](auto& acc, int ng) {
      for (int j = 0; j < ng; ++j) acc[j] = 0.25f;
      pk::add_monomial_sums(acc, (float)w, (float)r[0], (float)r[1], (float)r[2]);
      for (int j = 0; j < ng; ++j)
        worst_s = std::fmax(worst_s, std::fabs(acc[j] - (0.25 + w * mono(E[pk::kept_monomial(j)]))));
    };
    float a1[1], a6[6], a15[15], a28[28];
    check_sums(a1, 1);
    check_sums(a6, 6);
    check_sums(a15, 15);
    check_sums(a28, 28);
    for (int d = 0; d < pk::dep_count(6); ++d) {
      double sum = 0.0;
      for (int t = 0; t < pk::dep_terms(d); ++t) sum += pk::dep_coef(d, t) * mono(E[pk::kept_monomial(pk::dep_kept(d, t))]);
      worst = std::fmax(worst, std::fabs(sum - mono(E[pk::dep_monomial(d)])));
    }
  }
  std::printf("bad=%d identity=%.3e monomials=%.3e sums=%.3e\n", bad, worst, worst_m, worst_s);
  return (bad == 0 && worst < 1e-13 && worst_m < 1e-6 && worst_s < 4e-6) ? 0 : 1;
}
