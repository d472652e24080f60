// Accuracy of the table-driven segment-start factors of the pair-G passes
// (kernel_common.h), compiled for the host: exp_tab against a long double
// exponential, cis_neg against long double cos / sin.  Prints the largest
// errors as "exp_ulp <e> cis_abs <c>".
#include <cmath>
#include <cstdio>
#include <random>

#include "kernel_common.h"

int main() {
  double tab[pwdf::kStartTab];
  pwdf::start_tables(tab);
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const long double pi = 3.141592653589793238462643383279502884L;
  double exp_ulp = 0.0, cis_abs = 0.0;
  for (int i = 0; i < 2000000; ++i) {
    // Gaussian factors -a |G|^2 (down to deep underflow of the normal range) and
    // neighbour ratios of either sign
    const double x = (i % 3 == 0) ? -40.0 * U(g) : -700.0 + 760.0 * U(g);
    const long double ref = expl((long double)x);
    const double v = pwdf::exp_tab(x, tab);
    const double r = (double)ref;
    const double ulp = std::nextafter(r, INFINITY) - r;
    exp_ulp = std::fmax(exp_ulp, (double)(fabsl((long double)v - ref) / ulp));
    const double f = (i % 1000 == 0) ? 0.5 * ((i / 1000) % 3 - 1) : U(g) - 0.5;
    double c, s;
    pwdf::cis_neg(f, tab + 32, c, s);
    const long double rc = cosl(2 * pi * f), rs = -sinl(2 * pi * f);
    cis_abs = std::fmax(cis_abs, (double)fmaxl(fabsl(c - rc), fabsl(s - rs)));
  }
  std::printf("exp_ulp %.4f cis_abs %.4e\n", exp_ulp, cis_abs);
  return 0;
}
