// Compile-time index tables shared by the FP64 and FP32 kernels.
#pragma once
#include <cmath>

#include "pwdf_internal.h"

namespace pwdf {

// ---------------------------------------------------------------------------
// compile-time monomial tables: degree-ordered, descending lexicographic
// ---------------------------------------------------------------------------
template <int L>
struct Monos {
  int u[nherm(L)], v[nherm(L)], w[nherm(L)];
  constexpr Monos() : u(), v(), w() {
    int n = 0;
    for (int d = 0; d <= L; ++d)
      for (int a = d; a >= 0; --a)
        for (int b = d - a; b >= 0; --b) {
          u[n] = a;
          v[n] = b;
          w[n] = d - a - b;
          ++n;
        }
  }
};

// Cartesian components of one shell, descending lexicographic (lx, ly, lz).
template <int l>
struct Carts {
  int x[ncart(l)], y[ncart(l)], z[ncart(l)];
  constexpr Carts() : x(), y(), z() {
    int n = 0;
    for (int a = l; a >= 0; --a)
      for (int b = l - a; b >= 0; --b) {
        x[n] = a;
        y[n] = b;
        z[n] = l - a - b;
        ++n;
      }
  }
};

__host__ __device__ constexpr int mono_idx(int a, int b, int c) {
  // index of (a,b,c) inside its degree block, descending lexicographic
  int d = a + b + c;
  int idx = 0;
  for (int x = d; x > a; --x) idx += d - x + 1;
  return idx + (d - a) - b;
}

// ---------------------------------------------------------------------------
// McMurchie-Davidson Hermite coefficients along one axis:
//   x_A^i x_B^j e^{-p x_P^2} = sum_t E[i][j][t] d^t/dP^t e^{-p x_P^2}
//   E[i+1][j][t] = E[i][j][t-1]/(2p) + X_PA E[i][j][t] + (t+1) E[i][j][t+1]
// ---------------------------------------------------------------------------
template <int LA, int LB>
__device__ __forceinline__ void md_axis(double inv2p, double xpa, double xpb,
                                        double (&E)[LA + 1][LB + 1][LA + LB + 1]) {
#pragma unroll
  for (int i = 0; i <= LA; ++i)
#pragma unroll
    for (int j = 0; j <= LB; ++j)
#pragma unroll
      for (int t = 0; t <= LA + LB; ++t) E[i][j][t] = 0.0;
  E[0][0][0] = 1.0;
#pragma unroll
  for (int i = 0; i <= LA; ++i)
#pragma unroll
    for (int j = 0; j <= LB; ++j) {
      if (i == 0 && j == 0) continue;
#pragma unroll
      for (int t = 0; t <= i + j; ++t) {
        double v;
        if (i > 0) {
          v = xpa * E[i - 1][j][t];
          if (t > 0) v += inv2p * E[i - 1][j][t - 1];
          if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
        } else {
          v = xpb * E[i][j - 1][t];
          if (t > 0) v += inv2p * E[i][j - 1][t - 1];
          if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
        }
        E[i][j][t] = v;
      }
    }
}

// ---------------------------------------------------------------------------
// Segment-start factors of the pair-G passes, table-driven (Tang's method for
// the exponential):
//   e^x = 2^m 2^(j/32) e^r,  n = rint(32 x / ln 2) = 32 m + j (0 <= j < 32),
//   r = x - n ln2/32 (|r| <= ln2/64; ln2/32 split in a head and a tail, two
//   fma steps), e^r - 1 by its Taylor series to r^6 (remainder below 4e-18);
//   e^{-2 pi i f} for f in [-1/2, 1/2]: the table value e^{-2 pi i j/64}
//   (j = rint(64 f)) times e^{-i theta}, theta = 2 pi (f - j/64) (the difference
//   is exact), |theta| <= pi/64, by the Taylor series of cos - 1 to theta^8 and
//   of sin to theta^9 (remainders below 1e-19).
// The small parts are carried as corrections so that the table values enter
// with one rounding (about 1 ulp).  No range handling: the arguments are
// bounded (|x| < 700 for the Gaussian factor and its neighbour ratio; f is
// reduced mod 1 first).  Tables (kStartTab doubles): 2^(j/32) for j = 0..31,
// then (cos, sin)(2 pi j/64) for j = -32..32.
// ---------------------------------------------------------------------------
constexpr int kStartTab = 32 + 2 * 65;

inline void start_tables(double *t) {
  for (int j = 0; j < 32; ++j) t[j] = (double)exp2l((long double)j / 32);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = -32; j <= 32; ++j) {
    t[32 + 2 * (j + 32)] = (double)cosl(2 * pi * j / 64);
    t[33 + 2 * (j + 32)] = (double)sinl(2 * pi * j / 64);
  }
}

__host__ __device__ inline double exp_tab(double x, const double *e2) {
  constexpr double k32_ln2 = 46.16624130844683;
  constexpr double ln2_32_hi = 0.02166084939249829, ln2_32_lo = 7.247021293269686e-19;
  const double n = rint(x * k32_ln2);
  double r = fma(-n, ln2_32_hi, x);
  r = fma(-n, ln2_32_lo, r);
  const int ni = (int)n;
  double p = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  // 2^(j/32) e^r = T + T (e^r - 1)
  const double t = e2[ni & 31];
  return ldexp(fma(t, p * r, t), ni >> 5);
}

// (c, s) = (cos 2 pi f, -sin 2 pi f) = e^{-2 pi i f}, f in [-1/2, 1/2]; cis is
// the (cos, sin) table of 65 pairs
__host__ __device__ inline void cis_neg(double f, const double *cis, double &c, double &s) {
  constexpr double k2pi = 6.283185307179586;
  const double jd = rint(f * 64.0);
  const double th = fma(jd, -1.0 / 64.0, f) * k2pi;
  const double t2 = th * th;
  double cm = fma(t2, 1.0 / 40320.0, -1.0 / 720.0);  // cos(theta) - 1
  cm = fma(cm, t2, 1.0 / 24.0);
  cm = fma(cm, t2, -0.5);
  cm *= t2;
  double sn = fma(t2, 1.0 / 362880.0, -1.0 / 5040.0);
  sn = fma(sn, t2, 1.0 / 120.0);
  sn = fma(sn, t2, -1.0 / 6.0);
  sn = fma(sn, t2, 1.0);
  sn *= th;
  const int k = 2 * ((int)jd + 32);
  const double tc = cis[k], ts = cis[k + 1];
  c = tc + fma(tc, cm, -ts * sn);
  s = -(ts + fma(ts, cm, tc * sn));
}

}  // namespace pwdf
