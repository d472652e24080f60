// Compile-time index tables shared by the FP64 and FP32 kernels.
#pragma once
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

}  // namespace pwdf
