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

}  // namespace pwdf
