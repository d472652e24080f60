// Helpers shared by the MFMA-tile kernels of the FP32-MFMA form (FP32 tiles of
// the G set's tail, FP64 tiles of its head).
#pragma once
#include <hip/hip_runtime.h>

#include "kernel_common.h"
#include "pwdf_internal.h"

namespace pwdf {

__device__ __forceinline__ double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

constexpr double kLog2e = 1.4426950408889634;

// Exponents (a, b, c) of the k-th relative monomial in the degree-ordered,
// descending lexicographic list (the order of Monos), decoded at run time so
// that no table is indexed by a run-time value (that would put it on the stack).
__device__ __forceinline__ void mono_of(int k, int &a, int &b, int &c) {
  int d = 0;
  while (deg_off(d + 1) <= k) ++d;
  int r = k - deg_off(d);
  a = d;
  while (r > d - a) {
    r -= d - a + 1;
    --a;
  }
  b = d - a - r;
  c = d - a - b;
}

// Degree a + b + c of the k-th relative monomial.
__device__ __forceinline__ int mono_degree(int k) {
  int d = 0;
  while (deg_off(d + 1) <= k) ++d;
  return d;
}

// Pair data of the direct evaluation: log2(e)/4p, the fractional coordinates
// of P in the (u, v, w) axis order, and the squared cut radius (a pair sees the
// G with |G|^2 <= gc2; 1e300 without per-pair cuts).
struct PairF {
  double il2, fu, fv, fw, gc2;
};

__device__ __forceinline__ PairF pair_f(const PairHot &h) { return {h.inv4p * kLog2e, h.fu, h.fv, h.fw, h.gc2}; }

}  // namespace pwdf
