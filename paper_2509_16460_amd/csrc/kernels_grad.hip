// Nuclear gradient of E_J at fixed D(k), pair list and G set (adjoint form).
//
//   dE_J/dR = sum_unique w sum_ab D_ab(L) 2 Re sum_{G half space} conj V(G) dF_abL(G)/dR
//
// (E_J = 1/2 Omega sum_G v |rho|^2, rho linear in F).  The centre derivative of a
// Cartesian Gaussian, d/dA_x (x-A_x)^l e^{-a(x-A_x)^2} = 2a (x-A_x)^{l+1}(...) -
// l (x-A_x)^{l-1}(...), keeps the Gaussian product (same p, P), so dF/dA_x has a
// Hermite expansion of degree L+1 with coefficients 2 a_a E^{a+1_x, b} -
// a_x E^{a-1_x, b}; the J pass of degree L+1 over the class-L pairs supplies
// Y_t = sum_G conj V S (-iG)^t and this kernel contracts it with those
// coefficients and with D.  V(G) is the one of the energy evaluation.
#include <hip/hip_runtime.h>

#include "kernel_common.h"
#include "kernels.h"

namespace pwdf {

template <int LA, int LB>
__global__ __launch_bounds__(64) void k_force_back(const BlockRec *__restrict__ blocks, int b0, int b1,
                                                   const PairAux *__restrict__ aux, const double *__restrict__ ttab,
                                                   const double *__restrict__ yF, int64_t yF_size, int64_t yF_off,
                                                   int nchunks, int Lp0, int Lp1, const int *__restrict__ cut_rank,
                                                   const double *__restrict__ Dblk, int64_t nelem,
                                                   double *__restrict__ gblk, int nblocks,
                                                   const int *__restrict__ dd_of, const double *__restrict__ yddF,
                                                   int ndd) {
  constexpr int L = LA + LB;
  constexpr int L1 = L + 1;
  constexpr int NT1 = nherm(L1);
  constexpr Carts<LA> CA{};
  constexpr Carts<LB> CB{};
  constexpr int NCA = ncart(LA), NCB = ncart(LB);
  const int bi = b0 + blockIdx.x * blockDim.x + threadIdx.x;
  const int dm = blockIdx.y;
  if (bi >= b1) return;
  const BlockRec b = blocks[bi];
  const int np = Lp1 - Lp0;
  const double *D = Dblk + (size_t)dm * nelem + b.eoff;
  double gA[3] = {0.0, 0.0, 0.0}, gB[3] = {0.0, 0.0, 0.0};
  for (int q = b.p0; q < b.p1; ++q) {
    const double *ys = yF + (size_t)dm * yF_size + yF_off + (cut_rank[q] - Lp0);  // J walk order
    // a DD pair (compact/diffuse classification) takes its force moments of V_D
    // from the DD kernel
    const int dq = dd_of ? dd_of[q] : -1;
    double y[NT1];
#pragma unroll
    for (int k = 0; k < NT1; ++k) {
      double s = 0.0;
      if (dq >= 0) {
        s = yddF[((size_t)dm * ndd + dq) * kDDStride + k];
      } else {
        for (int c = 0; c < nchunks; ++c) s += ys[((size_t)c * NT1 + k) * np];
      }
      y[k] = s;
    }
    // Hermite moments J~_t = Re sum_G conj V S (-iG)^t, |t| <= L+1
    double Jt[NT1];
#pragma unroll
    for (int d = 0; d <= L1; ++d) {
      const int nc = ncart(d);
      const double *T = ttab + tblk_off(d);
      const double sg = ((d & 3) >= 2) ? -1.0 : 1.0;
#pragma unroll
      for (int t = 0; t < nc; ++t) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < nc; ++k) s = fma(T[t * nc + k], y[deg_off(d) + k], s);
        Jt[deg_off(d) + t] = sg * s;
      }
    }
    const PairAux x = aux[q];
    const double inv2p = 0.5 / x.p;
    double Ex[LA + 2][LB + 2][L + 3], Ey[LA + 2][LB + 2][L + 3], Ez[LA + 2][LB + 2][L + 3];
    md_axis<LA + 1, LB + 1>(inv2p, x.xpa[0], x.xpb[0], Ex);
    md_axis<LA + 1, LB + 1>(inv2p, x.xpa[1], x.xpb[1], Ey);
    md_axis<LA + 1, LB + 1>(inv2p, x.xpa[2], x.xpb[2], Ez);
    const double ta = 2.0 * x.alpha_a, tb = 2.0 * x.alpha_b;
#pragma unroll
    for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
      for (int ib = 0; ib < NCB; ++ib) {
        const int la3[3] = {CA.x[ia], CA.y[ia], CA.z[ia]};
        const int lb3[3] = {CB.x[ib], CB.y[ib], CB.z[ib]};
        const double dab = D[ia * NCB + ib] * x.w * x.pref_j;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // derivative along axis c on centre A (da) and centre B (db)
          double da = 0.0, db = 0.0;
          const int ax = la3[0], ay = la3[1], az = la3[2];
          const int bx = lb3[0], by = lb3[1], bz = lb3[2];
#pragma unroll
          for (int tx = 0; tx <= ax + bx + 1; ++tx)
#pragma unroll
            for (int ty = 0; ty <= ay + by + 1; ++ty)
#pragma unroll
              for (int tz = 0; tz <= az + bz + 1; ++tz) {
                const int tsum = tx + ty + tz;
                if (tsum > L1) continue;
                // only the differentiated axis may exceed the undifferentiated range
                if (c != 0 && tx > ax + bx) continue;
                if (c != 1 && ty > ay + by) continue;
                if (c != 2 && tz > az + bz) continue;
                const int t = deg_off(tsum) + mono_idx(tx, ty, tz);
                const double J = Jt[t];
                // E products with the raised / lowered exponent on axis c
                double ea = 0.0, eb = 0.0;
                if (c == 0) {
                  const double oth = Ey[ay][by][ty] * Ez[az][bz][tz];
                  double ra = ta * Ex[ax + 1][bx][tx];
                  if (ax > 0) ra -= ax * Ex[ax - 1][bx][tx];
                  double rb = tb * Ex[ax][bx + 1][tx];
                  if (bx > 0) rb -= bx * Ex[ax][bx - 1][tx];
                  ea = ra * oth;
                  eb = rb * oth;
                } else if (c == 1) {
                  const double oth = Ex[ax][bx][tx] * Ez[az][bz][tz];
                  double ra = ta * Ey[ay + 1][by][ty];
                  if (ay > 0) ra -= ay * Ey[ay - 1][by][ty];
                  double rb = tb * Ey[ay][by + 1][ty];
                  if (by > 0) rb -= by * Ey[ay][by - 1][ty];
                  ea = ra * oth;
                  eb = rb * oth;
                } else {
                  const double oth = Ex[ax][bx][tx] * Ey[ay][by][ty];
                  double ra = ta * Ez[az + 1][bz][tz];
                  if (az > 0) ra -= az * Ez[az - 1][bz][tz];
                  double rb = tb * Ez[az][bz + 1][tz];
                  if (bz > 0) rb -= bz * Ez[az][bz - 1][tz];
                  ea = ra * oth;
                  eb = rb * oth;
                }
                da = fma(ea, J, da);
                db = fma(eb, J, db);
              }
          gA[c] = fma(dab, da, gA[c]);
          gB[c] = fma(dab, db, gB[c]);
        }
      }
  }
  double *out = gblk + ((size_t)dm * nblocks + bi) * 6;
  out[0] = gA[0];
  out[1] = gA[1];
  out[2] = gA[2];
  out[3] = gB[0];
  out[4] = gB[1];
  out[5] = gB[2];
}

// dE/dR for every atom: fixed-order sum over the atom's (block, centre) entries.
__global__ __launch_bounds__(256) void k_force_atoms(const double *__restrict__ gblk, int nblocks,
                                                     const int *__restrict__ atom_off,
                                                     const int *__restrict__ atom_ent, int natm,
                                                     double *__restrict__ dEdR) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int dm = blockIdx.y;
  if (i >= natm * 3) return;
  const int atom = i / 3, c = i - 3 * atom;
  const double *g = gblk + (size_t)dm * nblocks * 6;
  double s = 0.0;
  for (int e = atom_off[atom]; e < atom_off[atom + 1]; ++e) s += g[(size_t)atom_ent[e] + c];
  dEdR[((size_t)dm * natm + atom) * 3 + c] = s;
}

#define PWDF_CHECK_LAUNCHG()                         \
  do {                                               \
    hipError_t e_ = hipGetLastError();               \
    if (e_ != hipSuccess) return e_;                 \
  } while (0)

template <int LA, int LB>
static hipError_t fback_one(const Dev &d, int ndm, hipStream_t st) {
  const int c = LA * 4 + LB;
  const int b0 = d.cls_b0[c], b1 = d.cls_b1[c];
  if (b1 <= b0) return hipSuccess;
  constexpr int L = LA + LB;
  dim3 grid((unsigned)((b1 - b0 + 63) / 64), ndm);
  hipLaunchKernelGGL((k_force_back<LA, LB>), grid, dim3(64), 0, st, d.blocks, b0, b1, d.aux, d.ttab, d.yF, d.yF_size,
                     d.yF_off[L], d.j_chunks[L], d.L_p0[L], d.L_p1[L], d.cut_rank, d.Dblk, d.nelem, d.gblk,
                     d.nblocks, d.ndd > 0 ? d.dd_of : nullptr, d.yddF, d.ndd);
  PWDF_CHECK_LAUNCHG();
  return hipSuccess;
}

hipError_t launch_force_back_cls(const Dev &d, int la, int lb, int ndm, hipStream_t st) {
  switch (la * 4 + lb) {
    case 0: return fback_one<0, 0>(d, ndm, st);
    case 4: return fback_one<1, 0>(d, ndm, st);
    case 5: return fback_one<1, 1>(d, ndm, st);
    case 8: return fback_one<2, 0>(d, ndm, st);
    case 9: return fback_one<2, 1>(d, ndm, st);
    case 10: return fback_one<2, 2>(d, ndm, st);
    case 12: return fback_one<3, 0>(d, ndm, st);
    case 13: return fback_one<3, 1>(d, ndm, st);
    case 14: return fback_one<3, 2>(d, ndm, st);
    case 15: return fback_one<3, 3>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_force_atoms(const Dev &d, int ndm, double *dEdR, hipStream_t st) {
  dim3 grid((unsigned)((d.natm * 3 + 255) / 256), ndm);
  hipLaunchKernelGGL(k_force_atoms, grid, dim3(256), 0, st, d.gblk, d.nblocks, d.atom_off, d.atom_ent, d.natm, dEdR);
  PWDF_CHECK_LAUNCHG();
  return hipSuccess;
}

}  // namespace pwdf
