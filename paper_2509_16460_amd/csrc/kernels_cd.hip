// Compact/diffuse classification of the pair densities (section "Density
// classification: compact and diffuse", eq. "cd cutoff").
//
// A primitive pair whose two exponents both lie below alpha_cut is a diffuse
// (DD) pair.  Every interaction with a DD side is taken in full in reciprocal
// space, with v_f(G) = 4 pi / |G|^2 (G != 0), while the compact pairs (CC, CD)
// keep the long-range kernel v(G) among themselves.  With rho = rho_C + rho_D
// split by pair class, the potentials seen by the two kinds of pair are combined
// before the J contraction (the paper combines every planewave-fitted potential
// before its Coulomb construction kernel):
//
//   V_C(G) = v(G) rho_C(G) + v_f(G) rho_D(G)     J of the compact pairs
//   V_D(G) = v_f(G) (rho_C(G) + rho_D(G))        J of the DD pairs
//   E_J    = 1/2 Omega sum_G [rho_C(G) V_C(-G) + rho_D(G) V_D(-G)]
//
// The compact pairs run through the class kernels unchanged (a DD pair's cut of
// -1 takes it out of them; their reduce gives rho_C).  The DD pairs -- a thin
// layer of the most diffuse functions -- are evaluated here, point by point over
// the whole G set, in FP64 in both precision forms: S = e^{-|G|^2/4p}
// e^{-2 pi i n.f_P} from the library exp and sincospi, and the relative-monomial
// polynomial of the pair's coefficients (the density transform's output, in the
// layout of the form).  Sums run in a fixed order (no atomics).
#include <hip/hip_runtime.h>

#include "kernel_common.h"
#include "kernels.h"

namespace pwdf {

// exponents (a, b, c) of the relative monomials n_u^a n_v^b n_w^c in the
// degree-ordered layout of the coefficients and moments
__constant__ Monos<kMaxLsum> kMonoDD = Monos<kMaxLsum>();

// G vector of a slot: relative coordinates (n_u, n_v, n_w) and |G|^2 (false on
// padding); along a segment |G|^2 grows by dg0, dg0 + 2 M_uu, ...
__device__ __forceinline__ bool slot_point(const Dev &d, int slot, double (&n)[3], double &g2) {
  const int sg = slot / d.seg_len, s = slot - sg * d.seg_len;
  const SegDesc sd = d.segs[sg];
  if (s >= sd.cnt) return false;
  n[0] = sd.nu0 + s;
  n[1] = sd.nv;
  n[2] = sd.nw;
  g2 = sd.gq0 + s * sd.dg0 + s * (s - 1.0) * d.muu;
  return true;
}

// S = e^{-|G|^2/4p} e^{-2 pi i n.f_P} of one pair
__device__ __forceinline__ double2 pair_factor(const PairHot &h, const double (&n)[3], double g2) {
  const double e = exp(-g2 * h.inv4p);
  double ph = fma(n[0], h.fu, fma(n[1], h.fv, n[2] * h.fw));
  ph -= rint(ph);
  double sn, cs;
  sincospi(2.0 * ph, &sn, &cs);
  return make_double2(e * cs, -e * sn);
}

// coefficient k of DD pair q (class L) for density dm: FP64 form [dm][class
// block][rho rank][k]; FP32-MFMA form: the FP64 copy in the operand layout
// [class block][cut rank][k * ndmp + dm]
__device__ __forceinline__ double dd_coef(const Dev &d, int q, int L, int k, int dm) {
  if (d.dh32)
    return d.dhat[d.d32_off[L] + (int64_t)(d.cut_rank[q] - d.L_p0[L]) * d.ncols32[L] + k * d.ndmp + dm];
  return d.dhat[(size_t)dm * d.dhat_size + d.dhat_off[L] + (int64_t)(d.rho_rank[q] - d.L_p0[L]) * nherm(L) + k];
}

// rho_D(G) = sum_{DD pairs} S P, P = sum_k d_k n^k (real part from even |k|,
// imaginary from odd |k|): one thread per slot and chunk of DD pairs (grid y),
// the chunk's pairs in list order into its partial row; k_rho_dd_sum adds the
// rows in chunk order
__global__ __launch_bounds__(256) void k_rho_dd(const Dev d) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int chunk = blockIdx.y, dm = blockIdx.z;
  if (slot >= d.nslot) return;
  double n[3], g2;
  double rr = 0.0, ri = 0.0;
  const int i1 = min(d.ndd, (chunk + 1) * d.dd_ppc);
  if (slot_point(d, slot, n, g2)) {
    for (int i = chunk * d.dd_ppc; i < i1; ++i) {
      const int q = d.dd_q[i], L = d.dd_L[i];
      const double2 S = pair_factor(d.hot[q], n, g2);
      double pr = 0.0, pi = 0.0;
      for (int k = 0; k < nherm(L); ++k) {
        const int a = kMonoDD.u[k], b = kMonoDD.v[k], c = kMonoDD.w[k];
        double mono = 1.0;
        for (int e = 0; e < a; ++e) mono *= n[0];
        for (int e = 0; e < b; ++e) mono *= n[1];
        for (int e = 0; e < c; ++e) mono *= n[2];
        const double t = dd_coef(d, q, L, k, dm) * mono;
        if ((a + b + c) & 1)
          pi += t;
        else
          pr += t;
      }
      rr = fma(S.x, pr, fma(-S.y, pi, rr));
      ri = fma(S.x, pi, fma(S.y, pr, ri));
    }
  }
  d.rhoDp[((size_t)dm * d.dd_chunks + chunk) * d.nslot + slot] = make_double2(rr, ri);
}

__global__ __launch_bounds__(256) void k_rho_dd_sum(const Dev d) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x, dm = blockIdx.y;
  if (slot >= d.nslot) return;
  double rr = 0.0, ri = 0.0;
  for (int c = 0; c < d.dd_chunks; ++c) {
    const double2 v = d.rhoDp[((size_t)dm * d.dd_chunks + c) * d.nslot + slot];
    rr += v.x;
    ri += v.y;
  }
  d.rhoD[(size_t)dm * d.nslot + slot] = make_double2(rr, ri);
}

// Per slot: V_C and V_D (stored conjugated, as the J passes read them), rho =
// rho_C + rho_D, and the energy Omega [v |rho_C|^2 + v_f (2 Re rho_C conj rho_D +
// |rho_D|^2)] of the half-space slot (G and -G), summed four slots per block in
// the layout of the reduce's partials.
__global__ __launch_bounds__(64) void k_combine_dd(const Dev d) {
  __shared__ double sh[4];
  const int t = threadIdx.x;
  const int dm = blockIdx.y;
  if (t < 4) {
    const int slot = blockIdx.x * 4 + t;
    double e = 0.0;
    if (slot < d.nslot) {
      const size_t o = (size_t)dm * d.nslot + slot;
      const double v = d.slot_v[slot], vf = d.slot_vf[slot];
      const double2 c = d.rho[o], r = d.rhoD[o];
      const double vcr = fma(v, c.x, vf * r.x), vci = fma(v, c.y, vf * r.y);
      const double tr = c.x + r.x, ti = c.y + r.y;
      d.Vc[o] = make_double2(vcr, -vci);
      d.VDc[o] = make_double2(vf * tr, -vf * ti);
      d.rho[o] = make_double2(tr, ti);
      const double cc = fma(c.x, c.x, c.y * c.y), cr = fma(c.x, r.x, c.y * r.y), rr = fma(r.x, r.x, r.y * r.y);
      e = d.vol * fma(v, cc, vf * fma(2.0, cr, rr));
    }
    sh[t] = e;
  }
  __syncthreads();
  if (t == 0) d.Epart[(size_t)dm * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Moments of one DD pair for one density, y_k = sum_G n^k (Re U if |k| even,
// else Im U), U = conj V_D(G) S(G), over the half space (the J pass's moments,
// with V_D for V_C): the workgroup stages U and the powers n_u^e, n_v^e, n_w^e of
// 256 slots in LDS; the 256 threads form 256 / NT groups of NT, thread (g, k)
// adding moment k over the slots g, g + groups, ... of the tile; at the end the
// groups' sums of each moment are added in group order.  Degree L (J) or L+1
// (force moments).
__global__ __launch_bounds__(256) void k_jpass_dd(const Dev d, int deg, double *__restrict__ out) {
  __shared__ double2 sU[256];
  __shared__ double spw[3][kMaxLsum + 1][256];
  __shared__ double red[256];
  const int i = blockIdx.x, dm = blockIdx.y, t = threadIdx.x;
  const int q = d.dd_q[i];
  const int NT = nherm(d.dd_L[i] + deg);
  const int groups = 256 / NT;
  const int k = t % NT, g = t / NT;
  const bool active = g < groups;
  const PairHot h = d.hot[q];
  const int a = kMonoDD.u[k], b = kMonoDD.v[k], c = kMonoDD.w[k];
  const bool odd = (a + b + c) & 1;
  double acc = 0.0;
  for (int base = 0; base < d.nslot; base += 256) {
    const int slot = base + t;
    double n[3] = {0.0, 0.0, 0.0}, g2;
    double2 U = make_double2(0.0, 0.0);
    if (slot < d.nslot && slot_point(d, slot, n, g2)) {
      const double2 S = pair_factor(h, n, g2);
      const double2 V = d.VDc[(size_t)dm * d.nslot + slot];
      U = make_double2(fma(V.x, S.x, -V.y * S.y), fma(V.x, S.y, V.y * S.x));
    }
    __syncthreads();
    sU[t] = U;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      double pw = 1.0;
#pragma unroll
      for (int e = 0; e <= kMaxLsum; ++e) {
        spw[x][e][t] = pw;
        pw *= n[x];
      }
    }
    __syncthreads();
    if (active) {
      const int m = min(256, d.nslot - base);
      for (int j = g; j < m; j += groups) {
        const double mono = spw[0][a][j] * spw[1][b][j] * spw[2][c][j];
        acc = fma(mono, odd ? sU[j].y : sU[j].x, acc);
      }
    }
  }
  __syncthreads();
  red[t] = active ? acc : 0.0;
  __syncthreads();
  if (t < NT) {
    double s = 0.0;
    for (int gg = 0; gg < groups; ++gg) s += red[gg * NT + t];
    out[((size_t)dm * d.ndd + i) * kDDStride + t] = s;
  }
}

#define PWDF_CHECK_LAUNCH_DD()          \
  do {                                  \
    hipError_t e_ = hipGetLastError();  \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

hipError_t launch_rho_dd(const Dev &d, int ndm, hipStream_t st) {
  const unsigned bx = (unsigned)((d.nslot + 255) / 256);
  hipLaunchKernelGGL(k_rho_dd, dim3(bx, d.dd_chunks, ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_DD();
  hipLaunchKernelGGL(k_rho_dd_sum, dim3(bx, ndm), dim3(256), 0, st, d);
  PWDF_CHECK_LAUNCH_DD();
  return hipSuccess;
}

hipError_t launch_combine_dd(const Dev &d, int ndm, hipStream_t st) {
  hipLaunchKernelGGL(k_combine_dd, dim3((unsigned)d.nred_blocks, ndm), dim3(64), 0, st, d);
  PWDF_CHECK_LAUNCH_DD();
  return hipSuccess;
}

hipError_t launch_jpass_dd(const Dev &d, bool force, int ndm, hipStream_t st) {
  hipLaunchKernelGGL(k_jpass_dd, dim3((unsigned)d.ndd, ndm), dim3(256), 0, st, d, force ? 1 : 0,
                     force ? d.yddF : d.ydd);
  PWDF_CHECK_LAUNCH_DD();
  return hipSuccess;
}

}  // namespace pwdf
