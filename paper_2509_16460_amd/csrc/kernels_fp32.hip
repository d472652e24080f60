// FP32-MFMA form of the two pair-G passes (gfx950, v_mfma_f32_16x16x4_f32).
//
// Both passes are written as dense contractions over a generated pair-G tile
// S(G, pair) = e^{-|G|^2/4p} e^{-iG.P} (section "Long-range contributions",
// algorithms "non-ortho rho eval" and "non-ortho J eval"):
//
//   rho:  R[G][(k,dm)]  = sum_pair S(G, pair) dhat_k(pair, dm)     (K = pairs)
//         rho(G, dm)    = sum_k n^k (1 or i) R[G][(k,dm)]          (FP64 epilogue;
//         dhat_k = sigma_|k| d_k carries the sign of (-i)^{|k|}, odd |k| take i)
//   J:    yhat[pair][(k,dm)] = sum_G Re( S(G, pair) W'(G, (k,dm)) ), (K = G)
//         W'(G, k, dm) = n^k conj V(G, dm) (x -i for odd |k|),
//
// with n^k the relative monomial n_u^a n_v^b n_w^c.  S is advanced along each
// line segment by the shift-term recurrence in FP64 and rounded to FP32 only as
// an MFMA operand; MFMA accumulates in FP32 inside one pair chunk (rho) or one
// segment chunk (J), and chunks are summed in FP64 afterwards.  The E-coefficient
// transforms, the phase sums and the energy stay FP64 (kernels_fp64.hip).
//
// Lane layout of the 16x16x4 f32 MFMA (lane l = 0..63): A[l%16][l/16],
// B[l/16][l%16], D[4*(l/16)+i][l%16], i = 0..3.
#include <hip/hip_runtime.h>

#include "kernel_common.h"
#include "kernels.h"

namespace pwdf {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

// ---------------------------------------------------------------------------
// rho, K = pairs.  A workgroup = 4 waves = 64 segments (16 per wave as the MFMA
// rows).  The chunk's pairs are staged in LDS in tiles of kQTile pairs (record
// and the coefficient columns of the current N-tile group).  Lane
// (r16 = l%16, g4 = l/16) generates S for segment r16 of its wave and pair g4 of
// each group of four, for all T points of the segment, once per N-tile group,
// and feeds NTG N-tiles (16 columns of (k, dm) each) with it: one MFMA
// accumulator tile per (N-tile, point).  After the chunk the FP64 epilogue
// contracts each N-tile's columns with n^k (times i for odd |k|) and adds the
// lanes of equal density.
// ---------------------------------------------------------------------------
constexpr int kQTile = 64;  // pairs per LDS tile of the rho pass

template <int L, int T, int NTG>
__global__ __launch_bounds__(256) void k_rho_mfma(const SegDesc *__restrict__ segs, int nseg,
                                                  const PairHot *__restrict__ hot, int Lp0, int Lp1, int ppc,
                                                  const float *__restrict__ dh32, int64_t d32_off, int ncols,
                                                  int ndmp, int ndm, double2 *__restrict__ part, int row0,
                                                  int nrows, int nslot, const double *__restrict__ start_tab) {
  constexpr int NT = nherm(L);
  constexpr Monos<L> MT{};
  __shared__ PairHot sh[kQTile];
  __shared__ float sc[kQTile * NTG * 16];
  __shared__ double se2[32];
  __shared__ double scis[130];
  for (int i = threadIdx.x; i < kStartTab; i += blockDim.x) {
    if (i < 32)
      se2[i] = start_tab[i];
    else
      scis[i - 32] = start_tab[i];
  }
  __syncthreads();
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int chunk = blockIdx.y;
  const int p0 = Lp0 + chunk * ppc, p1 = min(Lp1, p0 + ppc);
  const int seg0 = blockIdx.x * 64 + w * 16;
  const int sa = seg0 + r16;
  const SegDesc sdA = segs[sa < nseg ? sa : nseg - 1];
  const float *dcls = dh32 + d32_off;
  const int ntiles = ncols >> 4;

  // lanes r16 < ndm write density r16 of the wave's rows; each N-tile group adds
  // its epilogue into the chunk's partial row (same lane, same addresses: no race)
  double2 *out = part + ((size_t)min(r16, ndm - 1) * nrows + row0 + chunk) * nslot;
  for (int ng = 0; ng < ntiles; ng += NTG) {
    const int ntg = min(NTG, ntiles - ng);
    f4 are[NTG][T], aim[NTG][T];
#pragma unroll
    for (int n = 0; n < NTG; ++n)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        are[n][t] = f4{0.f, 0.f, 0.f, 0.f};
        aim[n][t] = f4{0.f, 0.f, 0.f, 0.f};
      }
    for (int t0 = p0; t0 < p1; t0 += kQTile) {
      const int nq = min(kQTile, p1 - t0);
      __syncthreads();
      for (int i = tid; i < nq; i += 256) sh[i] = hot[t0 + i];
      // coefficient columns [ng*16, (ng+ntg)*16) of the tile's pairs
      // four elements per thread and step, their loads issued before the stores
      for (int i0 = tid; i0 < nq * NTG * 16; i0 += 4 * 256) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int i = i0 + u * 256;
          const int q = i / (NTG * 16), c = i - q * (NTG * 16);
          v[u] = i < nq * NTG * 16 && c < ntg * 16 ? dcls[(size_t)(t0 + q - Lp0) * ncols + ng * 16 + c] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u * 256 < nq * NTG * 16) sc[i0 + u * 256] = v[u];
      }
      __syncthreads();
      for (int q0 = 0; q0 < nq; q0 += 4) {
        const int q = q0 + g4;
        const bool vq = q < nq;
        const PairHot h = sh[vq ? q : 0];
        float Sre[T], Sim[T];
        {
          const double e0 = exp_tab(-sdA.gq0 * h.inv4p, se2);
          const double eR = exp_tab(-sdA.dg0 * h.inv4p, se2);
          double ph = fma((double)sdA.nu0, h.fu, fma((double)sdA.nv, h.fv, (double)sdA.nw * h.fw));
          ph -= rint(ph);
          double cs, sn;
          cis_neg(ph, scis, cs, sn);
          double Sr = e0 * cs, Si = e0 * sn;
          double Rr = eR * h.cu, Ri = eR * h.su;
#pragma unroll
          for (int t = 0; t < T; ++t) {
            Sre[t] = (float)Sr;
            Sim[t] = (float)Si;
            const double tr = fma(Sr, Rr, -Si * Ri);
            Si = fma(Sr, Ri, Si * Rr);
            Sr = tr;
            Rr *= h.q;
            Ri *= h.q;
          }
        }
#pragma unroll
        for (int n = 0; n < NTG; ++n) {
          if (n < ntg) {
            const float b = vq ? sc[q * (NTG * 16) + n * 16 + r16] : 0.f;
#pragma unroll
            for (int t = 0; t < T; ++t) {
              are[n][t] = mfma4(Sre[t], b, are[n][t]);
              aim[n][t] = mfma4(Sim[t], b, aim[n][t]);
            }
          }
        }
      }
    }
    // epilogue of this N-tile group: lane holds R[segment 4*g4+i][column r16] at point t
    double accr[T][4], acci[T][4];
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) accr[t][i] = acci[t][i] = 0.0;
#pragma unroll
    for (int n = 0; n < NTG; ++n) {
      if (n >= ntg) break;
      const int c = (ng + n) * 16 + r16;
      const int k = c / ndmp;
      const bool vk = k < NT;
      const int ka = vk ? MT.u[k] : 0, kb = vk ? MT.v[k] : 0, kc = vk ? MT.w[k] : 0;
      const bool odd = (ka + kb + kc) & 1;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int sr = seg0 + 4 * g4 + i;
        const SegDesc sd = segs[sr < nseg ? sr : nseg - 1];
        const double mvw = ipow((double)sd.nv, kb) * ipow((double)sd.nw, kc);
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const double mono = vk ? ipow((double)(sd.nu0 + t), ka) * mvw : 0.0;
          // d_k carries sigma_|k| already (real part from even |k|, imaginary from odd):
          // the column contributes R for even |k| and i R for odd |k|
          double cr = (double)are[n][t][i], ci = (double)aim[n][t][i];
          if (odd) {
            const double tr = -ci;
            ci = cr;
            cr = tr;
          }
          cr *= mono;
          ci *= mono;
          for (int off = ndmp; off < 16; off <<= 1) {
            cr += __shfl_xor(cr, off, 64);
            ci += __shfl_xor(ci, off, 64);
          }
          accr[t][i] += cr;
          acci[t][i] += ci;
        }
      }
    }
    if (r16 < ndm) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int sr = seg0 + 4 * g4 + i;
        if (sr >= nseg) continue;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          double2 v = make_double2(accr[t][i], acci[t][i]);
          if (ng > 0) {
            const double2 o = out[(size_t)sr * T + t];
            v.x += o.x;
            v.y += o.y;
          }
          out[(size_t)sr * T + t] = v;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// W'[slot][k * ndmp + dm] = n^k conj V(slot, dm) (times -i for odd |k|), so that
// Re(S W') is the parity-selected moment term of the J pass.  Padding slots carry
// V = 0.
// ---------------------------------------------------------------------------
template <int LMAX, int T>
__global__ __launch_bounds__(256) void k_wprep(const double2 *__restrict__ Vc, int nslot, const SegDesc *__restrict__ segs,
                                               int ncolsW, int ndmp, int ndm, float *__restrict__ wre,
                                               float *__restrict__ wim) {
  constexpr int NT = nherm(LMAX);
  constexpr Monos<LMAX> MT{};
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = blockIdx.y;
  if (col >= ncolsW) return;
  const int k = col / ndmp, dm = col - k * ndmp;
  float xr = 0.f, xi = 0.f;
  if (k < NT && dm < ndm) {
    const SegDesc sd = segs[slot / T];
    const int t = slot - (slot / T) * T;
    const int a = MT.u[k], b = MT.v[k], c = MT.w[k];
    const double mono = ipow((double)(sd.nu0 + t), a) * ipow((double)sd.nv, b) * ipow((double)sd.nw, c);
    const double2 v = Vc[(size_t)dm * nslot + slot];
    double r = mono * v.x, i = mono * v.y;
    if ((a + b + c) & 1) {  // -i (r + i i) = i - i r
      const double tr = i;
      i = -r;
      r = tr;
    }
    xr = (float)r;
    xi = (float)i;
  }
  wre[(size_t)slot * ncolsW + col] = xr;
  wim[(size_t)slot * ncolsW + col] = xi;
}

// ---------------------------------------------------------------------------
// J moments, K = G.  A workgroup = 4 waves = 64 pairs (16 per wave as the MFMA
// rows); lane (r16, g4) generates S for pair r16 of its wave on segment g4 of
// each group of four, point by point (one MFMA K-step per point), and feeds NTW
// N-tiles of W' with the same S.  yhat per (segment chunk, k, pair) in FP64.
// ---------------------------------------------------------------------------
template <int L, int T, int NTW>
__global__ __launch_bounds__(256) void k_jpass_mfma(const SegDesc *__restrict__ segs, int nseg, int spc,
                                                    const float *__restrict__ wre, const float *__restrict__ wim,
                                                    int ncolsW, int ntiles, int ndmp, int ndm,
                                                    const PairHot *__restrict__ hot, int Lp0, int Lp1,
                                                    double *__restrict__ yhat, int64_t yhat_size, int64_t ycls_off,
                                                    const double *__restrict__ start_tab) {
  constexpr int NT = nherm(L);
  __shared__ double se2[32];
  __shared__ double scis[130];
  for (int i = threadIdx.x; i < kStartTab; i += blockDim.x) {
    if (i < 32)
      se2[i] = start_tab[i];
    else
      scis[i - 32] = start_tab[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int np = Lp1 - Lp0;
  const int prow0 = blockIdx.x * 64 + w * 16;
  const int chunk = blockIdx.y;
  const int nt0 = blockIdx.z * NTW;
  const int s0 = chunk * spc, s1 = min(nseg, s0 + spc);
  const int pa = prow0 + r16;
  const PairHot h = hot[Lp0 + (pa < np ? pa : 0)];
  f4 acc[NTW];
#pragma unroll
  for (int n = 0; n < NTW; ++n) acc[n] = f4{0.f, 0.f, 0.f, 0.f};
  for (int sg0 = s0; sg0 < s1; sg0 += 4) {
    const int s = sg0 + g4;
    const bool vs = s < s1;
    const SegDesc sd = segs[vs ? s : s0];
    const double e0 = exp_tab(-sd.gq0 * h.inv4p, se2);
    const double eR = exp_tab(-sd.dg0 * h.inv4p, se2);
    double ph = fma((double)sd.nu0, h.fu, fma((double)sd.nv, h.fv, (double)sd.nw * h.fw));
    ph -= rint(ph);
    double cs, sn;
    cis_neg(ph, scis, cs, sn);
    double Sr = e0 * cs, Si = e0 * sn;
    double Rr = eR * h.cu, Ri = eR * h.su;
    const size_t rowW = (size_t)(vs ? s : s0) * T * ncolsW;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float ar = vs ? (float)Sr : 0.f;
      const float ai = vs ? -(float)Si : 0.f;
      const float *wr = wre + rowW + (size_t)t * ncolsW + r16;
      const float *wi = wim + rowW + (size_t)t * ncolsW + r16;
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        if (nt0 + n < ntiles) {
          acc[n] = mfma4(ar, wr[(nt0 + n) * 16], acc[n]);
          acc[n] = mfma4(ai, wi[(nt0 + n) * 16], acc[n]);
        }
      }
      const double tr = fma(Sr, Rr, -Si * Ri);
      Si = fma(Sr, Ri, Si * Rr);
      Sr = tr;
      Rr *= h.q;
      Ri *= h.q;
    }
  }
  // lane holds Y[pair row 4*g4+i][column r16 of each tile]
#pragma unroll
  for (int n = 0; n < NTW; ++n) {
    if (nt0 + n >= ntiles) continue;
    const int col = (nt0 + n) * 16 + r16;
    const int k = col / ndmp, dm = col - k * ndmp;
    if (k >= NT || dm >= ndm) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int prow = prow0 + 4 * g4 + i;
      if (prow < np) yhat[(size_t)dm * yhat_size + ycls_off + ((size_t)chunk * NT + k) * np + prow] = acc[n][i];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define PWDF_CHECK_LAUNCH32()                        \
  do {                                               \
    hipError_t e_ = hipGetLastError();               \
    if (e_ != hipSuccess) return e_;                 \
  } while (0)

template <int L, int T>
static hipError_t rho_mfma_one(const Dev &d, int ndm, hipStream_t st) {
  const int np = d.L_p1[L] - d.L_p0[L];
  if (np <= 0) return hipSuccess;
  dim3 grid((unsigned)((d.nseg + 63) / 64), d.rho_chunks[L]);
  // N-tiles per S generation: all of them when there is one, else as many as the
  // accumulator budget allows
  if (d.ncols32[L] == 16)
    hipLaunchKernelGGL((k_rho_mfma<L, T, 1>), grid, dim3(256), 0, st, d.segs, d.nseg, d.hot, d.L_p0[L], d.L_p1[L],
                       d.rho_ppc[L], d.dh32, d.d32_off[L], d.ncols32[L], d.ndmp, ndm, d.part, d.rho_row0[L],
                       d.nrows, d.nslot, d.start_tab);
  else
    hipLaunchKernelGGL((k_rho_mfma<L, T, (T <= 4 ? 4 : 2)>), grid, dim3(256), 0, st, d.segs, d.nseg, d.hot, d.L_p0[L],
                       d.L_p1[L], d.rho_ppc[L], d.dh32, d.d32_off[L], d.ncols32[L], d.ndmp, ndm, d.part,
                       d.rho_row0[L], d.nrows, d.nslot, d.start_tab);
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

template <int T>
static hipError_t rho_mfma_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (L) {
    case 0: return rho_mfma_one<0, T>(d, ndm, st);
    case 1: return rho_mfma_one<1, T>(d, ndm, st);
    case 2: return rho_mfma_one<2, T>(d, ndm, st);
    case 3: return rho_mfma_one<3, T>(d, ndm, st);
    case 4: return rho_mfma_one<4, T>(d, ndm, st);
    case 5: return rho_mfma_one<5, T>(d, ndm, st);
    case 6: return rho_mfma_one<6, T>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rho_mfma_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (d.seg_len) {
    case 4: return rho_mfma_L<4>(d, L, ndm, st);
    case 8: return rho_mfma_L<8>(d, L, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wprep(const Dev &d, int ndm, hipStream_t st) {
  dim3 grid((unsigned)((d.ncolsW + 255) / 256), d.nslot);
  switch (d.seg_len) {
    case 4:
      hipLaunchKernelGGL((k_wprep<2 * kMaxL, 4>), grid, dim3(256), 0, st, d.Vc, d.nslot, d.segs, d.ncolsW, d.ndmp,
                         ndm, d.wre, d.wim);
      break;
    case 8:
      hipLaunchKernelGGL((k_wprep<2 * kMaxL, 8>), grid, dim3(256), 0, st, d.Vc, d.nslot, d.segs, d.ncolsW, d.ndmp,
                         ndm, d.wre, d.wim);
      break;
    default: return hipErrorInvalidValue;
  }
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

template <int L, int T>
static hipError_t j_mfma_one(const Dev &d, int ndm, hipStream_t st) {
  const int np = d.L_p1[L] - d.L_p0[L];
  if (np <= 0) return hipSuccess;
  constexpr int NTW = 4;
  const int ntiles = d.ncols32[L] / 16;
  dim3 grid((unsigned)((np + 63) / 64), d.j_chunks[L], (unsigned)((ntiles + NTW - 1) / NTW));
  hipLaunchKernelGGL((k_jpass_mfma<L, T, NTW>), grid, dim3(256), 0, st, d.segs, d.nseg, d.j_spc[L], d.wre, d.wim,
                     d.ncolsW, ntiles, d.ndmp, ndm, d.hot, d.L_p0[L], d.L_p1[L], d.yhat, d.yhat_size,
                     d.yhat_off[L], d.start_tab);
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

template <int T>
static hipError_t j_mfma_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (L) {
    case 0: return j_mfma_one<0, T>(d, ndm, st);
    case 1: return j_mfma_one<1, T>(d, ndm, st);
    case 2: return j_mfma_one<2, T>(d, ndm, st);
    case 3: return j_mfma_one<3, T>(d, ndm, st);
    case 4: return j_mfma_one<4, T>(d, ndm, st);
    case 5: return j_mfma_one<5, T>(d, ndm, st);
    case 6: return j_mfma_one<6, T>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_jpass_mfma_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (d.seg_len) {
    case 4: return j_mfma_L<4>(d, L, ndm, st);
    case 8: return j_mfma_L<8>(d, L, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pwdf
