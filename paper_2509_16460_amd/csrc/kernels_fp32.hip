// FP32-MFMA form of the two pair-G passes (gfx950, v_mfma_f32_16x16x4_f32).
//
// Both passes are written as dense contractions over a pair-G tile
// S(G, pair) = e^{-|G|^2/4p} e^{-iG.P} generated in FP32 (section "Long-range
// contributions", algorithms "non-ortho rho eval" and "non-ortho J eval"):
//
//   rho:  R[G][(k,dm)]  = sum_pair S(G, pair) dhat_k(pair, dm)     (K = pairs)
//         rho(G, dm)    = sum_k n^k (1 or i) R[G][(k,dm)]          (FP64 epilogue;
//         dhat_k = sigma_|k| d_k carries the sign of (-i)^{|k|}, odd |k| take i)
//   J:    yhat[pair][(k,dm)] = sum_G Re( S(G, pair) W'(G, (k,dm)) ), (K = G)
//         W'(G, k, dm) = n^k conj V(G, dm) (x -i for odd |k|),
//
// with n^k the relative monomial n_u^a n_v^b n_w^c of G = B n.
//
// The tile is evaluated point by point, not by the FP64 shift-term recurrence
// of the FP64 kernels: per (G, pair) the two arguments are reduced in FP64
// (y = -|G|^2 log2(e)/4p split into an integer and a part in [-1/2, 1/2];
// the phase n.f_P reduced mod 1 to [-1/2, 1/2]) and the FP32 hardware
// transcendentals finish it (v_exp_f32 on the reduced exponent, v_sin_f32 /
// v_cos_f32, which take revolutions, on the reduced phase; measured on gfx950
// over [-1/2, 1/2]: 1.4 ulp and 1.2e-7 absolute).  Each S is thus within a few
// FP32 ulp of the exact value, independent of its neighbours, so the rows of an
// MFMA tile can be any 16 G vectors (no line segments, no padding) and a tile
// can be regenerated cheaply for every group of output columns.
//
// MFMA accumulates in FP32 inside one pair chunk (rho) or one G chunk (J);
// chunks are summed in FP64 afterwards.  The E-coefficient transforms, the
// phase sums and the energy stay FP64 (kernels_fp64.hip).
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

constexpr double kLog2e = 1.4426950408889634;

// Pair data of the direct evaluation: log2(e)/4p and the fractional coordinates
// of P in the (u, v, w) axis order.
struct PairF {
  double il2, fu, fv, fw;
};

__device__ __forceinline__ PairF pair_f(const PairHot &h) { return {h.inv4p * kLog2e, h.fu, h.fv, h.fw}; }

// S = e^{-|G|^2/4p} e^{-2 pi i n.f} in FP32 from FP64-reduced arguments.
// |G|^2/4p is at most ~650 (checked by the plan), so y >= -940: the integer part
// fits an int and ldexp underflows smoothly to 0 for the negligible factors.
__device__ __forceinline__ void s_direct(const GPoint &pt, const PairF &f, float &sr, float &si) {
  const double y = -pt.g2 * f.il2;
  const double yi = rint(y);
  const float e = ldexpf(__builtin_amdgcn_exp2f((float)(y - yi)), (int)yi);
  double ph = fma((double)pt.nu, f.fu, fma((double)pt.nv, f.fv, (double)pt.nw * f.fw));
  ph -= rint(ph);
  const float pf = (float)ph;
  sr = e * __builtin_amdgcn_cosf(pf);
  si = -e * __builtin_amdgcn_sinf(pf);
}

// ---------------------------------------------------------------------------
// rho, K = pairs.  A workgroup = 4 waves = 64 G points (16 per wave as the MFMA
// rows) and one chunk of pairs of class L, staged in LDS in tiles of kQTile
// pairs (pair data and the coefficient columns of the current N-tile group).
// Lane (r16 = l%16, g4 = l/16) evaluates S for point r16 of its wave and pair g4
// of each group of four, once per N-tile group, and feeds the NTG N-tiles
// (16 columns of (k, dm) each) of the group with it.  After the chunk the FP64
// epilogue contracts each column with n^k (times i for odd |k|) and adds the
// lanes of equal density.
// ---------------------------------------------------------------------------
constexpr int kQTile = 64;  // pairs per LDS tile of the rho pass

template <int L, int NTG>
__global__ __launch_bounds__(256) void k_rho_mfma(const GPoint *__restrict__ pts, int npts,
                                                  const PairHot *__restrict__ hot, int Lp0, int Lp1, int ppc,
                                                  const float *__restrict__ dh32, int64_t d32_off, int ncols,
                                                  int ndmp, int ndm, double2 *__restrict__ part, int row0,
                                                  int nrows, int nslot) {
  constexpr int NT = nherm(L);
  constexpr Monos<L> MT{};
  __shared__ PairF sh[kQTile];
  __shared__ float sc[kQTile * NTG * 16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int chunk = blockIdx.y;
  const int p0 = Lp0 + chunk * ppc, p1 = min(Lp1, p0 + ppc);
  const int pt0 = blockIdx.x * 64 + w * 16;  // first point of the wave's rows
  const GPoint ptA = pts[min(pt0 + r16, npts - 1)];
  const float *dcls = dh32 + d32_off;
  const int ntiles = ncols >> 4;

  // lanes r16 < ndm write density r16 of the wave's rows; each N-tile group adds
  // its epilogue into the chunk's partial row (same lane, same addresses: no race)
  double2 *out = part + ((size_t)min(r16, ndm - 1) * nrows + row0 + chunk) * nslot;
  for (int ng = 0; ng < ntiles; ng += NTG) {
    const int ntg = min(NTG, ntiles - ng);
    f4 are[NTG], aim[NTG];
#pragma unroll
    for (int n = 0; n < NTG; ++n) {
      are[n] = f4{0.f, 0.f, 0.f, 0.f};
      aim[n] = f4{0.f, 0.f, 0.f, 0.f};
    }
    for (int t0 = p0; t0 < p1; t0 += kQTile) {
      const int nq = min(kQTile, p1 - t0);
      __syncthreads();
      for (int i = tid; i < nq; i += 256) sh[i] = pair_f(hot[t0 + i]);
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
        const bool vq = q0 + g4 < nq;
        const int q = vq ? q0 + g4 : nq - 1;
        float Sr = 0.f, Si = 0.f;
        if (vq) s_direct(ptA, sh[q], Sr, Si);
#pragma unroll
        for (int n = 0; n < NTG; ++n) {
          if (n < ntg) {
            const float b = vq ? sc[q * (NTG * 16) + n * 16 + r16] : 0.f;
            are[n] = mfma4(Sr, b, are[n]);
            aim[n] = mfma4(Si, b, aim[n]);
          }
        }
      }
    }
    // epilogue of this N-tile group: lane holds R[point 4*g4+i][column r16]
    double accr[4], acci[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) accr[i] = acci[i] = 0.0;
    GPoint pr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) pr[i] = pts[min(pt0 + 4 * g4 + i, npts - 1)];
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
        const double mono =
            vk ? ipow((double)pr[i].nu, ka) * ipow((double)pr[i].nv, kb) * ipow((double)pr[i].nw, kc) : 0.0;
        // d_k carries sigma_|k| already (real part from even |k|, imaginary from odd):
        // the column contributes R for even |k| and i R for odd |k|
        double cr = (double)are[n][i], ci = (double)aim[n][i];
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
        accr[i] += cr;
        acci[i] += ci;
      }
    }
    if (r16 < ndm) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pi = pt0 + 4 * g4 + i;
        if (pi >= npts) continue;
        double2 v = make_double2(accr[i], acci[i]);
        if (ng > 0) {
          const double2 o = out[pr[i].slot];
          v.x += o.x;
          v.y += o.y;
        }
        out[pr[i].slot] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// W'[point][k * ndmp + dm] = n^k conj V(slot of the point, dm) (times -i for odd
// |k|), so that Re(S W') is the parity-selected moment term of the J pass.
// Columns past NT * ndm carry zeros.
// ---------------------------------------------------------------------------
template <int LMAX>
__global__ __launch_bounds__(256) void k_wprep(const double2 *__restrict__ Vc, int nslot,
                                               const GPoint *__restrict__ pts, int ncolsW, int ndmp, int ndm,
                                               float *__restrict__ wre, float *__restrict__ wim) {
  constexpr int NT = nherm(LMAX);
  constexpr Monos<LMAX> MT{};
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int pi = blockIdx.y;
  if (col >= ncolsW) return;
  const int k = col / ndmp, dm = col - k * ndmp;
  float xr = 0.f, xi = 0.f;
  if (k < NT && dm < ndm) {
    const GPoint pt = pts[pi];
    const int a = MT.u[k], b = MT.v[k], c = MT.w[k];
    const double mono = ipow((double)pt.nu, a) * ipow((double)pt.nv, b) * ipow((double)pt.nw, c);
    const double2 v = Vc[(size_t)dm * nslot + pt.slot];
    double r = mono * v.x, i = mono * v.y;
    if ((a + b + c) & 1) {  // -i (r + i i) = i - i r
      const double tr = i;
      i = -r;
      r = tr;
    }
    xr = (float)r;
    xi = (float)i;
  }
  wre[(size_t)pi * ncolsW + col] = xr;
  wim[(size_t)pi * ncolsW + col] = xi;
}

// ---------------------------------------------------------------------------
// J moments, K = G.  A workgroup = 4 waves = 64 pairs (16 per wave as the MFMA
// rows); lane (r16, g4) evaluates S for pair r16 of its wave at point g4 of each
// group of four (one MFMA K-step per four points) and feeds NTW N-tiles of W'
// with it.  The points of a chunk are staged in LDS tile by tile.  yhat per
// (G chunk, k, pair) in FP64.
// ---------------------------------------------------------------------------
constexpr int kPTile = 64;  // points per LDS tile of the J pass

template <int L, int NTW>
__global__ __launch_bounds__(256) void k_jpass_mfma(const GPoint *__restrict__ pts, int npts, int ppc,
                                                    const float *__restrict__ wre, const float *__restrict__ wim,
                                                    int ncolsW, int ntiles, int ndmp, int ndm,
                                                    const PairHot *__restrict__ hot, int Lp0, int Lp1,
                                                    double *__restrict__ yhat, int64_t yhat_size, int64_t ycls_off) {
  constexpr int NT = nherm(L);
  __shared__ GPoint sp[kPTile];
  __shared__ float sw[2][kPTile][NTW * 16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int np = Lp1 - Lp0;
  const int prow0 = blockIdx.x * 64 + w * 16;
  const int chunk = blockIdx.y;
  const int nt0 = blockIdx.z * NTW;
  const int ntw = min(NTW, ntiles - nt0);
  const int s0 = min(npts, chunk * ppc), s1 = min(npts, s0 + ppc);
  const int pa = prow0 + r16;
  const PairF f = pair_f(hot[Lp0 + (pa < np ? pa : 0)]);
  f4 acc[NTW];
#pragma unroll
  for (int n = 0; n < NTW; ++n) acc[n] = f4{0.f, 0.f, 0.f, 0.f};
  for (int t0 = s0; t0 < s1; t0 += kPTile) {
    const int nt = min(kPTile, s1 - t0);
    __syncthreads();
    if (tid < nt) sp[tid] = pts[t0 + tid];
    // W' columns [nt0*16, (nt0+ntw)*16) of the tile's points, real and imaginary
    for (int i = tid; i < nt * NTW * 16; i += 256) {
      const int q = i / (NTW * 16), c = i - q * (NTW * 16);
      const bool ok = c < ntw * 16;
      const size_t g = (size_t)(t0 + q) * ncolsW + nt0 * 16 + c;
      sw[0][q][c] = ok ? wre[g] : 0.f;
      sw[1][q][c] = ok ? wim[g] : 0.f;
    }
    __syncthreads();
    for (int q0 = 0; q0 < nt; q0 += 4) {
      const bool vq = q0 + g4 < nt;
      const int q = vq ? q0 + g4 : nt - 1;
      float Sr = 0.f, Si = 0.f;
      if (vq) s_direct(sp[q], f, Sr, Si);
      const float nSi = -Si;
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        if (n < ntw) {
          acc[n] = mfma4(Sr, vq ? sw[0][q][n * 16 + r16] : 0.f, acc[n]);
          acc[n] = mfma4(nSi, vq ? sw[1][q][n * 16 + r16] : 0.f, acc[n]);
        }
      }
    }
  }
  // lane holds Y[pair row 4*g4+i][column r16 of each tile]
#pragma unroll
  for (int n = 0; n < NTW; ++n) {
    if (n >= ntw) continue;
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

template <int L, int NTG>
static hipError_t rho_mfma_ntg(const Dev &d, int ndm, hipStream_t st) {
  dim3 grid((unsigned)((d.npts + 63) / 64), d.rho_chunks[L]);
  hipLaunchKernelGGL((k_rho_mfma<L, NTG>), grid, dim3(256), 0, st, d.pts, d.npts, d.hot, d.L_p0[L], d.L_p1[L],
                     d.rho_ppc[L], d.dh32, d.d32_off[L], d.ncols32[L], d.ndmp, ndm, d.part, d.rho_row0[L],
                     d.nrows, d.nslot);
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

// N-tiles per S generation: all of them up to 8 (accumulators 2 x 8 x 4 VGPRs)
template <int L>
static hipError_t rho_mfma_one(const Dev &d, int ndm, hipStream_t st) {
  const int np = d.L_p1[L] - d.L_p0[L];
  if (np <= 0 || d.npts <= 0) return hipSuccess;
  const int ntiles = d.ncols32[L] / 16;
  if (ntiles <= 1) return rho_mfma_ntg<L, 1>(d, ndm, st);
  if (ntiles <= 2) return rho_mfma_ntg<L, 2>(d, ndm, st);
  if (ntiles <= 4) return rho_mfma_ntg<L, 4>(d, ndm, st);
  return rho_mfma_ntg<L, 8>(d, ndm, st);
}

hipError_t launch_rho_mfma_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (L) {
    case 0: return rho_mfma_one<0>(d, ndm, st);
    case 1: return rho_mfma_one<1>(d, ndm, st);
    case 2: return rho_mfma_one<2>(d, ndm, st);
    case 3: return rho_mfma_one<3>(d, ndm, st);
    case 4: return rho_mfma_one<4>(d, ndm, st);
    case 5: return rho_mfma_one<5>(d, ndm, st);
    case 6: return rho_mfma_one<6>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wprep(const Dev &d, int ndm, hipStream_t st) {
  if (d.npts <= 0) return hipSuccess;
  dim3 grid((unsigned)((d.ncolsW + 255) / 256), d.npts);
  hipLaunchKernelGGL((k_wprep<2 * kMaxL>), grid, dim3(256), 0, st, d.Vc, d.nslot, d.pts, d.ncolsW, d.ndmp, ndm,
                     d.wre, d.wim);
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

template <int L>
static hipError_t j_mfma_one(const Dev &d, int ndm, hipStream_t st) {
  const int np = d.L_p1[L] - d.L_p0[L];
  if (np <= 0 || d.npts <= 0) return hipSuccess;
  constexpr int NTW = 4;
  const int ntiles = d.ncols32[L] / 16;
  dim3 grid((unsigned)((np + 63) / 64), d.j_chunks[L], (unsigned)((ntiles + NTW - 1) / NTW));
  hipLaunchKernelGGL((k_jpass_mfma<L, NTW>), grid, dim3(256), 0, st, d.pts, d.npts, d.j_spc[L], d.wre, d.wim,
                     d.ncolsW, ntiles, d.ndmp, ndm, d.hot, d.L_p0[L], d.L_p1[L], d.yhat, d.yhat_size,
                     d.yhat_off[L]);
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

hipError_t launch_jpass_mfma_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (L) {
    case 0: return j_mfma_one<0>(d, ndm, st);
    case 1: return j_mfma_one<1>(d, ndm, st);
    case 2: return j_mfma_one<2>(d, ndm, st);
    case 3: return j_mfma_one<3>(d, ndm, st);
    case 4: return j_mfma_one<4>(d, ndm, st);
    case 5: return j_mfma_one<5>(d, ndm, st);
    case 6: return j_mfma_one<6>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pwdf
