// The head of the G set in the FP32-MFMA form: FP64 tiles on FP64 MFMA
// (gfx950, v_mfma_f64_16x16x4_f64).
//
// The Coulomb weight v(G) = 4 pi e^{-|G|^2/4w^2} / |G|^2 falls by orders of
// magnitude over the first shells of G vectors, so the terms of largest size in
// both contractions sit on the few shortest G.  There the rounding of FP32
// operands and FP32 accumulation would set the error of E_J and J; the head --
// the G whose weight is at least a set fraction of the largest (2^-20 by
// default) -- is therefore contracted in FP64 here, with the same tile structure
// as the FP32 kernels:
//
//   rho:  R[G][(k,dm)] = sum_pair S(G, pair) dhat_k(pair, dm)   (K = pairs)
//   J:    yhat[pair][(k,dm)] = sum_G Re( S(G, pair) W'(G, (k,dm)) )   (K = G)
//
// S(G, pair) = e^{-|G|^2/4p} e^{-2 pi i n.f_P} is evaluated directly in FP64 per
// (G, pair) (the table-driven exponential and phase factor of the FP64 passes,
// tables in LDS); the coefficients come from the FP64 transform output and
// W' = n^k conj V(G) (times -i for odd |k|) is formed once per build in FP64
// (k_wprep).  The head rho rows go to their own partial rows (one per chunk of
// pairs and N-tile group), the J moments to the first jh_chunks chunks of yhat;
// the reduction and the back transform add them.
//
// Lane layout of the 16x16x4 f64 MFMA (lane l = 0..63): A[l%16][l/16],
// B[l/16][l%16], D[4*i + l/16][l%16], i = 0..3 (the rows of D interleave across
// the four lane groups, unlike the f32 form of the same shape).
#include <hip/hip_runtime.h>

#include "kernel_common.h"
#include "kernels.h"
#include "mfma_common.h"

namespace pwdf {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma4d(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Pair data of the FP64 evaluation: 1/4p, the fractional coordinates of P in
// the (u, v, w) axis order, the squared cut radius.
struct PairD {
  double inv4p, fu, fv, fw, gc2;
};

__device__ __forceinline__ PairD pair_d(const PairHot &h) { return {h.inv4p, h.fu, h.fv, h.fw, h.gc2}; }

// the segment-start tables (2^(j/32); e^{2 pi i j/64}) copied into LDS
__device__ __forceinline__ void head_tables(const double *__restrict__ g, double *e2, double *cis) {
  for (int i = threadIdx.x; i < kStartTab; i += blockDim.x) {
    if (i < 32)
      e2[i] = g[i];
    else
      cis[i - 32] = g[i];
  }
}

// S = e^{-|G|^2/4p} e^{-2 pi i n.f} in FP64, by the table-driven exponential and
// phase factor of the FP64 passes (about 1 ulp each; |G|^2/4p is bounded by the
// plan, the phase is reduced mod 1 first)
__device__ __forceinline__ void s_direct64(const GPoint &pt, const PairD &f, const double *e2, const double *cis,
                                           double &sr, double &si) {
  const double e = exp_tab(-pt.g2 * f.inv4p, e2);
  double ph = fma((double)pt.nu, f.fu, fma((double)pt.nv, f.fv, (double)pt.nw * f.fw));
  ph -= rint(ph);
  double c, s;
  cis_neg(ph, cis, c, s);
  sr = e * c;
  si = e * s;
}

// ---------------------------------------------------------------------------
// rho over the head points, K = pairs.  A workgroup = 4 waves = 64 points (16 per
// wave as the MFMA rows), one chunk of pairs of class L and one group of NTG
// N-tiles (grid z); the pairs are staged in LDS in tiles of kQTileH with the
// group's FP64 coefficient columns (the transform's FP64 output in the layout of
// the FP32 operands, [pair][k * ndmp + dm]).  Output: the partial row of (chunk,
// group), [dm][row][head point].
// ---------------------------------------------------------------------------
constexpr int kQTileH = 32;  // LDS: 32 KB of coefficient columns at NTG = 8

template <int L, int NTG>
__global__ __launch_bounds__(256) void k_rho_head(const GPoint *__restrict__ pts, int npts,
                                                  const PairHot *__restrict__ hot, int Lp0, int Lp1, int ppc,
                                                  const double *__restrict__ dh64, int64_t d_off, int ncols,
                                                  int ndmp, int ndm, double2 *__restrict__ parth, int row0,
                                                  int nrows_h, const double *__restrict__ pmono,
                                                  const double *__restrict__ start_tab) {
  constexpr int NT = nherm(L);
  constexpr int PER = kQTileH * NTG * 16 / 256;  // staged columns per thread and tile
  static_assert(PER * 256 == kQTileH * NTG * 16, "tile size");
  __shared__ PairD sh[kQTileH];
  __shared__ double sc[kQTileH * NTG * 16];
  __shared__ double se2[32], scis[2 * 65];
  head_tables(start_tab, se2, scis);  // (the tile loop's first barrier orders it)
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int chunk = blockIdx.y, grp = blockIdx.z;
  const int p0 = Lp0 + chunk * ppc, p1 = min(Lp1, p0 + ppc);
  const int pt0 = blockIdx.x * 64 + w * 16;
  const GPoint ptA = pts[min(pt0 + r16, npts - 1)];
  const int ntiles = ncols >> 4;
  const int ng = grp * NTG, ntg = min(NTG, ntiles - ng);
  d4 are[NTG], aim[NTG];
#pragma unroll
  for (int n = 0; n < NTG; ++n) {
    are[n] = d4{0.0, 0.0, 0.0, 0.0};
    aim[n] = d4{0.0, 0.0, 0.0, 0.0};
  }
  for (int t0 = p0; t0 < p1; t0 += kQTileH) {
    const int nq = min(kQTileH, p1 - t0);
    __syncthreads();
    if (tid < nq) sh[tid] = pair_d(hot[t0 + tid]);
    // the group's columns of the tile's pairs, loads issued before the stores;
    // columns of densities past ndm were not written by this call's transform
    // and are masked (the FP64 buffer is not cleared)
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = tid + u * 256;
      const int q = i / (NTG * 16), c = i - q * (NTG * 16);
      const int col = ng * 16 + c;
      const int k = col / ndmp, dm = col - k * ndmp;
      v[u] = q < nq && c < ntg * 16 && k < NT && dm < ndm ? dh64[d_off + (size_t)(t0 + q - Lp0) * ncols + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) sc[tid + u * 256] = v[u];
    __syncthreads();
    for (int q0 = 0; q0 < nq; q0 += 4) {
      const int q = q0 + g4 < nq ? q0 + g4 : nq - 1;
      const bool vq = (q0 + g4 < nq) & (ptA.g2 <= sh[q].gc2);  // no branch: q is in range
      double Sr, Si;
      s_direct64(ptA, sh[q], se2, scis, Sr, Si);
      Sr = vq ? Sr : 0.0;
      Si = vq ? Si : 0.0;
      const double *bq = sc + q * (NTG * 16) + r16;
#pragma unroll
      for (int n = 0; n < NTG; ++n) {
        const double b = bq[n * 16];
        are[n] = mfma4d(Sr, b, are[n]);
        aim[n] = mfma4d(Si, b, aim[n]);
      }
    }
  }
  // epilogue: lane holds R[point 4*i + g4][column r16]
  double accr[4], acci[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) accr[i] = acci[i] = 0.0;
  const double *pm[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) pm[i] = pmono + (size_t)min(pt0 + 4 * i + g4, npts - 1) * kMonoStride;
#pragma unroll
  for (int n = 0; n < NTG; ++n) {
    if (n >= ntg) break;
    const int c = (ng + n) * 16 + r16;
    const int k = c / ndmp;
    const bool vk = k < NT;
    const bool odd = vk && (mono_degree(k) & 1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double mono = vk ? pm[i][k] : 0.0;
      // even |k|: R; odd |k|: i R (the sign of (-i)^|k| is in the coefficients)
      double cr = are[n][i], ci = aim[n][i];
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
    double2 *out = parth + ((size_t)r16 * nrows_h + row0 + chunk * gridDim.z + grp) * npts;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pi = pt0 + 4 * i + g4;
      if (pi < npts) out[pi] = make_double2(accr[i], acci[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// J moments over the head points, K = G.  A workgroup = 4 waves = 64 pairs (16 per
// wave as the MFMA rows); the head points and their W' columns (formed once per
// build in FP64 by k_wprep) are staged in LDS tile by tile, the next tile's
// loads issued before the barrier that ends the current one; grid y splits the
// head points into chunks.  Output: yhat chunk blockIdx.y of the class, (k, pair).
// ---------------------------------------------------------------------------
// head points per LDS tile (the W' tile is 2 x kPTile x 16 NTW doubles, <= 32 KB)
template <int NTW>
constexpr int jh_ptile() {
  return NTW <= 4 ? 32 : 16;
}

template <int L, int NTW>
__global__ __launch_bounds__(256) void k_jpass_head(const GPoint *__restrict__ pts, int npts, int ppc,
                                                    const double *__restrict__ wre, const double *__restrict__ wim,
                                                    int ncolsW, int ntiles, int ndmp,
                                                    const PairHot *__restrict__ hot, int Lp0, int Lp1,
                                                    double *__restrict__ yhat, int64_t yhat_size, int64_t ycls_off,
                                                    int ndm, const double *__restrict__ start_tab) {
  constexpr int NT = nherm(L);
  constexpr int kPTile = jh_ptile<NTW>();
  __shared__ GPoint sp[kPTile];
  __shared__ double sw[2][kPTile][NTW * 16];
  __shared__ double se2[32], scis[2 * 65];
  head_tables(start_tab, se2, scis);  // (the tile loop's barriers order it)
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int np = Lp1 - Lp0;
  const int prow0 = blockIdx.x * 64 + w * 16;
  const int nt0 = blockIdx.z * NTW;
  const int ntw = min(NTW, ntiles - nt0);
  const int pa = prow0 + r16;
  const PairD f = pair_d(hot[Lp0 + (pa < np ? pa : 0)]);
  d4 acc[NTW];
#pragma unroll
  for (int n = 0; n < NTW; ++n) acc[n] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int PER = kPTile * NTW * 16 / 256;  // W' elements per thread and tile
  static_assert(PER * 256 == kPTile * NTW * 16, "tile size");
  // chunk blockIdx.y: head points [c ppc, (c + 1) ppc), moments to yhat chunk c
  const int pend = min(npts, (int)(blockIdx.y + 1) * ppc);
  for (int t0 = blockIdx.y * ppc; t0 < pend; t0 += kPTile) {
    const int nt = min(kPTile, pend - t0);
    // the tile's point records and W' elements (columns of k >= NT, densities
    // past ndm and points past the tile read as zeros), loaded before the barrier
    const GPoint *pp = pts + t0 + min(tid, nt - 1);
    const double pg2 = pp->g2;
    const int pnu = pp->nu, pnv = pp->nv, pnw = pp->nw, pslot = pp->slot;
    double2 x[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = tid + u * 256;
      const int q = i / (NTW * 16), c = i - q * (NTW * 16);
      const int col = (nt0 * 16) + c;
      const bool ok = q < nt && c < ntw * 16 && col / ndmp < NT;
      const size_t o = ok ? (size_t)(t0 + q) * ncolsW + col : 0;
      x[u] = make_double2(wre[o], wim[o]);
      if (!ok) x[u] = make_double2(0.0, 0.0);
    }
    __syncthreads();  // the previous tile's MFMA reads are done
    if (tid < nt) {
      sp[tid].g2 = pg2;
      sp[tid].nu = pnu;
      sp[tid].nv = pnv;
      sp[tid].nw = pnw;
      sp[tid].slot = pslot;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = tid + u * 256;
      const int q = i / (NTW * 16), c = i - q * (NTW * 16);
      sw[0][q][c] = x[u].x;
      sw[1][q][c] = x[u].y;
    }
    __syncthreads();
    for (int q0 = 0; q0 < nt; q0 += 4) {
      const int q = q0 + g4 < nt ? q0 + g4 : nt - 1;
      const bool vq = (q0 + g4 < nt) & (sp[q].g2 <= f.gc2);
      double Sr, Si;
      s_direct64(sp[q], f, se2, scis, Sr, Si);
      Sr = vq ? Sr : 0.0;
      const double nSi = vq ? -Si : 0.0;
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        acc[n] = mfma4d(Sr, sw[0][q][n * 16 + r16], acc[n]);
        acc[n] = mfma4d(nSi, sw[1][q][n * 16 + r16], acc[n]);
      }
    }
  }
  // lane holds Y[pair row 4*i + g4][column r16 of each tile]
#pragma unroll
  for (int n = 0; n < NTW; ++n) {
    if (n >= ntw) continue;
    const int col = (nt0 + n) * 16 + r16;
    const int k = col / ndmp, dm = col - k * ndmp;
    if (k >= NT || dm >= ndm) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int prow = prow0 + 4 * i + g4;
      if (prow < np)
        yhat[(size_t)dm * yhat_size + ycls_off + ((size_t)blockIdx.y * NT + k) * np + prow] = acc[n][i];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define PWDF_CHECK_LAUNCH_H()          \
  do {                                 \
    hipError_t e_ = hipGetLastError(); \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

template <int L, int NTG>
static hipError_t rho_head_ntg(const Dev &d, int ndm, hipStream_t st) {
  dim3 grid((unsigned)((d.npts_head + 63) / 64), d.rho_h_chunks[L], (unsigned)tile_groups(d.ncols32[L] / 16));
  hipLaunchKernelGGL((k_rho_head<L, NTG>), grid, dim3(256), 0, st, d.pts, d.npts_head, d.hot_cut, d.L_p0[L], d.L_p1[L],
                     d.rho_h_ppc[L], d.dhat, d.d32_off[L], d.ncols32[L], d.ndmp, ndm, d.parth, d.rho_h_row0[L],
                     d.nrows_h, d.ptmono, d.start_tab);
  PWDF_CHECK_LAUNCH_H();
  return hipSuccess;
}

template <int L>
static hipError_t rho_head_one(const Dev &d, int ndm, hipStream_t st) {
  const int np = d.L_p1[L] - d.L_p0[L];
  if (np <= 0 || d.npts_head <= 0 || d.rho_h_chunks[L] <= 0) return hipSuccess;
  switch (group_tiles(d.ncols32[L] / 16)) {
    case 1: return rho_head_ntg<L, 1>(d, ndm, st);
    case 2: return rho_head_ntg<L, 2>(d, ndm, st);
    case 3: return rho_head_ntg<L, 3>(d, ndm, st);
    case 4: return rho_head_ntg<L, 4>(d, ndm, st);
    case 5: return rho_head_ntg<L, 5>(d, ndm, st);
    case 6: return rho_head_ntg<L, 6>(d, ndm, st);
    case 7: return rho_head_ntg<L, 7>(d, ndm, st);
    case 8: return rho_head_ntg<L, 8>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rho_head_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (L) {
    case 0: return rho_head_one<0>(d, ndm, st);
    case 1: return rho_head_one<1>(d, ndm, st);
    case 2: return rho_head_one<2>(d, ndm, st);
    case 3: return rho_head_one<3>(d, ndm, st);
    case 4: return rho_head_one<4>(d, ndm, st);
    case 5: return rho_head_one<5>(d, ndm, st);
    case 6: return rho_head_one<6>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

template <int L, int NTW>
static hipError_t j_head_ntw(const Dev &d, int ndm, hipStream_t st) {
  const int np = d.L_p1[L] - d.L_p0[L];
  const int ntiles = d.ncols32[L] / 16;
  // the head's moments are chunks [0, jh_chunks[L]) of the class
  const int64_t off = d.yhat_off[L];
  dim3 grid((unsigned)((np + 63) / 64), (unsigned)d.jh_chunks[L], (unsigned)((ntiles + NTW - 1) / NTW));
  hipLaunchKernelGGL((k_jpass_head<L, NTW>), grid, dim3(256), 0, st, d.pts, d.npts_head, d.jh_ppc[L], d.wre64,
                     d.wim64, d.ncolsW, ntiles, d.ndmp, d.hot_cut, d.L_p0[L], d.L_p1[L], d.yhat, d.yhat_size, off,
                     ndm, d.start_tab);
  PWDF_CHECK_LAUNCH_H();
  return hipSuccess;
}

template <int L>
static hipError_t j_head_one(const Dev &d, int ndm, hipStream_t st) {
  const int np = d.L_p1[L] - d.L_p0[L];
  if (np <= 0 || d.npts_head <= 0 || d.jh_chunks[L] <= 0) return hipSuccess;
  switch (group_tiles(d.ncols32[L] / 16)) {
    case 1: return j_head_ntw<L, 1>(d, ndm, st);
    case 2: return j_head_ntw<L, 2>(d, ndm, st);
    case 3: return j_head_ntw<L, 3>(d, ndm, st);
    case 4: return j_head_ntw<L, 4>(d, ndm, st);
    case 5: return j_head_ntw<L, 5>(d, ndm, st);
    case 6: return j_head_ntw<L, 6>(d, ndm, st);
    case 7: return j_head_ntw<L, 7>(d, ndm, st);
    case 8: return j_head_ntw<L, 8>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_jpass_head_L(const Dev &d, int L, int ndm, hipStream_t st) {
  switch (L) {
    case 0: return j_head_one<0>(d, ndm, st);
    case 1: return j_head_one<1>(d, ndm, st);
    case 2: return j_head_one<2>(d, ndm, st);
    case 3: return j_head_one<3>(d, ndm, st);
    case 4: return j_head_one<4>(d, ndm, st);
    case 5: return j_head_one<5>(d, ndm, st);
    case 6: return j_head_one<6>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pwdf
