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
#include "mfma_common.h"

namespace pwdf {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

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
// rho over the tail of the G set, K = pairs.  A workgroup = 4 waves = one work
// item: a block of 64 G points (16 per wave as the MFMA rows; points in order of
// |G|^2) and a range of pairs of class L in cut order whose cuts reach the
// block's shortest G, staged in LDS in tiles of kQTile pairs (pair data and the
// coefficient columns of the current N-tile group).  Lane (r16 = l%16, g4 = l/16)
// evaluates S for point r16 of its wave and pair g4 of each group of four, once
// per N-tile group, and feeds the NTG N-tiles (16 columns of (k, dm) each) of
// the group with it; a wave stops at the first group of four whose largest cut
// lies below its shortest G.  After the range the FP64 epilogue contracts each
// column with n^k (times i for odd |k|), adds the lanes of equal density and
// writes the item's partial row.
// ---------------------------------------------------------------------------
constexpr int kQTile = 64;  // pairs per LDS tile of the rho pass

template <int L, int NTG>
__global__ __launch_bounds__(256) void k_rho_mfma(const int4 *__restrict__ items, const GPoint *__restrict__ pts,
                                                  int npts, const PairHot *__restrict__ hot, int Lp0,
                                                  const float *__restrict__ dh32, int64_t d32_off, int ncols,
                                                  int ndmp, int ndm, double2 *__restrict__ part, int nrows,
                                                  const double *__restrict__ pmono, int gps) {
  constexpr int NT = nherm(L);
  __shared__ PairF sh[kQTile];
  __shared__ float sc[kQTile * NTG * 16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int4 it = items[blockIdx.x];  // (point block, q0, q1, row)
  const int p0 = Lp0 + it.y, p1 = Lp0 + it.z;
  const int pt0 = it.x * 64 + w * 16;  // first point of the wave's rows
  const GPoint ptA = pts[min(pt0 + r16, npts - 1)];
  const float *dcls = dh32 + d32_off;
  const int ntiles = ncols >> 4;
  // smallest |G|^2 of the wave's 16 rows (wave-uniform)
  double rmin = pt0 + r16 < npts ? ptA.g2 : 1e300;
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) rmin = fmin(rmin, __shfl_xor(rmin, off, 64));

  // slice blockIdx.z of the N-tile groups: gps groups of NTG tiles, into the
  // item's partial row it.w + z; lanes r16 < ndm write density r16 of the wave's
  // rows; each group of the slice adds its epilogue into that row (same lane,
  // same addresses: no race)
  const int ng0 = blockIdx.z * gps * NTG, ng1 = min(ntiles, ng0 + gps * NTG);
  double2 *out = part + ((size_t)min(r16, ndm - 1) * nrows + it.w + blockIdx.z) * npts;
  for (int ng = ng0; ng < ng1; ng += NTG) {
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
      // branch-free: a lane past the tile's pairs evaluates a valid pair and
      // contributes zero; the columns past the group's tiles are zeros in LDS, so
      // every group runs NTG tiles (a run-time tile count would make the compiler
      // move the accumulators out of the MFMA registers around every MFMA).  The
      // wave stops at the first group of four pairs (cut order: the first has the
      // largest cut) whose cut lies below its shortest G; that count is found
      // first, so that the MFMA loop has one exit and a wave-uniform trip count
      // (an exit inside it has the same effect on the accumulators).
      int qend = nq;
      for (int q0 = 0; q0 < nq; q0 += 4)
        if (sh[q0].gc2 < rmin) {
          qend = q0;
          break;
        }
      qend = __builtin_amdgcn_readfirstlane(qend);
      for (int q0 = 0; q0 < qend; q0 += 4) {
        const int q = q0 + g4 < nq ? q0 + g4 : nq - 1;
        const bool vq = (q0 + g4 < nq) & (ptA.g2 <= sh[q].gc2);  // no branch: q is in range
        float Sr, Si;
        s_direct(ptA, sh[q], Sr, Si);
        Sr = vq ? Sr : 0.f;
        Si = vq ? Si : 0.f;
        const float *bq = sc + q * (NTG * 16) + r16;
#pragma unroll
        for (int n = 0; n < NTG; ++n) {
          const float b = bq[n * 16];
          are[n] = mfma4(Sr, b, are[n]);
          aim[n] = mfma4(Si, b, aim[n]);
        }
      }
    }
    // epilogue of this N-tile group: lane holds R[point 4*g4+i][column r16]
    double accr[4], acci[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) accr[i] = acci[i] = 0.0;
    const double *pm[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) pm[i] = pmono + (size_t)min(pt0 + 4 * g4 + i, npts - 1) * kMonoStride;
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
        if (ng > ng0) {
          const double2 o = out[pi];
          v.x += o.x;
          v.y += o.y;
        }
        out[pi] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// W'[point][k * ndmp + dm] = n^k conj V(slot of the point, dm) (times -i for odd
// |k|), so that Re(S W') is the parity-selected moment term of the J pass.
// Columns past NT * ndm carry zeros.  T = float for the tail's points (FP32
// MFMA operands), double for the head's (FP64 MFMA, kernels_head.hip).
// ---------------------------------------------------------------------------
template <int LMAX, typename T>
__global__ __launch_bounds__(256) void k_wprep(const double2 *__restrict__ Vc, int nslot,
                                               const GPoint *__restrict__ pts, int ncolsW, int ndmp, int ndm,
                                               T *__restrict__ wre, T *__restrict__ wim,
                                               const double *__restrict__ pmono) {
  constexpr int NT = nherm(LMAX);
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int pi = blockIdx.y;
  if (col >= ncolsW) return;
  const int k = col / ndmp, dm = col - k * ndmp;
  T xr = 0, xi = 0;
  if (k < NT && dm < ndm) {
    const GPoint pt = pts[pi];
    const double mono = pmono[(size_t)pi * kMonoStride + k];
    const double2 v = Vc[(size_t)dm * nslot + pt.slot];
    double r = mono * v.x, i = mono * v.y;
    if (mono_degree(k) & 1) {  // -i (r + i i) = i - i r
      const double tr = i;
      i = -r;
      r = tr;
    }
    xr = (T)r;
    xi = (T)i;
  }
  wre[(size_t)pi * ncolsW + col] = xr;
  wim[(size_t)pi * ncolsW + col] = xi;
}

// ---------------------------------------------------------------------------
// J moments over the tail of the G set, K = G.  A workgroup = 4 waves = one work
// item (one N-tile group per workgroup, grid z): a block of 64 pairs of class L
// in cut order (16 per wave as the MFMA rows) and a range of points (in order of
// |G|^2) inside the block's largest cut.  Lane (r16, g4) evaluates S for pair
// r16 of its wave at point g4 of each group of four (one MFMA K-step per four
// points) and feeds NTW N-tiles of W' with it; a wave stops at the first group
// of four whose shortest G lies beyond its largest cut.  The points are staged
// in LDS tile by tile.  yhat per (chunk, k, pair) in FP64.
// ---------------------------------------------------------------------------
// points per LDS tile of the J pass (the W' tile is 2 x kPTile x 16 NTW floats)
template <int NTW>
constexpr int j_ptile() {
  return NTW <= 4 ? 64 : 32;
}

template <int L, int NTW>
__global__ __launch_bounds__(256) void k_jpass_mfma(const int4 *__restrict__ items, const GPoint *__restrict__ pts,
                                                    const float *__restrict__ wre, const float *__restrict__ wim,
                                                    int ncolsW, int ntiles, int ndmp, int ndm,
                                                    const PairHot *__restrict__ hot, int Lp0, int Lp1,
                                                    double *__restrict__ yhat, int64_t yhat_size, int64_t ycls_off,
                                                    int chunk0) {
  constexpr int NT = nherm(L);
  constexpr int kPTile = j_ptile<NTW>();
  __shared__ GPoint sp[kPTile];
  __shared__ float sw[2][kPTile][NTW * 16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  const int np = Lp1 - Lp0;
  const int4 it = items[blockIdx.x];  // (pair block, s0, s1, chunk)
  const int prow0 = it.x * 64 + w * 16;
  const int chunk = chunk0 + it.w;
  const int nt0 = blockIdx.z * NTW;
  const int ntw = min(NTW, ntiles - nt0);
  const int s0 = it.y, s1 = it.z;
  const int pa = prow0 + r16;
  const PairF f = pair_f(hot[Lp0 + (pa < np ? pa : 0)]);
  // largest cut of the wave's 16 rows (wave-uniform)
  double cmax = pa < np ? f.gc2 : 0.0;
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
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
    // branch-free as in the rho pass: columns past the group's tiles are zeros;
    // the wave stops at the first group of four points (in order of |G|^2: the
    // first is the shortest) beyond its largest cut, counted first (see rho)
    int qend = nt;
    for (int q0 = 0; q0 < nt; q0 += 4)
      if (sp[q0].g2 > cmax) {
        qend = q0;
        break;
      }
    qend = __builtin_amdgcn_readfirstlane(qend);
    for (int q0 = 0; q0 < qend; q0 += 4) {
      const int q = q0 + g4 < nt ? q0 + g4 : nt - 1;
      const bool vq = (q0 + g4 < nt) & (sp[q].g2 <= f.gc2);
      float Sr, Si;
      s_direct(sp[q], f, Sr, Si);
      Sr = vq ? Sr : 0.f;
      const float nSi = vq ? -Si : 0.f;
      const float *wr = &sw[0][q][r16], *wi = &sw[1][q][r16];
#pragma unroll
      for (int n = 0; n < NTW; ++n) {
        acc[n] = mfma4(Sr, wr[n * 16], acc[n]);
        acc[n] = mfma4(nSi, wi[n * 16], acc[n]);
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
  const int ntail = d.npts - d.npts_head;
  hipLaunchKernelGGL((k_rho_mfma<L, NTG>), dim3((unsigned)d.rho_nitems[L], 1, (unsigned)d.rho_zs[L]), dim3(256), 0, st,
                     d.rho_items + d.rho_item0[L], d.pts + d.npts_head, ntail, d.hot_cut, d.L_p0[L], d.dh32,
                     d.d32_off[L], d.ncols32[L], d.ndmp, ndm, d.part, d.nrows,
                     d.ptmono + (size_t)d.npts_head * kMonoStride, d.rho_gps[L]);
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

template <int L>
static hipError_t rho_mfma_one(const Dev &d, int ndm, hipStream_t st) {
  if (d.rho_nitems[L] <= 0) return hipSuccess;
  switch (group_tiles(d.ncols32[L] / 16)) {
    case 1: return rho_mfma_ntg<L, 1>(d, ndm, st);
    case 2: return rho_mfma_ntg<L, 2>(d, ndm, st);
    case 3: return rho_mfma_ntg<L, 3>(d, ndm, st);
    case 4: return rho_mfma_ntg<L, 4>(d, ndm, st);
    case 5: return rho_mfma_ntg<L, 5>(d, ndm, st);
    case 6: return rho_mfma_ntg<L, 6>(d, ndm, st);
    case 7: return rho_mfma_ntg<L, 7>(d, ndm, st);
    case 8: return rho_mfma_ntg<L, 8>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
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
  const int ntail = d.npts - d.npts_head;
  if (ntail > 0) {
    dim3 grid((unsigned)((d.ncolsW + 255) / 256), ntail);
    hipLaunchKernelGGL((k_wprep<2 * kMaxL, float>), grid, dim3(256), 0, st, d.Vc, d.nslot, d.pts + d.npts_head,
                       d.ncolsW, d.ndmp, ndm, d.wre, d.wim, d.ptmono + (size_t)d.npts_head * kMonoStride);
    PWDF_CHECK_LAUNCH32();
  }
  if (d.npts_head > 0) {
    dim3 grid((unsigned)((d.ncolsW + 255) / 256), d.npts_head);
    hipLaunchKernelGGL((k_wprep<2 * kMaxL, double>), grid, dim3(256), 0, st, d.Vc, d.nslot, d.pts, d.ncolsW, d.ndmp,
                       ndm, d.wre64, d.wim64, d.ptmono);
    PWDF_CHECK_LAUNCH32();
  }
  return hipSuccess;
}

template <int L, int NTW>
static hipError_t j_mfma_ntw(const Dev &d, int ndm, hipStream_t st) {
  const int ntiles = d.ncols32[L] / 16;
  // yhat chunks [0, jh_chunks[L]) hold the head's moments
  dim3 grid((unsigned)d.j_nitems[L], 1, (unsigned)((ntiles + NTW - 1) / NTW));
  hipLaunchKernelGGL((k_jpass_mfma<L, NTW>), grid, dim3(256), 0, st, d.j_items + d.j_item0[L], d.pts + d.npts_head,
                     d.wre, d.wim, d.ncolsW, ntiles, d.ndmp, ndm, d.hot_cut, d.L_p0[L], d.L_p1[L], d.yhat,
                     d.yhat_size, d.yhat_off[L], d.jh_chunks[L]);
  PWDF_CHECK_LAUNCH32();
  return hipSuccess;
}

// N-tile groups (grid z) as for rho: ceil(ntiles / 8) groups of equal size
template <int L>
static hipError_t j_mfma_one(const Dev &d, int ndm, hipStream_t st) {
  if (d.j_nitems[L] <= 0) return hipSuccess;
  switch (group_tiles(d.ncols32[L] / 16)) {
    case 1: return j_mfma_ntw<L, 1>(d, ndm, st);
    case 2: return j_mfma_ntw<L, 2>(d, ndm, st);
    case 3: return j_mfma_ntw<L, 3>(d, ndm, st);
    case 4: return j_mfma_ntw<L, 4>(d, ndm, st);
    case 5: return j_mfma_ntw<L, 5>(d, ndm, st);
    case 6: return j_mfma_ntw<L, 6>(d, ndm, st);
    case 7: return j_mfma_ntw<L, 7>(d, ndm, st);
    case 8: return j_mfma_ntw<L, 8>(d, ndm, st);
    default: return hipErrorInvalidValue;
  }
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
