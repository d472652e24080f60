// FP64 kernels of libpwdf for gfx950.
//
// Pipeline per density (section "Long-range contributions"):
//   k_phase_d      D(k) -> D(L) on the unique pair blocks            (eq. "FT for D")
//   k_transform    per primitive pair: D block x McMurchie-Davidson Hermite
//                  coefficients -> Hermite coefficients -> relative-monomial
//                  coefficients d_k                                  (algorithm "density matrix transformation")
//   k_rho          rho(G) partial sums: lane = one segment of a G line, the
//                  wave walks a chunk of pairs                       (algorithm "non-ortho rho eval")
//   k_reduce       sum of partial rows, V(G) = v rho, energy partials (contraction step 2)
//   k_jpass        lane = one pair, the wave walks a chunk of segments and
//                  accumulates the relative-monomial moments of conj(V) F
//                                                                    (algorithm "non-ortho J eval")
//   k_backtransform moments -> Hermite -> Cartesian J block          (algorithm "J matrix transformation")
//   k_phase_j      J(L) -> J(k), dense output                        (eq. "FT of J")
//
// Per pair and G the transform is
//   F_abL(G) = C e^{-|G|^2/4p} e^{-iG.P} sum_t E^{ab}_t (-iG)^t
// (Hermite expansion of the Gaussian product; the transform of the t-th
// derivative of e^{-p x_P^2} with respect to P carries (-iG)^t), and with
// G = B n the Cartesian monomials G^t are rewritten as relative monomials
// n_u^a n_v^b n_w^c (appendix "Expansion of angular prefactor in relative
// coordinate"), so along a line (n_v, n_w fixed) the polynomial is a
// one-variable polynomial in n_u and the Gaussian/phase factor follows the
// shift-term recurrence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "kernel_common.h"
#include "kernels.h"

namespace pwdf {

// ---------------------------------------------------------------------------
// Phase factors of the k <-> L sums: for the k-point (k1,k2,k3) of an
// n1 x n2 x n3 mesh and the image m, k.L/2pi = sum_i k_i m_i / n_i, an integer
// multiple t of 1/N (N = lcm of the n_i).  An image enters only through its
// Born-von Karman class c_i = (m_i mod n_i) N / n_i, so t = k1 c1 + k2 c2 + k3 c3
// and the phase is ptab[t] = e^{2 pi i t / N} (t < (n1+n2+n3) N, no reduction).
// Class codes pack (c1, c2, c3) as c1 | c2 << 10 | c3 << 20; k-points are
// walked in the order k = (k1 n2 + k2) n3 + k3.
// ---------------------------------------------------------------------------

// a1: D(k) -> D(L) on the unique blocks (real part: the Hermitian input makes
// the imaginary part cancel between (a,b,L) and its mirror (b,a,-L)).  One thread
// per (matrix element, BvK class) segment, segments ordered by element so that
// the lanes of a wave read neighbouring elements of D(k) (kU loads in flight);
// D_c = Re sum_k w_k e^{ik.L} D(k)[mu][nu] is the same for every image of the
// class and is written to each of them.
constexpr int kU = 8;

// copies the segment-start tables into LDS (callers synchronise before use)
__device__ __forceinline__ void load_start_tabs(const double *__restrict__ g, double *e2, double2 *cis) {
  for (int i = threadIdx.x + threadIdx.y * blockDim.x; i < kStartTab; i += blockDim.x * blockDim.y) {
    if (i < 32)
      e2[i] = g[i];
    else if ((i - 32) % 2 == 0)
      cis[(i - 32) / 2] = make_double2(g[i], g[i + 1]);
  }
}

__device__ __forceinline__ double2 cis_neg(double f, const double2 *__restrict__ cis) {
  double c, s;
  cis_neg(f, reinterpret_cast<const double *>(cis), c, s);
  return make_double2(c, s);
}

__global__ __launch_bounds__(256) void k_phase_d(const double2 *__restrict__ Dk, int nk, int64_t nn, int n2, int n3,
                                                 int nsegD, const int *__restrict__ sD_el,
                                                 const int *__restrict__ sD_code, const int *__restrict__ sD_e0,
                                                 const int *__restrict__ eD, const double2 *__restrict__ ptab,
                                                 int ptab_len, double wk, double *__restrict__ Dblk, int64_t nelem,
                                                 int *__restrict__ nonfinite) {
  __shared__ double2 sph[kPtabMax];
  for (int i = threadIdx.x; i < ptab_len; i += blockDim.x) sph[i] = ptab[i];
  __syncthreads();
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  const int dm = blockIdx.y;
  if (sg >= nsegD) return;
  const int code = sD_code[sg];
  const int c1 = code & 1023, c2 = (code >> 10) & 1023, c3 = code >> 20;
  const double2 *D = Dk + (size_t)dm * nk * nn + sD_el[sg];
  double acc = 0.0;
  // the phase of k = (k1, k2, k3) is the table's per-axis steps raised to k1, k2,
  // k3: it advances by one complex multiplication per k (k3 fastest; the row
  // starts kept for the wrap-arounds), at most n1 + n2 + n3 products from the
  // exact table values
  const double2 o1 = sph[c1], o2 = sph[c2], o3 = sph[c3];
  double2 w1 = make_double2(1.0, 0.0), w2 = w1, w = w1;
  int k2 = 0, k3 = 0;
  for (int kb = 0; kb < nk; kb += kU) {
    double2 d[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) d[u] = kb + u < nk ? D[(size_t)(kb + u) * nn] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      acc = fma(w.x, d[u].x, fma(-w.y, d[u].y, acc));  // zero past nk
      if (++k3 == n3) {
        k3 = 0;
        if (++k2 == n2) {
          k2 = 0;
          w1 = make_double2(fma(w1.x, o1.x, -w1.y * o1.y), fma(w1.x, o1.y, w1.y * o1.x));
          w2 = w1;
        } else {
          w2 = make_double2(fma(w2.x, o2.x, -w2.y * o2.y), fma(w2.x, o2.y, w2.y * o2.x));
        }
        w = w2;
      } else {
        w = make_double2(fma(w.x, o3.x, -w.y * o3.y), fma(w.x, o3.y, w.y * o3.x));
      }
    }
  }
  const double v = acc * wk;
  // a non-finite D(k) value read makes the phase sum non-finite (NaN or inf
  // propagates through the products); the host reads the flag on request
  if (!isfinite(v)) *nonfinite = 1;
  double *out = Dblk + (size_t)dm * nelem;
  for (int j = sD_e0[sg]; j < sD_e0[sg + 1]; ++j) out[eD[j]] = v;
}

// ---------------------------------------------------------------------------
// a2: per block of class (LA, LB): for every primitive pair
//   D~_t = pref_rho sum_{a,b} D_ab E^x_{ax bx tx} E^y_{ay by ty} E^z_{az bz tz}
//   d_k  = sigma_|k| sum_{|t| = |k|} T[t][k] D~_t,  sigma = (+,-,-,+)[|k| mod 4]
// so that rho's polynomial along a line is sum_k d_k n^k with even |k| in the
// real part and odd |k| in the imaginary part.
// ---------------------------------------------------------------------------
template <int LA, int LB>
__device__ __forceinline__ void transform_thread(const Dev &dv, int bi, int dm) {
  constexpr int L = LA + LB;
  constexpr int NT = nherm(L);
  constexpr Carts<LA> CA{};
  constexpr Carts<LB> CB{};
  constexpr int NCA = ncart(LA), NCB = ncart(LB);
  const PairAux *__restrict__ aux = dv.aux;
  const double *__restrict__ Dblk = dv.Dblk;
  const double *__restrict__ ttab = dv.ttab;
  double *__restrict__ dhat = dv.dhat;
  float *__restrict__ dh32 = dv.dh32;
  const int64_t nelem = dv.nelem, dhat_size = dv.dhat_size, cls_off = dv.dhat_off[L], d32_off = dv.d32_off[L];
  const int Lp0 = dv.L_p0[L], ncols = dv.ncols32[L], ndmp = dv.ndmp;
  const BlockRec b = dv.blocks[bi];
  const double *D = Dblk + (size_t)dm * nelem + b.eoff;
  double *out_base = dhat + (size_t)dm * dhat_size + cls_off;
  for (int q = b.p0; q < b.p1; ++q) {
    const PairAux x = aux[q];
    const double inv2p = 0.5 / x.p;
    double Ex[LA + 1][LB + 1][L + 1], Ey[LA + 1][LB + 1][L + 1], Ez[LA + 1][LB + 1][L + 1];
    md_axis<LA, LB>(inv2p, x.xpa[0], x.xpb[0], Ex);
    md_axis<LA, LB>(inv2p, x.xpa[1], x.xpb[1], Ey);
    md_axis<LA, LB>(inv2p, x.xpa[2], x.xpb[2], Ez);
    double Dt[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) Dt[t] = 0.0;
#pragma unroll
    for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
      for (int ib = 0; ib < NCB; ++ib) {
        const double dab = D[ia * NCB + ib] * x.pref_rho;
        const int ax = CA.x[ia], ay = CA.y[ia], az = CA.z[ia];
        const int bx = CB.x[ib], by = CB.y[ib], bz = CB.z[ib];
#pragma unroll
        for (int tx = 0; tx <= ax + bx; ++tx)
#pragma unroll
          for (int ty = 0; ty <= ay + by; ++ty) {
            const double exy = dab * Ex[ax][bx][tx] * Ey[ay][by][ty];
#pragma unroll
            for (int tz = 0; tz <= az + bz; ++tz) {
              const int t = deg_off(tx + ty + tz) + mono_idx(tx, ty, tz);
              Dt[t] = fma(exy, Ez[az][bz][tz], Dt[t]);
            }
          }
      }
    double *out = out_base + (size_t)(dv.rho_rank[q] - Lp0) * NT;  // rho's walk order
#pragma unroll
    for (int d = 0; d <= L; ++d) {
      const int nc = ncart(d);
      const double *T = ttab + tblk_off(d);
      const double sg = ((d & 3) == 1 || (d & 3) == 2) ? -1.0 : 1.0;
#pragma unroll
      for (int k = 0; k < nc; ++k) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < nc; ++t) s = fma(T[t * nc + k], Dt[deg_off(d) + t], s);
        // FP32-MFMA form: [pair][k * ndmp + dm], in FP32 for the tiles of the G
        // set's tail and in FP64 (dhat in that layout) for the tiles of its head
        if (dh32) {
          const size_t o = d32_off + (size_t)(dv.cut_rank[q] - Lp0) * ncols + (deg_off(d) + k) * ndmp + dm;
          dh32[o] = (float)(sg * s);
          dhat[o] = sg * s;
        } else {
          out[deg_off(d) + k] = sg * s;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// a3: rho(G) partial sums.  Lane = one segment (SEG consecutive n_u of a line);
// the W waves of a workgroup share 64 segments and split a chunk of pairs of
// class L.  Pair records are staged in LDS tile by tile (wave-uniform reads).
//   rho(n) += S(n) P(n),   P(n_u) = sum_a C_a n_u^a  (Horner),
//   C_a = sum_{b,c} d_{abc} n_v^b n_w^c  (real part from even a+b+c, imaginary
//   from odd), S advanced by S <- S R, R <- q R.
// The W partial sums are added in LDS (fixed order) into one row per workgroup.
// ---------------------------------------------------------------------------
template <int L>
struct RhoTile {
  static constexpr int NT = nherm(L);
  static constexpr int REC = 8 + NT;  // PairHot (8 doubles) + coefficients
  static constexpr int TP = NT <= 20 ? 64 : 32;
};

// Contributions of one pair (LDS record r: PairHot, then NT coefficients for each
// of NDB densities) to the SEG points of one segment.  The Gaussian/phase factor
// S is generated once and shared by the densities; each density keeps its own
// accumulators, filled in the same pair order as a one-density call.
// CUT: the pair sees only the points with |G|^2 <= its gc2 (record field 7);
// g2s holds |G|^2 of the lane's SEG points.
template <int L, int SEG, int NDB, bool CUT>
__device__ __forceinline__ void rho_pair(const double *__restrict__ r, const SegDesc &sd, const double (&mv)[L + 1],
                                         const double (&mw)[L + 1], double (&accr)[NDB][SEG],
                                         double (&acci)[NDB][SEG], const double *__restrict__ e2,
                                         const double2 *__restrict__ cis, double &pc, double &e0, double &eR,
                                         const double (&g2s)[SEG]) {
  constexpr int NT = nherm(L);
  constexpr Monos<L> MT{};
  const double nu0 = sd.nu0, nv = sd.nv, nw = sd.nw;
  const double inv4p = r[0], fu = r[1], fv = r[2], fw = r[3];
  double cr[NDB][L + 1], ci[NDB][L + 1];
#pragma unroll
  for (int b = 0; b < NDB; ++b) {
    const double *d = r + 8 + b * NT;
#pragma unroll
    for (int a = 0; a <= L; ++a) cr[b][a] = ci[b][a] = 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      const int a = MT.u[k], bb = MT.v[k], c = MT.w[k];
      const double t = d[k] * (mv[bb] * mw[c]);
      if ((a + bb + c) & 1)
        ci[b][a] += t;
      else
        cr[b][a] += t;
    }
  }
  // |S| and |R| at the segment start depend on the pair only through p: the low
  // classes (walked in order of p) keep them from the previous pair of this wave
  // when its p is the same; the high classes, whose register pressure makes the
  // branch cost more than the exponentials, always evaluate them
  if (L > 2 || inv4p != pc) {
    pc = inv4p;
    e0 = exp_tab(-sd.gq0 * inv4p, e2);
    eR = exp_tab(-sd.dg0 * inv4p, e2);
  }
  double ph = fma(nu0, fu, fma(nv, fv, nw * fw));
  ph -= rint(ph);
  const double2 w = cis_neg(ph, cis);
  double Sr_ = e0 * w.x, Si_ = e0 * w.y;
  double Rr = eR * r[4], Ri = eR * r[5];
  const double q = r[6];
  // the degree-L coefficient exists only in the part of parity L (real for even
  // L, imaginary for odd L): the Horner sums start below it in the other part
  constexpr int topR = (L & 1) ? L - 1 : L, topI = (L & 1) ? L : L - 1;
  const double gc2 = r[7];
#pragma unroll
  for (int s = 0; s < SEG; ++s) {
    const double n = nu0 + s;
    // the point's share: S, or 0 outside the pair's cut
    const double Sr = CUT && g2s[s] > gc2 ? 0.0 : Sr_, Si = CUT && g2s[s] > gc2 ? 0.0 : Si_;
#pragma unroll
    for (int b = 0; b < NDB; ++b) {
      double Pr = cr[b][topR];
#pragma unroll
      for (int a = topR - 1; a >= 0; --a) Pr = fma(Pr, n, cr[b][a]);
      if constexpr (L == 0) {
        accr[b][s] = fma(Sr, Pr, accr[b][s]);
        acci[b][s] = fma(Si, Pr, acci[b][s]);
      } else {
        double Pi = ci[b][topI];
#pragma unroll
        for (int a = topI - 1; a >= 0; --a) Pi = fma(Pi, n, ci[b][a]);
        accr[b][s] = fma(Sr, Pr, fma(-Si, Pi, accr[b][s]));
        acci[b][s] = fma(Sr, Pi, fma(Si, Pr, acci[b][s]));
      }
    }
    const double tr = fma(Sr_, Rr, -Si_ * Ri);
    Si_ = fma(Sr_, Ri, Si_ * Rr);
    Sr_ = tr;
    Rr *= q;
    Ri *= q;
  }
}

template <int L, int SEG, int W, int NDB, bool CUT>
__device__ __forceinline__ void rho_block(const Dev &dv, int sgi, int chunk, int db, int ndm, double *__restrict__ sp,
                                          double2 *__restrict__ red, const double *__restrict__ e2,
                                          const double2 *__restrict__ cis) {
  constexpr int NT = nherm(L);
  constexpr int REC = 8 + NT * NDB;
  constexpr int TP = RhoTile<L>::TP;
  const SegDesc *__restrict__ segs = dv.segs;
  const PairHot *__restrict__ hot = dv.hot_rho;  // walk order, as the coefficients
  const double *__restrict__ dhat = dv.dhat;
  double2 *__restrict__ part = dv.part;
  const int nseg = dv.nseg, Lp0 = dv.L_p0[L], Lp1 = dv.L_p1[L], pairs_per_chunk = dv.rho_ppc[L];
  const int row0 = dv.rho_row0[L], nrows = dv.nrows, nslot = dv.nslot;
  const int64_t dhat_size = dv.dhat_size, cls_off = dv.dhat_off[L];
  const int lane = threadIdx.x, w = threadIdx.y, tid = w * 64 + lane;
  const int seg = sgi * 64 + lane;
  const int p0 = Lp0 + chunk * pairs_per_chunk;
  const int p1 = min(Lp1, p0 + pairs_per_chunk);
  const bool active = seg < nseg;
  const SegDesc sd = segs[active ? seg : 0];
  double mv[L + 1], mw[L + 1];
  mv[0] = 1.0;
  mw[0] = 1.0;
#pragma unroll
  for (int b = 1; b <= L; ++b) {
    mv[b] = mv[b - 1] * sd.nv;
    mw[b] = mw[b - 1] * sd.nw;
  }
  double accr[NDB][SEG], acci[NDB][SEG];
#pragma unroll
  for (int b = 0; b < NDB; ++b)
#pragma unroll
    for (int s = 0; s < SEG; ++s) accr[b][s] = acci[b][s] = 0.0;
  const int dm0 = db * NDB;
  double pc = -1.0, e0 = 0.0, eR = 0.0;  // p-dependent start factors of the last pair (inv4p > 0)
  // per-pair cuts: |G|^2 of the lane's points, and the smallest |G|^2 of the
  // block's 64 segments (a pair whose cut lies below it is skipped by every wave)
  double g2s[SEG];
  double wmin = 1e300;
  if constexpr (CUT) {
    double g2 = sd.gq0, dg = sd.dg0;
#pragma unroll
    for (int s = 0; s < SEG; ++s) {
      g2s[s] = g2;
      g2 += dg;
      dg += 2.0 * dv.muu;
    }
    wmin = active ? sd.g2min : 1e300;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wmin = fmin(wmin, __shfl_xor(wmin, off, 64));
  }
  for (int t0 = p0; t0 < p1; t0 += TP) {
    const int nt = min(TP, p1 - t0);
    __syncthreads();
    // pair records: PairHot, then the coefficients of densities dm0 .. dm0+NDB-1
    // (zeros past ndm)
    // four elements per thread and step, their loads issued before the stores
    for (int i0 = tid; i0 < nt * REC; i0 += 4 * 64 * W) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * 64 * W;
        const int pi = i / REC, f = i - pi * REC;
        const double *src = nullptr;
        if (i < nt * REC) {
          if (f < 8) {
            src = reinterpret_cast<const double *>(hot + t0 + pi) + f;
          } else {
            const int b = (f - 8) / NT, k = (f - 8) - b * NT;
            if (dm0 + b < ndm) src = dhat + (size_t)(dm0 + b) * dhat_size + cls_off + (size_t)(t0 + pi - Lp0) * NT + k;
          }
        }
        v[u] = src ? *src : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u * 64 * W < nt * REC) sp[i0 + u * 64 * W] = v[u];
    }
    __syncthreads();
    for (int j = w; j < nt; j += W) {
      if (CUT && sp[j * REC + 7] < wmin) continue;
      rho_pair<L, SEG, NDB, CUT>(sp + j * REC, sd, mv, mw, accr, acci, e2, cis, pc, e0, eR, g2s);
    }
  }
  // the W waves' partial sums are added in LDS in fixed order, one density at a time
  if (W > 1) {
#pragma unroll
    for (int b = 0; b < NDB; ++b) {
      if (w > 0) {
#pragma unroll
        for (int s = 0; s < SEG; ++s) red[((w - 1) * SEG + s) * 64 + lane] = make_double2(accr[b][s], acci[b][s]);
      }
      __syncthreads();
      if (w == 0) {
#pragma unroll
        for (int v = 1; v < W; ++v)
#pragma unroll
          for (int s = 0; s < SEG; ++s) {
            const double2 x = red[((v - 1) * SEG + s) * 64 + lane];
            accr[b][s] += x.x;
            acci[b][s] += x.y;
          }
      }
      __syncthreads();
    }
    if (w > 0) return;
  }
  if (!active) return;
#pragma unroll
  for (int b = 0; b < NDB; ++b) {
    if (dm0 + b >= ndm) break;
    double2 *out = part + ((size_t)(dm0 + b) * nrows + row0 + chunk) * nslot + (size_t)seg * SEG;
#pragma unroll
    for (int s = 0; s < SEG; ++s) out[s] = make_double2(accr[b][s], acci[b][s]);
  }
}

// ---------------------------------------------------------------------------
// a4: rho = sum of the partial rows in a fixed order (two stages: groups of
// rows, then the groups), V = v rho stored conjugated for the J pass, and the
// energy partials Omega sum v |rho|^2 per block (G half space).
// ---------------------------------------------------------------------------
// FP32-MFMA form (slot_pidx non-null): a slot's rows are those of its point --
// the head's partial rows [nrows_h][nhead] for a head point, else the first
// rows_of_block[b] tail rows [nrows][ntail] of its point block b; padding slots
// sum nothing.
__global__ __launch_bounds__(256) void k_reduce_rows(const double2 *__restrict__ part, int nrows, int nslot,
                                                     int rows_per_group, double2 *__restrict__ part2,
                                                     int ngroups, const int *__restrict__ slot_pidx,
                                                     const double2 *__restrict__ parth, int nrows_h,
                                                     int rows_per_group_h, int nhead, int ntail,
                                                     const int *__restrict__ rows_of_block) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int grp = blockIdx.y;
  const int dm = blockIdx.z;
  if (g >= nslot) return;
  int r0 = grp * rows_per_group, r1 = min(nrows, r0 + rows_per_group);
  size_t stride = (size_t)nslot;
  const double2 *pp = part + (size_t)dm * nrows * nslot + g;
  if (slot_pidx) {
    const int pi = slot_pidx[g];
    if (pi < 0) {
      r1 = r0;
    } else if (pi < nhead) {
      r0 = grp * rows_per_group_h;
      r1 = min(nrows_h, r0 + rows_per_group_h);
      pp = parth + (size_t)dm * nrows_h * nhead + pi;
      stride = (size_t)nhead;
    } else {
      const int tp = pi - nhead;
      r1 = min(rows_of_block[tp >> 6], r0 + rows_per_group);
      pp = part + (size_t)dm * nrows * ntail + tp;
      stride = (size_t)ntail;
    }
  }
  double r = 0.0, i = 0.0;
  int row = r0;
  // rows added in order; the loads of eight rows are issued together
  for (; row + 8 <= r1; row += 8) {
    double2 x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = pp[(size_t)(row + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      r += x[u].x;
      i += x[u].y;
    }
  }
  for (; row < r1; ++row) {
    const double2 x = pp[(size_t)row * stride];
    r += x.x;
    i += x.y;
  }
  part2[((size_t)dm * ngroups + grp) * nslot + g] = make_double2(r, i);
}

// Second stage: 4 slots per workgroup, one wave per slot; lane r holds group r
// (ngroups <= 64) and a fixed xor-butterfly adds them.
__global__ __launch_bounds__(256) void k_reduce(const double2 *__restrict__ part2, int ngroups, int nslot,
                                                const double *__restrict__ slot_v, double vol,
                                                double2 *__restrict__ rho, double2 *__restrict__ Vc,
                                                double *__restrict__ Epart) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = blockIdx.x * 4 + wv;
  const int dm = blockIdx.y;
  double r = 0.0, i = 0.0;
  if (g < nslot && lane < ngroups) {
    const double2 x = part2[((size_t)dm * ngroups + lane) * nslot + g];
    r = x.x;
    i = x.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    r += __shfl_xor(r, off, 64);
    i += __shfl_xor(i, off, 64);
  }
  __shared__ double sh[4];
  if (lane == 0) {
    double e = 0.0;
    if (g < nslot) {
      const double v = slot_v[g];
      // padding slots (v = 0) hold no G vector: the FP32-MFMA rho pass never
      // writes them, so whatever their partial rows hold is dropped here
      if (v == 0.0) r = i = 0.0;
      rho[(size_t)dm * nslot + g] = make_double2(r, i);
      Vc[(size_t)dm * nslot + g] = make_double2(v * r, -v * i);
      e = vol * v * (r * r + i * i);
    }
    sh[wv] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) Epart[(size_t)dm * gridDim.x + blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// E_J of density dm from its energy partials, by one 256-thread block in a fixed
// order (sh: 256 doubles of LDS).  Shared by k_energy and the extra block of the
// J(k) launch, so both give the same bits.
__device__ inline void energy_block(const double *__restrict__ Epart, int nparts, double *__restrict__ EJ, int dm,
                                    double *sh) {
  double e = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) e += Epart[(size_t)dm * nparts + i];
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) EJ[dm] = sh[0];
}

__global__ __launch_bounds__(256) void k_energy(const double *__restrict__ Epart, int nparts,
                                                double *__restrict__ EJ) {
  __shared__ double sh[256];
  energy_block(Epart, nparts, EJ, blockIdx.x, sh);
}

// ---------------------------------------------------------------------------
// a5: J moments.  Lane = one pair of class L; the wave walks segments
// [s0, s1) with wave-uniform segment data and conj(V):
//   U(n) = conj V(n) S(n);  m_a = sum_{n_u} n_u^a U  along the segment;
//   yhat_{abc} += n_v^b n_w^c (Re m_a if a+b+c even else Im m_a).
// Padding slots carry V = 0.
// ---------------------------------------------------------------------------
constexpr int kJTile = 32;  // segments per LDS tile of the J pass

// binomial coefficient as a double (small arguments, compile-time after unrolling)
__host__ __device__ constexpr double binom_d(int a, int c) {
  double r = 1.0;
  for (int i = 1; i <= c; ++i) r = r * (a - c + i) / i;
  return r;
}

// J moments of one pair per lane for NDB densities (dm0 .. dm0+NDB-1, those past
// ndm skipped): S is generated once per point and shared by the densities.
template <int L, int SEG, int NDB, bool CUT>
__device__ __forceinline__ void jpass_block(const SegDesc *__restrict__ segs, int nseg, int segs_per_chunk,
                                            const double2 *__restrict__ Vc, int nslot,
                                            const PairHot *__restrict__ hot, int Lp0, int Lp1,
                                            double *__restrict__ yhat, int64_t yhat_size, int64_t ycls_off, int pb,
                                            int chunk, int dm0, int ndm, SegDesc *__restrict__ ss,
                                            double2 *__restrict__ sv, const double *__restrict__ e2,
                                            const double2 *__restrict__ cis, double muu) {
  constexpr int NT = nherm(L);
  constexpr int TS = kJTile;
  constexpr Monos<L> MT{};
  const int np = Lp1 - Lp0;
  const int pl = pb * blockDim.x + threadIdx.x;
  const bool active = pl < np;
  const PairHot h = hot[Lp0 + (active ? pl : 0)];
  const int s0 = chunk * segs_per_chunk;
  const int s1 = min(nseg, s0 + segs_per_chunk);
  double y[NDB][NT];
#pragma unroll
  for (int b = 0; b < NDB; ++b)
#pragma unroll
    for (int k = 0; k < NT; ++k) y[b][k] = 0.0;
  // S, R of the walk; a segment that continues the previous one on the same line
  // (same n_v, n_w, n_u0 = previous n_u0 + SEG) starts from where the recurrence
  // stopped, so only the first segment of each line costs the exponentials and
  // the sincos (the test is wave-uniform: segments come from LDS)
  double Sr = 0.0, Si = 0.0, Rr = 0.0, Ri = 0.0;
  int pnv = INT_MIN, pnw = INT_MIN, pnext = INT_MIN;
  const double q = h.q;
  for (int t0 = s0; t0 < s1; t0 += TS) {
    const int nt = min(TS, s1 - t0);
    __syncthreads();
    // conj V of the tile's slots for each density (zeros past ndm), [b][slot]
    for (int i = threadIdx.x; i < NDB * nt * SEG; i += blockDim.x) {
      const int b = i / (nt * SEG), r = i - b * (nt * SEG);
      sv[b * TS * SEG + r] =
          dm0 + b < ndm ? Vc[(size_t)(dm0 + b) * nslot + (size_t)t0 * SEG + r] : make_double2(0.0, 0.0);
    }
    if ((int)threadIdx.x < nt) ss[threadIdx.x] = segs[t0 + threadIdx.x];
    __syncthreads();
    for (int j = 0; j < nt; ++j) {
      const SegDesc sd = ss[j];
      const double nu0 = sd.nu0, nv = sd.nv, nw = sd.nw;
      // per-pair cuts: a segment outside every lane's cut is skipped (the next
      // segment of its line then restarts the recurrence)
      if (CUT && !__any(h.gc2 >= sd.g2min)) continue;
      if (!(sd.nv == pnv && sd.nw == pnw && sd.nu0 == pnext)) {
        const double e0 = exp_tab(-sd.gq0 * h.inv4p, e2);
        const double eR = exp_tab(-sd.dg0 * h.inv4p, e2);
        double ph = fma(nu0, h.fu, fma(nv, h.fv, nw * h.fw));
        ph -= rint(ph);
        const double2 w = cis_neg(ph, cis);
        Sr = e0 * w.x;
        Si = e0 * w.y;
        Rr = eR * h.cu;
        Ri = eR * h.su;
      }
      pnv = sd.nv;
      pnw = sd.nw;
      pnext = sd.nu0 + SEG;
      double mr[NDB][L + 1], mi[NDB][L + 1];
#pragma unroll
      for (int b = 0; b < NDB; ++b)
#pragma unroll
        for (int a = 0; a <= L; ++a) mr[b][a] = mi[b][a] = 0.0;
      // degrees L <= 3 take the moments in the point offset s (powers known at
      // compile time) and shift them to n_u = nu0 + s once per segment below
      constexpr bool kShift = L <= 3;
      double g2 = sd.gq0, dg = sd.dg0;  // |G|^2 along the segment (per-pair cuts)
#pragma unroll
      for (int s = 0; s < SEG; ++s) {
        const double n = nu0 + s;
        const bool out = CUT && g2 > h.gc2;
        const double sr = out ? 0.0 : Sr, si = out ? 0.0 : Si;
        if constexpr (CUT) {
          g2 += dg;
          dg += 2.0 * muu;
        }
#pragma unroll
        for (int b = 0; b < NDB; ++b) {
          const double2 v = sv[b * TS * SEG + j * SEG + s];
          const double Ur = fma(v.x, sr, -v.y * si);
          const double Ui = fma(v.x, si, v.y * sr);
          if constexpr (kShift) {
            mr[b][0] += Ur;
            mi[b][0] += Ui;
            double sp = 1.0;
#pragma unroll
            for (int a = 1; a <= L; ++a) {
              sp *= (double)s;
              if (s > 0) {
                mr[b][a] = fma(sp, Ur, mr[b][a]);
                mi[b][a] = fma(sp, Ui, mi[b][a]);
              }
            }
          } else {
            double pw = 1.0;
#pragma unroll
            for (int a = 0; a <= L; ++a) {
              mr[b][a] = fma(pw, Ur, mr[b][a]);
              mi[b][a] = fma(pw, Ui, mi[b][a]);
              pw *= n;
            }
          }
        }
        const double tr = fma(Sr, Rr, -Si * Ri);
        Si = fma(Sr, Ri, Si * Rr);
        Sr = tr;
        Rr *= q;
        Ri *= q;
      }
      if constexpr (kShift) {
        // sum_s (nu0 + s)^a U_s = sum_c C(a, c) nu0^(a - c) sum_s s^c U_s, highest a first
        double pn[L + 1];
        pn[0] = 1.0;
#pragma unroll
        for (int a = 1; a <= L; ++a) pn[a] = pn[a - 1] * nu0;
#pragma unroll
        for (int b = 0; b < NDB; ++b)
#pragma unroll
          for (int a = L; a >= 1; --a) {
            double r = mr[b][a], i = mi[b][a];
#pragma unroll
            for (int c = 0; c < a; ++c) {
              const double w = binom_d(a, c) * pn[a - c];
              r = fma(w, mr[b][c], r);
              i = fma(w, mi[b][c], i);
            }
            mr[b][a] = r;
            mi[b][a] = i;
          }
      }
      double mv[L + 1], mw[L + 1];
      mv[0] = mw[0] = 1.0;
#pragma unroll
      for (int c = 1; c <= L; ++c) {
        mv[c] = mv[c - 1] * nv;
        mw[c] = mw[c - 1] * nw;
      }
#pragma unroll
      for (int b = 0; b < NDB; ++b)
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          const int a = MT.u[k], bb = MT.v[k], c = MT.w[k];
          const double m = ((a + bb + c) & 1) ? mi[b][a] : mr[b][a];
          y[b][k] = fma(mv[bb] * mw[c], m, y[b][k]);
        }
    }
  }
  if (!active) return;
#pragma unroll
  for (int b = 0; b < NDB; ++b) {
    if (dm0 + b >= ndm) break;
    double *out = yhat + (size_t)(dm0 + b) * yhat_size + ycls_off + (size_t)chunk * NT * np + pl;
#pragma unroll
    for (int k = 0; k < NT; ++k) out[(size_t)k * np] = y[b][k];
  }
}

// ---------------------------------------------------------------------------
// a6: per block of class (LA, LB): for every primitive pair
//   y_k  = s_|k| sum_chunks yhat_k,  s = (+,+,-,-)[|k| mod 4]   (Re of (-i)^|k| Y_k)
//   J~_t = sum_{|k| = |t|} T[t][k] y_k
//   J_ab += pref_j sum_t E^{ab}_t J~_t
// ---------------------------------------------------------------------------
// classes whose J moments k_ysum sums over the chunks before the back transform
// (FP32-MFMA form): L >= 3 holds every wave-per-pair class
constexpr int kYsumL0 = 3;

template <int LA, int LB>
__device__ __forceinline__ void back_thread(const Dev &dv, int bi, int dm, int jsum) {
  constexpr int L = LA + LB;
  constexpr int NT = nherm(L);
  constexpr Carts<LA> CA{};
  constexpr Carts<LB> CB{};
  constexpr int NCA = ncart(LA), NCB = ncart(LB);
  const PairAux *__restrict__ aux = dv.aux;
  const double *__restrict__ ttab = dv.ttab;
  const double *__restrict__ yhat = dv.yhat;
  double *__restrict__ Jblk = dv.Jblk;
  const int64_t yhat_size = dv.yhat_size, ycls_off = dv.yhat_off[L], nelem = dv.nelem;
  const int nchunks_L = dv.j_chunks[L], Lp0 = dv.L_p0[L], Lp1 = dv.L_p1[L];
  const BlockRec b = dv.blocks[bi];
  const int np = Lp1 - Lp0;
  double J[NCA * NCB];
#pragma unroll
  for (int e = 0; e < NCA * NCB; ++e) J[e] = 0.0;
  for (int q = b.p0; q < b.p1; ++q) {
    const int rq = dv.cut_rank[q];  // J walk order
    const double *ys = yhat + (size_t)dm * yhat_size + ycls_off + (rq - Lp0);
    // FP32-MFMA form: the chunks the pair's block of the J pass wrote (for the
    // classes L >= kYsumL0 summed into chunk 0 by k_ysum when jsum is set)
    int nchunks = dv.jn_of ? dv.jn_of[rq] : nchunks_L;
    if (jsum && L >= kYsumL0) nchunks = min(nchunks, 1);
    // y_k = sum over the J chunks in chunk order; the loads of four chunks are
    // issued together (one thread per pair leaves little other parallelism)
    double y[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) y[k] = 0.0;
    // a DD pair (compact/diffuse classification) takes its moments of V_D from
    // the DD kernel instead of the chunks (which hold zeros for it)
    const int dq = dv.dd_of ? dv.dd_of[q] : -1;
    if (dq >= 0 && !dv.gpw) {  // (GPW route: the DD pairs' J is added to J(L) afterwards)
#pragma unroll
      for (int k = 0; k < NT; ++k) y[k] = dv.ydd[((size_t)dm * dv.ndd + dq) * kDDStride + k];
    }
    // chunks whose loads are issued together: 4 for the small classes, 1 for
    // (3, 0), whose 20 moments per chunk would otherwise hold 160 registers
    constexpr int NB = NT <= 10 ? 4 : 1;
    int c = 0;
    if (dq >= 0) c = nchunks;
    for (; c + NB <= nchunks; c += NB) {
      double v[NB][NT];
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int k = 0; k < NT; ++k) v[u][k] = ys[((size_t)(c + u) * NT + k) * np];
#pragma unroll
      for (int u = 0; u < NB; ++u)
#pragma unroll
        for (int k = 0; k < NT; ++k) y[k] += v[u][k];
    }
    for (; c < nchunks; ++c)
#pragma unroll
      for (int k = 0; k < NT; ++k) y[k] += ys[((size_t)c * NT + k) * np];
    double Jt[NT];
#pragma unroll
    for (int d = 0; d <= L; ++d) {
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
    double Ex[LA + 1][LB + 1][L + 1], Ey[LA + 1][LB + 1][L + 1], Ez[LA + 1][LB + 1][L + 1];
    md_axis<LA, LB>(inv2p, x.xpa[0], x.xpb[0], Ex);
    md_axis<LA, LB>(inv2p, x.xpa[1], x.xpb[1], Ey);
    md_axis<LA, LB>(inv2p, x.xpa[2], x.xpb[2], Ez);
#pragma unroll
    for (int ia = 0; ia < NCA; ++ia)
#pragma unroll
      for (int ib = 0; ib < NCB; ++ib) {
        const int ax = CA.x[ia], ay = CA.y[ia], az = CA.z[ia];
        const int bx = CB.x[ib], by = CB.y[ib], bz = CB.z[ib];
        double s = 0.0;
#pragma unroll
        for (int tx = 0; tx <= ax + bx; ++tx)
#pragma unroll
          for (int ty = 0; ty <= ay + by; ++ty) {
            const double exy = Ex[ax][bx][tx] * Ey[ay][by][ty];
#pragma unroll
            for (int tz = 0; tz <= az + bz; ++tz) {
              const int t = deg_off(tx + ty + tz) + mono_idx(tx, ty, tz);
              s = fma(exy * Ez[az][bz][tz], Jt[t], s);
            }
          }
        J[ia * NCB + ib] = fma(x.pref_j, s, J[ia * NCB + ib]);
      }
  }
  double *out = Jblk + (size_t)dm * nelem + b.eoff;
#pragma unroll
  for (int e = 0; e < NCA * NCB; ++e) out[e] = J[e];
}

// ---------------------------------------------------------------------------
// a2 / a6 for high angular classes: one wave per block.  The thread-per-block
// kernels above keep the three E tables, the Hermite vector and the Cartesian
// block of one pair in registers; for L = la + lb >= 4 that is several hundred
// doubles per lane and the few pairs of such classes end up as one long serial
// chain.  Here lanes 0..2 build the E table of one axis each into LDS and the
// wave then works lane-parallel over Hermite indices t, monomials k or
// Cartesian elements (ia, ib).
// ---------------------------------------------------------------------------
template <int LA, int LB>
struct WaveTabs {
  static constexpr int L = LA + LB;
  static constexpr int NT = nherm(L);
  static constexpr int NCA = ncart(LA), NCB = ncart(LB);
  static constexpr int NE = (LA + 1) * (LB + 1) * (L + 1);  // one axis: E[i][j][t]
  static constexpr int eidx(int i, int j, int t) { return (i * (LB + 1) + j) * (L + 1) + t; }
  // LDS doubles of the wave-per-block transform and back-transform
  static constexpr int kTransformLds = 3 * NE + NCA * NCB + NT + (3 * NCA * NCB + 1) / 2;
  static constexpr int kBackLds = 3 * NE + NT + (L + 1) * (L + 1) * (L + 1);
};

// (tx, ty, tz) of Hermite index t in the degree-ordered list (runtime inverse).
__device__ __forceinline__ void herm_of(int t, int &tx, int &ty, int &tz) {
  int d = 0;
  while (deg_off(d + 1) <= t) ++d;
  int r = t - deg_off(d);
  int a = d;
  while (r > d - a) {
    r -= d - a + 1;
    --a;
  }
  tx = a;
  ty = d - a - r;
  tz = d - tx - ty;
}

// Cartesian component ic of shell l (descending lexicographic), runtime.
__device__ __forceinline__ void cart_of(int l, int ic, int &x, int &y, int &z) {
  int a = l, r = ic;
  while (r > l - a) {
    r -= l - a + 1;
    --a;
  }
  x = a;
  y = l - a - r;
  z = l - x - y;
}

// E table of one axis written column by column into E[i][j][t] (LDS), with the
// recurrence of md_axis: only the column E[0][j] and the current E[i][j] live
// in registers.  Entries t > i + j are written as zeros.
template <int LA, int LB>
__device__ __forceinline__ void md_axis_lds(double inv2p, double xpa, double xpb, double *E) {
  using W = WaveTabs<LA, LB>;
  constexpr int L = LA + LB;
  double c0[L + 1];
#pragma unroll
  for (int t = 0; t <= L; ++t) c0[t] = t == 0 ? 1.0 : 0.0;
#pragma unroll
  for (int j = 0; j <= LB; ++j) {
    if (j > 0) {
      double n[L + 1];
#pragma unroll
      for (int t = 0; t <= L; ++t) {
        double v = 0.0;
        if (t <= j) {
          v = xpb * c0[t];
          if (t > 0) v += inv2p * c0[t - 1];
          if (t + 1 <= j - 1) v += (t + 1) * c0[t + 1];
        }
        n[t] = v;
      }
#pragma unroll
      for (int t = 0; t <= L; ++t) c0[t] = n[t];
    }
    double cur[L + 1];
#pragma unroll
    for (int t = 0; t <= L; ++t) {
      cur[t] = c0[t];
      E[W::eidx(0, j, t)] = cur[t];
    }
#pragma unroll
    for (int i = 1; i <= LA; ++i) {
      double n[L + 1];
#pragma unroll
      for (int t = 0; t <= L; ++t) {
        double v = 0.0;
        if (t <= i + j) {
          v = xpa * cur[t];
          if (t > 0) v += inv2p * cur[t - 1];
          if (t + 1 <= i - 1 + j) v += (t + 1) * cur[t + 1];
        }
        n[t] = v;
      }
#pragma unroll
      for (int t = 0; t <= L; ++t) {
        cur[t] = n[t];
        E[W::eidx(i, j, t)] = cur[t];
      }
    }
  }
}

// Wave bodies run four to a workgroup, each on its own pair and LDS slice, so
// they synchronise their lanes at wavefront scope (LDS writes of the wave
// visible to its lanes, no wait on the other waves of the workgroup).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes 0..2 build the E table of axis x, y, z (read straight from the pair
// record in global memory: a lane-indexed field of a local copy would go
// through scratch).
template <int LA, int LB>
__device__ __forceinline__ void wave_etabs(const PairAux *__restrict__ xq, double *sE) {
  using W = WaveTabs<LA, LB>;
  const int lane = threadIdx.x & 63;
  if (lane < 3) md_axis_lds<LA, LB>(0.5 / xq->p, xq->xpa[lane], xq->xpb[lane], sE + lane * W::NE);
}

template <int LA, int LB>
__device__ __forceinline__ void transform_wave(const Dev &dv, int bi, int dm, double *__restrict__ lds) {
  using W = WaveTabs<LA, LB>;
  constexpr int L = W::L, NT = W::NT, NCA = W::NCA, NCB = W::NCB, NE = W::NE;
  constexpr Carts<LA> CA{};
  constexpr Carts<LB> CB{};
  const PairAux *__restrict__ aux = dv.aux;
  const double *__restrict__ Dblk = dv.Dblk;
  const double *__restrict__ ttab = dv.ttab;
  double *__restrict__ dhat = dv.dhat;
  float *__restrict__ dh32 = dv.dh32;
  const int64_t nelem = dv.nelem, dhat_size = dv.dhat_size, cls_off = dv.dhat_off[L], d32_off = dv.d32_off[L];
  const int Lp0 = dv.L_p0[L], ncols = dv.ncols32[L], ndmp = dv.ndmp;
  double *sE = lds;
  double *sD = sE + 3 * NE;
  double *sH = sD + NCA * NCB;
  int3 *sOff = reinterpret_cast<int3 *>(sH + NT);  // E-table offsets of element (ia, ib) per axis
  const int lane = threadIdx.x & 63;
  const BlockRec b = dv.blocks[bi];
  for (int e = lane; e < NCA * NCB; e += 64) {
    int ax, ay, az, bx, by, bz;
    cart_of(LA, e / NCB, ax, ay, az);
    cart_of(LB, e % NCB, bx, by, bz);
    sOff[e] = make_int3(W::eidx(ax, bx, 0), NE + W::eidx(ay, by, 0), 2 * NE + W::eidx(az, bz, 0));
  }
  for (int e = lane; e < NCA * NCB; e += 64) sD[e] = Dblk[(size_t)dm * nelem + b.eoff + e];
  double *out_base = dhat + (size_t)dm * dhat_size + cls_off;
  for (int q = b.p0; q < b.p1; ++q) {
    const PairAux x = aux[q];
    wave_sync();
    wave_etabs<LA, LB>(aux + q, sE);
    wave_sync();
    for (int t = lane; t < NT; t += 64) {
      int tx, ty, tz;
      herm_of(t, tx, ty, tz);
      double s = 0.0;
      // element (ia, ib) in a runtime loop, four at a time: a fully unrolled loop
      // lets the scheduler hoist every LDS read and the register count explodes
#pragma unroll 4
      for (int e = 0; e < NCA * NCB; ++e) {
        const int3 o = sOff[e];
        s = fma(sD[e] * sE[o.x + tx], sE[o.y + ty] * sE[o.z + tz], s);
      }
      sH[t] = s * x.pref_rho;
    }
    wave_sync();
    double *out = out_base + (size_t)(dv.rho_rank[q] - Lp0) * NT;  // rho's walk order
    for (int k = lane; k < NT; k += 64) {
      int d = 0;
      while (deg_off(d + 1) <= k) ++d;
      const int nc = ncart(d), r = k - deg_off(d);
      const double *T = ttab + tblk_off(d);
      const double sg = ((d & 3) == 1 || (d & 3) == 2) ? -1.0 : 1.0;
      // unrolled to the widest degree of the class (predicated) so that the
      // table loads are issued together instead of one latency after another
      double tv[ncart(L)];
#pragma unroll
      for (int t = 0; t < ncart(L); ++t) tv[t] = t < nc ? T[t * nc + r] : 0.0;
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < ncart(L); ++t)
        if (t < nc) s = fma(tv[t], sH[deg_off(d) + t], s);
      if (dh32) {  // FP32-MFMA form: the MFMA layout (see transform_thread)
        const size_t o = d32_off + (size_t)(dv.cut_rank[q] - Lp0) * ncols + k * ndmp + dm;
        dh32[o] = (float)(sg * s);
        dhat[o] = sg * s;
      } else {
        out[k] = sg * s;
      }
    }
  }
}

template <int LA, int LB>
__device__ __forceinline__ void back_wave(const Dev &dv, int bi, int dm, double *__restrict__ lds, int jsum) {
  using W = WaveTabs<LA, LB>;
  constexpr int L = W::L, NT = W::NT, NCA = W::NCA, NCB = W::NCB, NE = W::NE;
  constexpr int NEL = NCA * NCB;
  constexpr int ROUNDS = (NEL + 63) / 64;
  const PairAux *__restrict__ aux = dv.aux;
  const double *__restrict__ ttab = dv.ttab;
  const double *__restrict__ yhat = dv.yhat;
  double *__restrict__ Jblk = dv.Jblk;
  const int64_t yhat_size = dv.yhat_size, ycls_off = dv.yhat_off[L], nelem = dv.nelem;
  const int nchunks_L = dv.j_chunks[L], Lp0 = dv.L_p0[L], Lp1 = dv.L_p1[L];
  // sJ3: the Hermite-basis J moments at their (tx, ty, tz), so that the
  // contraction reads them by position (one LDS read, no index table)
  double *sE = lds;
  double *sY = sE + 3 * NE;
  double *sJ3 = sY + NT;
  const int lane = threadIdx.x & 63;
  const BlockRec b = dv.blocks[bi];
  const int np = Lp1 - Lp0;
  double acc[ROUNDS];
  int ax[ROUNDS], ay[ROUNDS], az[ROUNDS], bx[ROUNDS], by[ROUNDS], bz[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    acc[r] = 0.0;
    const int e = min(lane + 64 * r, NEL - 1);
    cart_of(LA, e / NCB, ax[r], ay[r], az[r]);
    cart_of(LB, e % NCB, bx[r], by[r], bz[r]);
  }
  for (int q = b.p0; q < b.p1; ++q) {
    const PairAux x = aux[q];
    wave_sync();
    const int rq = dv.cut_rank[q];  // J walk order
    const double *ys = yhat + (size_t)dm * yhat_size + ycls_off + (rq - Lp0);
    // FP32-MFMA form: the chunks the pair's block of the J pass wrote (summed
    // into chunk 0 by k_ysum when jsum is set: every wave-per-pair class has
    // L >= kYsumL0)
    int nchunks = dv.jn_of ? dv.jn_of[rq] : nchunks_L;
    if (jsum && L >= kYsumL0) nchunks = min(nchunks, 1);
    const int dq = dv.dd_of ? dv.dd_of[q] : -1;  // DD pair: the DD kernel's moments
    for (int k = lane; k < NT; k += 64) {
      if (dq >= 0) {
        sY[k] = dv.gpw ? 0.0 : dv.ydd[((size_t)dm * dv.ndd + dq) * kDDStride + k];
        continue;
      }
      // chunk order kept; up to 16 loads in flight
      double s = 0.0;
      for (int c0 = 0; c0 < nchunks; c0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = c0 + u < nchunks ? ys[((size_t)(c0 + u) * NT + k) * np] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (c0 + u < nchunks) s += v[u];
      }
      sY[k] = s;
    }
    wave_etabs<LA, LB>(aux + q, sE);
    wave_sync();
    for (int t = lane; t < NT; t += 64) {
      int d = 0;
      while (deg_off(d + 1) <= t) ++d;
      const int nc = ncart(d), r = t - deg_off(d);
      const double *T = ttab + tblk_off(d);
      const double sg = ((d & 3) >= 2) ? -1.0 : 1.0;
      // table loads issued together (see transform_wave)
      double tv[ncart(L)];
#pragma unroll
      for (int k = 0; k < ncart(L); ++k) tv[k] = k < nc ? T[r * nc + k] : 0.0;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < ncart(L); ++k)
        if (k < nc) s = fma(tv[k], sY[deg_off(d) + k], s);
      int tx, ty, tz;
      herm_of(t, tx, ty, tz);
      sJ3[(tx * (L + 1) + ty) * (L + 1) + tz] = sg * s;
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      if (lane + 64 * r < NEL) {
        double s = 0.0;
        for (int tx = 0; tx <= ax[r] + bx[r]; ++tx) {
          const double ex = sE[W::eidx(ax[r], bx[r], tx)];
          for (int ty = 0; ty <= ay[r] + by[r]; ++ty) {
            const double exy = ex * sE[NE + W::eidx(ay[r], by[r], ty)];
            const double *jz = sJ3 + (tx * (L + 1) + ty) * (L + 1);
            for (int tz = 0; tz <= az[r] + bz[r]; ++tz)
              s = fma(exy * sE[2 * NE + W::eidx(az[r], bz[r], tz)], jz[tz], s);
          }
        }
        acc[r] = fma(x.pref_j, s, acc[r]);
      }
    }
  }
  double *out = Jblk + (size_t)dm * nelem + b.eoff;
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r)
    if (lane + 64 * r < NEL) out[lane + 64 * r] = acc[r];
}

// ---------------------------------------------------------------------------
// a7: J(L) -> J(k).  First the blocks of every matrix element are summed per
// BvK class (k_fold_j, one thread per (element, class) segment, fixed order);
// then J(k)_{mu nu} = sum over the element's classes of e^{2 pi i t/N} J_c
// (k_phase_j, one thread per element, all k).  Mirror entries (b,a,-L) were
// given the class of -m and the transposed element.  Every output is written
// (zeros off the support); for each k the threads of a wave write consecutive
// elements of one row of J(k).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fold_j(const double *__restrict__ Jblk, int64_t nelem, int nsegJ,
                                                const int *__restrict__ sJ_e0, const int *__restrict__ eJ,
                                                double *__restrict__ Jfold) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  const int dm = blockIdx.y;
  if (sg >= nsegJ) return;
  const double *J = Jblk + (size_t)dm * nelem;
  double s = 0.0;
  for (int i = sJ_e0[sg]; i < sJ_e0[sg + 1]; ++i) s += J[eJ[i]];
  Jfold[(size_t)dm * nsegJ + sg] = s;
}

__device__ __forceinline__ void store_jk(double2 *p, double re, double im) { *p = make_double2(re, im); }

// Light elements (at most kPhaseLight classes, zeros included): one thread per
// element, codes and values in registers; for each k the threads of a wave
// write consecutive elements of one row of J(k).  The body is chosen by the
// wave's largest class count (lanes with fewer classes carry zero values), the
// phase offsets advance by one add per class and k, and all NC table reads of a
// k-point are issued before their multiply-adds.
template <int NC>
__device__ __forceinline__ void phase_j_body(const double2 *__restrict__ sph, const int *c1, const int *c2,
                                             const int *c3, const double *v, int n1, int n2, int n3, size_t nn,
                                             double2 *__restrict__ out) {
  size_t ko = 0;
  for (int k1 = 0; k1 < n1; ++k1)
    for (int k2 = 0; k2 < n2; ++k2) {
      int t[NC];
#pragma unroll
      for (int i = 0; i < NC; ++i) t[i] = k1 * c1[i] + k2 * c2[i];
      for (int k3 = 0; k3 < n3; ++k3, ko += nn) {
        double2 w[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) w[i] = sph[t[i]];
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
          re = fma(w[i].x, v[i], re);
          im = fma(w[i].y, v[i], im);
          t[i] += c3[i];
        }
        store_jk(out + ko, re, im);
      }
    }
}

// i0 indexes the light support list lightJ when it is given (support-only J(k):
// only elements with 1 .. kPhaseLight classes are visited), else the elements
// of the whole matrix (zeros written off the support).  J(k) of density dm and
// k-point k starts at Jk + (dm nk + k) kstride; the element goes to offset e (in
// place) or to its list position i0 (packed).
__device__ __forceinline__ void phase_j_light(const double2 *__restrict__ sph, const double *__restrict__ Jfold,
                                              int nsegJ, const int *__restrict__ sJ_off,
                                              const int *__restrict__ sJ_code, int nk, int n1, int n2, int n3,
                                              double2 *__restrict__ Jk, int64_t kstride, bool packed,
                                              const int *__restrict__ lightJ, int64_t nlist, int64_t i0, int dm) {
  // lanes past the end and heavy elements take part with no classes and store nothing
  const bool inb = i0 < nlist;
  const int64_t ii = inb ? i0 : nlist - 1;
  const int64_t e = lightJ ? (int64_t)lightJ[ii] : ii;
  const int s0 = sJ_off[e];
  int n = sJ_off[e + 1] - s0;
  const bool mine = inb && n <= kPhaseLight;
  if (!mine) n = 0;
  const double *Jf = Jfold + (size_t)dm * nsegJ;
  int c1[kPhaseLight], c2[kPhaseLight], c3[kPhaseLight];
  double v[kPhaseLight];
#pragma unroll
  for (int i = 0; i < kPhaseLight; ++i) {
    const int code = i < n ? sJ_code[s0 + i] : 0;
    c1[i] = code & 1023;
    c2[i] = (code >> 10) & 1023;
    c3[i] = code >> 20;
    v[i] = i < n ? Jf[s0 + i] : 0.0;
  }
  int nmax = n;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) nmax = max(nmax, __shfl_xor(nmax, off, 64));
  if (!mine) return;
  double2 *out = Jk + (size_t)dm * nk * kstride + (packed ? ii : e);
  if (nmax == 0) {
    for (int k = 0; k < nk; ++k) store_jk(out + (size_t)k * kstride, 0.0, 0.0);
  } else if (nmax == 1) {
    phase_j_body<1>(sph, c1, c2, c3, v, n1, n2, n3, (size_t)kstride, out);
  } else if (nmax == 2) {
    phase_j_body<2>(sph, c1, c2, c3, v, n1, n2, n3, (size_t)kstride, out);
  } else if (nmax <= 4) {
    phase_j_body<4>(sph, c1, c2, c3, v, n1, n2, n3, (size_t)kstride, out);
  } else {
    phase_j_body<kPhaseLight>(sph, c1, c2, c3, v, n1, n2, n3, (size_t)kstride, out);
  }
}

// Heavy elements: one wave per element, lanes = k-points (64 at a time), the
// element's classes loaded 64 at a time and broadcast lane by lane, four per
// step so that their table reads overlap.
// (packed J(k): heavy element h goes to list position hpos0 + h)
__device__ __forceinline__ void phase_j_heavy(const double2 *__restrict__ sph, const double *__restrict__ Jfold,
                                              int nsegJ, const int *__restrict__ heavy, int nheavy,
                                              const int *__restrict__ sJ_off, const int *__restrict__ sJ_code,
                                              int nk, int n2, int n3, double2 *__restrict__ Jk, int64_t kstride,
                                              bool packed, int64_t hpos0, int h, int dm) {
  const int lane = threadIdx.x & 63;
  if (h >= nheavy) return;
  const int64_t e = heavy[h];
  const int s0 = sJ_off[e], s1 = sJ_off[e + 1];
  const double *Jf = Jfold + (size_t)dm * nsegJ;
  double2 *out = Jk + (size_t)dm * nk * kstride + (packed ? hpos0 + h : e);
  const int n23 = n2 * n3;
  for (int kb = 0; kb < nk; kb += 64) {
    const int k = kb + lane;
    const int kk = k < nk ? k : 0;
    const int k1 = kk / n23, r = kk - k1 * n23;
    const int k2 = r / n3, k3 = r - k2 * n3;
    double re = 0.0, im = 0.0;
    for (int cb = s0; cb < s1; cb += 64) {
      const int nb = min(64, s1 - cb);
      const int mycode = lane < nb ? sJ_code[cb + lane] : 0;
      const double myv = lane < nb ? Jf[cb + lane] : 0.0;
      // lanes past nb hold code 0 and value 0: rounding nb up to 4 adds zeros
      for (int i = 0; i < nb; i += 4) {
        int code[4];
        double x[4];
        double2 w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          code[u] = __shfl(mycode, i + u, 64);
          x[u] = __shfl(myv, i + u, 64);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          w[u] = sph[k1 * (code[u] & 1023) + k2 * ((code[u] >> 10) & 1023) + k3 * (code[u] >> 20)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          re = fma(w[u].x, x[u], re);
          im = fma(w[u].y, x[u], im);
        }
      }
    }
    if (k < nk) store_jk(out + (size_t)k * kstride, re, im);
  }
}

// ---------------------------------------------------------------------------
// Fused launches.  Every pass launches the blocks of all its classes at once: a
// class table maps ranges of blockIdx.x to a class and its per-class body, so
// the classes fill the chip together and a build issues about ten launches.
// ---------------------------------------------------------------------------
struct ClassTab {
  int n;              // entries
  int first[17];      // first flattened block of each entry; first[n] = total
  int cls[16];        // class: la * 4 + lb (transform, back) or L (rho, J)
  int mode[16];       // transform / back: 1 = one wave per block, 0 = one thread per block
  int gx[16];         // rho: segment groups; J: pair blocks (the other index is the chunk)
};

__device__ __forceinline__ int tab_entry(const ClassTab &t, int b) {
  int i = 0;
  while (i + 1 < t.n && b >= t.first[i + 1]) ++i;
  return i;
}

template <int LA, int LB>
constexpr int wave_lds() {
  return WaveTabs<LA, LB>::kBackLds > WaveTabs<LA, LB>::kTransformLds ? WaveTabs<LA, LB>::kBackLds
                                                                       : WaveTabs<LA, LB>::kTransformLds;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kWaveLds = cmax(cmax(cmax(wave_lds<2, 1>(), wave_lds<3, 0>()), cmax(wave_lds<2, 2>(), wave_lds<3, 1>())),
                              cmax(wave_lds<3, 2>(), wave_lds<3, 3>()));

// Wave-per-block bodies for the classes with L = la + lb >= 3: their per-lane
// tables (E coefficients, Hermite and Cartesian vectors) would hold hundreds of
// registers in a thread-per-block body.  (3, 0) -- one f shell with one s shell,
// 20 Hermite terms and 10 elements -- runs a thread per block instead, where a
// wave per block would leave most lanes idle: inside the fused transform launch
// (108 VGPRs), and in a launch of its own after the fused back transform (its
// body inside the fused launch would take that launch to 255 VGPRs, one wave per
// SIMD for every class).
static bool wave_per_block(int la, int lb) { return la + lb >= 3 && !(la == 3 && lb == 0); }

#define PWDF_CLASS_SWITCH_THREAD(F, ...)      \
  switch (cl) {                               \
    case 0: F<0, 0>(__VA_ARGS__); break;      \
    case 4: F<1, 0>(__VA_ARGS__); break;      \
    case 5: F<1, 1>(__VA_ARGS__); break;      \
    case 8: F<2, 0>(__VA_ARGS__); break;      \
    case 12:                                  \
      if constexpr (kThread30) F<3, 0>(__VA_ARGS__); \
      break;                                  \
    default: break;                           \
  }
#define PWDF_CLASS_SWITCH_WAVE(F, ...)        \
  switch (cl) {                               \
    case 9: F<2, 1>(__VA_ARGS__); break;      \
    case 10: F<2, 2>(__VA_ARGS__); break;     \
    case 13: F<3, 1>(__VA_ARGS__); break;     \
    case 14: F<3, 2>(__VA_ARGS__); break;     \
    case 15: F<3, 3>(__VA_ARGS__); break;     \
    default: break;                           \
  }

// Workgroups of 256 threads (many single-wave workgroups launch more slowly than
// they run): thread mode takes 256 pair blocks per workgroup, wave mode four,
// one per wave, each wave with its own LDS slice.
constexpr int kPairWG = 256;
constexpr int kWavesPerWG = kPairWG / 64;

// The transform takes the blocks in storage order (neighbouring lanes read
// neighbouring D(L) blocks); the back transform takes them in the J walk order
// (blk_cut), in which it reads the moments.
//
// fold (FP32-MFMA form): the densities of the call are folded into the x
// dimension instead of y, so that the ndmp consecutive operand columns of one
// (pair, k) -- [pair][k * ndmp + dm] -- are written by neighbouring lanes (thread
// mode: lane = (block, density), density fastest) or by consecutive workgroups
// (wave mode: workgroup = (group of four blocks, density), density fastest)
// rather than by workgroups far apart in the dispatch order, each filling a few
// bytes of every line.
template <bool FOLD>
__global__ __launch_bounds__(kPairWG) void k_transform_all(const Dev dv, const ClassTab tab, int ndm) {
  constexpr bool kThread30 = true;  // (3, 0): a thread per block
  __shared__ double lds[kWavesPerWG * kWaveLds];
  const int i = tab_entry(tab, blockIdx.x);
  int local = blockIdx.x - tab.first[i];
  const int cl = tab.cls[i];
  int dm = blockIdx.y;
  if (tab.mode[i]) {
    if (FOLD) {
      dm = local % ndm;
      local /= ndm;
    }
    const int w = threadIdx.x >> 6;
    const int bi = dv.cls_b0[cl] + local * kWavesPerWG + w;
    if (bi >= dv.cls_b1[cl]) return;
    PWDF_CLASS_SWITCH_WAVE(transform_wave, dv, bi, dm, lds + w * kWaveLds)
  } else {
    int bi;
    if (FOLD) {
      const int dpt = dv.ndmp;  // a power of two <= 16
      dm = threadIdx.x & (dpt - 1);
      bi = dv.cls_b0[cl] + local * (kPairWG / dpt) + threadIdx.x / dpt;
      if (dm >= ndm) return;
    } else {
      bi = dv.cls_b0[cl] + local * kPairWG + threadIdx.x;
    }
    if (bi >= dv.cls_b1[cl]) return;
    PWDF_CLASS_SWITCH_THREAD(transform_thread, dv, bi, dm)
  }
}

// FP32-MFMA form, before the back transform: the J moments of the pairs of the
// classes L >= kYsumL0 summed over the chunks their block of the J pass wrote,
// in chunk order, into chunk 0.  One thread per (class, moment k, pair):
// neighbouring lanes read neighbouring pairs of a chunk, where the wave-per-pair
// back transform of those classes would read each moment of each chunk from a
// line of its own.  The sums are the ones the back transform formed itself,
// term for term.
struct YsumTab {
  int64_t start[kMaxLsum + 2];  // first thread of class L (0 below kYsumL0); start[kMaxLsum + 1] = total
};

__global__ __launch_bounds__(256) void k_ysum(const Dev dv, const YsumTab t) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= t.start[kMaxLsum + 1]) return;
  const int dm = blockIdx.y;
  int L = kYsumL0;
  while (i >= t.start[L + 1]) ++L;
  const int np = dv.L_p1[L] - dv.L_p0[L], NT = nherm(L);
  const int64_t j = i - t.start[L];
  const int k = (int)(j / np), r = (int)(j - (int64_t)k * np);
  const int n = dv.jn_of[dv.L_p0[L] + r];
  if (n <= 0) return;  // no chunk: the back transform reads none either
  double *ys = dv.yhat + (size_t)dm * dv.yhat_size + dv.yhat_off[L] + (size_t)k * np + r;
  const size_t cs = (size_t)NT * np;
  double s = 0.0;
  for (int c0 = 0; c0 < n; c0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = c0 + u < n ? ys[(size_t)(c0 + u) * cs] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c0 + u < n) s += v[u];
  }
  ys[0] = s;
}

__global__ __launch_bounds__(kPairWG) void k_back_all(const Dev dv, const ClassTab tab, int jsum) {
  constexpr bool kThread30 = false;  // (3, 0): k_back_30
  __shared__ double lds[kWavesPerWG * kWaveLds];
  const int i = tab_entry(tab, blockIdx.x);
  const int local = blockIdx.x - tab.first[i];
  const int cl = tab.cls[i];
  const int dm = blockIdx.y;
  if (tab.mode[i]) {
    const int w = threadIdx.x >> 6;
    const int j = dv.cls_b0[cl] + local * kWavesPerWG + w;
    if (j >= dv.cls_b1[cl]) return;
    PWDF_CLASS_SWITCH_WAVE(back_wave, dv, dv.blk_cut[j], dm, lds + w * kWaveLds, jsum)
  } else {
    const int j = dv.cls_b0[cl] + local * kPairWG + threadIdx.x;
    if (j >= dv.cls_b1[cl]) return;
    PWDF_CLASS_SWITCH_THREAD(back_thread, dv, dv.blk_cut[j], dm, jsum)
  }
}

// The back transform of the class (3, 0), a thread per block in the J walk order.
__global__ __launch_bounds__(kPairWG) void k_back_30(const Dev dv, int jsum) {
  const int j = dv.cls_b0[12] + blockIdx.x * kPairWG + threadIdx.x;
  if (j >= dv.cls_b1[12]) return;
  back_thread<3, 0>(dv, dv.blk_cut[j], blockIdx.y, jsum);
}

template <int L, int NDB>
constexpr int rho_sp_doubles() {
  return RhoTile<L>::TP * (8 + nherm(L) * NDB);
}
// LDS of the fused rho launch: pair records of the largest class of the group
template <int L0, int L1, int NDB>
constexpr int rho_sp_max() {
  return L0 > L1 ? 0 : cmax(rho_sp_doubles<L0, NDB>(), rho_sp_max<(L0 < L1 ? L0 + 1 : L1 + 1), L1, NDB>());
}

// rho of the classes L in [L0, L1] for NDB densities per block (blockIdx.y is the
// density block).  Low and high groups as for the J pass: the Horner
// coefficients and monomials of class L set the register footprint.
template <int SEG, int L0, int L1, int NDB, bool CUT>
__global__ __launch_bounds__(256) void k_rho_all(const Dev dv, const ClassTab tab, int ndm) {
  constexpr int W = 4;
  __shared__ double sp[rho_sp_max<L0, L1, NDB>()];
  __shared__ double2 red[(W - 1) * 64 * SEG];
  __shared__ double se2[32];
  __shared__ double2 scis[65];
  load_start_tabs(dv.start_tab, se2, scis);
  __syncthreads();
  const int i = tab_entry(tab, blockIdx.x);
  const int local = blockIdx.x - tab.first[i];
  const int nsg = tab.gx[i];
  const int sgi = local % nsg, chunk = local / nsg;
  const int db = blockIdx.y;
#define PWDF_RCASE(LL)                                                                                      \
  case LL:                                                                                                  \
    if (LL >= L0 && LL <= L1)                                                                               \
      rho_block<(LL >= L0 && LL <= L1 ? LL : L0), SEG, W, NDB, CUT>(dv, sgi, chunk, db, ndm, sp, red, se2, scis); \
    break;
  switch (tab.cls[i]) {
    PWDF_RCASE(0)
    PWDF_RCASE(1)
    PWDF_RCASE(2)
    PWDF_RCASE(3)
    PWDF_RCASE(4)
    PWDF_RCASE(5)
    PWDF_RCASE(6)
    default: break;
  }
#undef PWDF_RCASE
}

// J moments of the classes L in [L0, L1] (degree L + DEG: DEG = 1 gives the force
// moments of the class-L pairs), NDB densities per block (blockIdx.y).  Classes
// are split into a low and a high group because the moment count NT(L) sets the
// register footprint of the launch.
template <int SEG, int DEG, int L0, int L1, int NDB, bool CUT>
__global__ __launch_bounds__(256) void k_jpass_all(const Dev dv, const ClassTab tab, int ndm) {
  __shared__ SegDesc ss[kJTile];
  __shared__ double2 sv[NDB * kJTile * SEG];
  __shared__ double se2[32];
  __shared__ double2 scis[65];
  load_start_tabs(dv.start_tab, se2, scis);
  __syncthreads();
  const int i = tab_entry(tab, blockIdx.x);
  const int local = blockIdx.x - tab.first[i];
  const int npb = tab.gx[i];
  const int pb = local % npb, chunk = local / npb;
  const int dm0 = blockIdx.y * NDB;
  const int L = tab.cls[i];
  double *y = DEG ? dv.yF : dv.yhat;
  const int64_t ysz = DEG ? dv.yF_size : dv.yhat_size;
  const int64_t yoff = DEG ? dv.yF_off[L] : dv.yhat_off[L];
#define PWDF_JCASE(LL)                                                                                         \
  case LL:                                                                                                     \
    if (LL >= L0 && LL <= L1)                                                                                  \
      jpass_block<(LL >= L0 && LL <= L1 ? LL + DEG : 0), SEG, NDB, CUT>(                                      \
          dv.segs, dv.nseg, dv.j_spc[LL], dv.Vc, dv.nslot, dv.hot_cut, dv.L_p0[LL], dv.L_p1[LL], y, ysz, yoff, pb, \
          chunk, dm0, ndm, ss, sv, se2, scis, dv.muu);                                                             \
    break;
  switch (L) {
    PWDF_JCASE(0)
    PWDF_JCASE(1)
    PWDF_JCASE(2)
    PWDF_JCASE(3)
    PWDF_JCASE(4)
    PWDF_JCASE(5)
    PWDF_JCASE(6)
    default: break;
  }
#undef PWDF_JCASE
}

// J(L) -> J(k): blocks [0, nlight) take 256 elements each (light path), the next
// ones four heavy elements each (one wave per element).  With EJ non-null one more
// block of each density, dispatched first so that it overlaps the others, sums
// its energy partials into EJ (saves the separate k_energy launch on the J build
// path) and the element blocks follow it.
__global__ __launch_bounds__(256) void k_phase_j_all(const double *__restrict__ Jfold, int nsegJ,
                                                     const int *__restrict__ sJ_off, const int *__restrict__ sJ_code,
                                                     const int *__restrict__ heavy, int nheavy,
                                                     const int *__restrict__ lightJ, int64_t nlist, int nlight,
                                                     const double2 *__restrict__ ptab, int ptab_len, int nk, int n1,
                                                     int n2, int n3, double2 *__restrict__ Jk, int64_t kstride,
                                                     int packed,
                                                     const double *__restrict__ Epart, int nparts,
                                                     double *__restrict__ EJ) {
  __shared__ double2 sph[kPtabMax];
  static_assert(kPtabMax * 2 >= 256, "the energy block reuses the phase table's LDS");
  if (EJ != nullptr && blockIdx.x == 0) {
    energy_block(Epart, nparts, EJ, blockIdx.y, reinterpret_cast<double *>(sph));
    return;
  }
  const int bx = (int)blockIdx.x - (EJ != nullptr ? 1 : 0);
  for (int i = threadIdx.x; i < ptab_len; i += blockDim.x) sph[i] = ptab[i];
  __syncthreads();
  const int dm = blockIdx.y;
  if (bx < nlight)
    phase_j_light(sph, Jfold, nsegJ, sJ_off, sJ_code, nk, n1, n2, n3, Jk, kstride, packed != 0, lightJ, nlist,
                  (int64_t)bx * blockDim.x + threadIdx.x, dm);
  else
    phase_j_heavy(sph, Jfold, nsegJ, heavy, nheavy, sJ_off, sJ_code, nk, n2, n3, Jk, kstride, packed != 0, nlist,
                  (bx - nlight) * 4 + (threadIdx.x >> 6), dm);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
#define PWDF_CHECK_LAUNCH()                          \
  do {                                               \
    hipError_t e_ = hipGetLastError();               \
    if (e_ != hipSuccess) return e_;                 \
  } while (0)

hipError_t launch_phase_d(const Dev &d, const double *Dk, int ndm, hipStream_t st) {
  const bool packed = d.dk_layout == 1;
  const int nseg = packed ? d.nsegDp : d.nsegD;
  if (nseg <= 0) return hipSuccess;
  if (d.ptab_len > kPtabMax) return hipErrorInvalidValue;
  // a plane of D(k): the dense matrix, or the J(k) support in its packed order
  const int64_t nn = packed ? (int64_t)d.nlightJ + d.nheavyJ : (int64_t)d.nbf * d.nbf;
  dim3 grid((unsigned)((nseg + 255) / 256), ndm);
  hipLaunchKernelGGL(k_phase_d, grid, dim3(256), 0, st, (const double2 *)Dk, d.nk, nn, d.kmesh[1], d.kmesh[2], nseg,
                     packed ? d.sDp_el : d.sD_el, packed ? d.sDp_code : d.sD_code, packed ? d.sDp_e0 : d.sD_e0,
                     packed ? d.eDp : d.eD, d.ptab, d.ptab_len, 1.0 / d.nk, d.Dblk, d.nelem, d.nonfinite);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

static void add_entry(ClassTab &t, int cls, int mode, int gx, int nblocks) {
  if (t.n == 0) t.first[0] = 0;
  t.cls[t.n] = cls;
  t.mode[t.n] = mode;
  t.gx[t.n] = gx;
  t.first[t.n + 1] = t.first[t.n] + nblocks;
  ++t.n;
}

// transform / back: one entry per non-empty class (la, lb); the wave-mode classes
// first, so that their long per-pair chains start early and overlap the
// thread-mode blocks instead of forming the launch's tail
// fold: the transform of the FP32-MFMA form (densities in x, see k_transform_all):
// thread-mode entries take kPairWG / ndmp blocks per workgroup, wave-mode entries
// ndm workgroups per group of four blocks
static ClassTab pair_class_tab(const Dev &d, bool back, bool fold = false, int ndm = 1) {
  // the back transform's (3, 0) blocks go to k_back_30
  ClassTab t{};
  for (int wave = 1; wave >= 0; --wave)
    for (int la = 0; la <= kMaxL; ++la)
      for (int lb = 0; lb <= la; ++lb) {
        const int cl = la * 4 + lb, nb = d.cls_b1[cl] - d.cls_b0[cl];
        if (nb <= 0 || (wave_per_block(la, lb) ? 1 : 0) != wave || (back && cl == 12)) continue;
        const int bpw = fold ? kPairWG / d.ndmp : kPairWG;
        add_entry(t, cl, wave, 0,
                  wave ? (nb + kWavesPerWG - 1) / kWavesPerWG * (fold ? ndm : 1) : (nb + bpw - 1) / bpw);
      }
  return t;
}

hipError_t launch_transform_all(const Dev &d, int ndm, hipStream_t st) {
  const bool fold = d.dh32 != nullptr;
  if (fold && (d.ndmp < 1 || d.ndmp > 16 || (d.ndmp & (d.ndmp - 1)) != 0 || ndm > d.ndmp))
    return hipErrorInvalidValue;
  const ClassTab t = pair_class_tab(d, false, fold, ndm);
  if (t.n == 0) return hipSuccess;
  if (fold)
    hipLaunchKernelGGL(k_transform_all<true>, dim3((unsigned)t.first[t.n], 1), dim3(kPairWG), 0, st, d, t, ndm);
  else
    hipLaunchKernelGGL(k_transform_all<false>, dim3((unsigned)t.first[t.n], ndm), dim3(kPairWG), 0, st, d, t, ndm);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_back_all(const Dev &d, int ndm, hipStream_t st) {
  // FP32-MFMA form: the chunk sums of the classes L >= kYsumL0 first
  const int jsum = d.jn_of != nullptr ? 1 : 0;
  if (jsum) {
    YsumTab y{};
    int64_t n = 0;
    for (int L = 0; L <= kMaxLsum; ++L) {
      y.start[L] = n;
      if (L >= kYsumL0) n += (int64_t)nherm(L) * (d.L_p1[L] - d.L_p0[L]);
    }
    y.start[kMaxLsum + 1] = n;
    if (n > 0) {
      hipLaunchKernelGGL(k_ysum, dim3((unsigned)((n + 255) / 256), ndm), dim3(256), 0, st, d, y);
      PWDF_CHECK_LAUNCH();
    }
  }
  const ClassTab t = pair_class_tab(d, true);
  if (t.n > 0) {
    hipLaunchKernelGGL(k_back_all, dim3((unsigned)t.first[t.n], ndm), dim3(kPairWG), 0, st, d, t, jsum);
    PWDF_CHECK_LAUNCH();
  }
  const int n30 = d.cls_b1[12] - d.cls_b0[12];
  if (n30 > 0) {
    hipLaunchKernelGGL(k_back_30, dim3((unsigned)((n30 + kPairWG - 1) / kPairWG), ndm), dim3(kPairWG), 0, st, d,
                       jsum);
    PWDF_CHECK_LAUNCH();
  }
  return hipSuccess;
}

// Class groups of the pair-G passes: [0, kJSplit] and [kJSplit + 1, 6].
constexpr int kJSplit = 2;

// Densities per block of the low class group (S shared by them): d.ndb, at most
// 32 / SEG so that the per-density accumulators stay within the register file.
// The high group takes one density per block.
static int group_ndb(const Dev &d, int group) {
  if (group != 0) return 1;
  return std::min(d.ndb, 32 / d.seg_len);
}

template <int SEG, int NDB, bool CUT>
static hipError_t rho_launch_cut(const Dev &d, const ClassTab &t, int ndm, hipStream_t st, int group) {
  dim3 grid((unsigned)t.first[t.n], (unsigned)((ndm + NDB - 1) / NDB)), block(64, 4);
  if (group == 0)
    hipLaunchKernelGGL((k_rho_all<SEG, 0, kJSplit, NDB, CUT>), grid, block, 0, st, d, t, ndm);
  else
    hipLaunchKernelGGL((k_rho_all<SEG, kJSplit + 1, 2 * kMaxL, 1, CUT>), grid, block, 0, st, d, t, ndm);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

template <int SEG, int NDB>
static hipError_t rho_launch(const Dev &d, const ClassTab &t, int ndm, hipStream_t st, int group) {
  return d.pair_gcut ? rho_launch_cut<SEG, NDB, true>(d, t, ndm, st, group)
                     : rho_launch_cut<SEG, NDB, false>(d, t, ndm, st, group);
}

template <int SEG>
static hipError_t rho_group(const Dev &d, int ndm, hipStream_t st, int group) {
  ClassTab t{};
  const int nsg = (d.nseg + 63) / 64;
  const int La = group == 0 ? 0 : kJSplit + 1, Lb = group == 0 ? kJSplit : 2 * kMaxL;
  for (int L = La; L <= Lb; ++L)
    if (d.L_p1[L] > d.L_p0[L]) add_entry(t, L, 0, nsg, nsg * d.rho_chunks[L]);
  if (t.n == 0) return hipSuccess;
  switch (group_ndb(d, group)) {
    case 1: return rho_launch<SEG, 1>(d, t, ndm, st, group);
    case 2: return rho_launch<SEG, 2>(d, t, ndm, st, group);
    case 4:
      if constexpr (SEG <= 8) return rho_launch<SEG, 4>(d, t, ndm, st, group);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rho_group(const Dev &d, int group, int ndm, hipStream_t st) {
  switch (d.seg_len) {
    case 4: return rho_group<4>(d, ndm, st, group);
    case 5: return rho_group<5>(d, ndm, st, group);
    case 8: return rho_group<8>(d, ndm, st, group);
    case 16: return rho_group<16>(d, ndm, st, group);
    default: return hipErrorInvalidValue;
  }
}

template <int SEG, int DEG, int NDB, bool CUT>
static hipError_t jpass_launch_cut(const Dev &d, const ClassTab &t, int ndm, hipStream_t st, int group) {
  dim3 grid((unsigned)t.first[t.n], (unsigned)((ndm + NDB - 1) / NDB));
  if (group == 0)
    hipLaunchKernelGGL((k_jpass_all<SEG, DEG, 0, kJSplit, NDB, CUT>), grid, dim3(256), 0, st, d, t, ndm);
  else
    hipLaunchKernelGGL((k_jpass_all<SEG, DEG, kJSplit + 1, 2 * kMaxL, 1, CUT>), grid, dim3(256), 0, st, d, t, ndm);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

template <int SEG, int DEG, int NDB>
static hipError_t jpass_launch(const Dev &d, const ClassTab &t, int ndm, hipStream_t st, int group) {
  return d.pair_gcut ? jpass_launch_cut<SEG, DEG, NDB, true>(d, t, ndm, st, group)
                     : jpass_launch_cut<SEG, DEG, NDB, false>(d, t, ndm, st, group);
}

template <int SEG, int DEG>
static hipError_t jpass_groups(const Dev &d, int ndm, hipStream_t st, int group) {
  ClassTab t{};
  const int La = group == 0 ? 0 : kJSplit + 1, Lb = group == 0 ? kJSplit : 2 * kMaxL;
  for (int L = La; L <= Lb; ++L) {
    const int np = d.L_p1[L] - d.L_p0[L];
    if (np <= 0) continue;
    const int npb = (np + 255) / 256;
    add_entry(t, L, 0, npb, npb * d.j_chunks[L]);
  }
  if (t.n == 0) return hipSuccess;
  switch (group_ndb(d, group)) {
    case 1: return jpass_launch<SEG, DEG, 1>(d, t, ndm, st, group);
    case 2: return jpass_launch<SEG, DEG, 2>(d, t, ndm, st, group);
    case 4:
      if constexpr (SEG <= 8) return jpass_launch<SEG, DEG, 4>(d, t, ndm, st, group);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_jpass_group(const Dev &d, int group, bool force, int ndm, hipStream_t st) {
  switch (d.seg_len * 2 + (force ? 1 : 0)) {
    case 8: return jpass_groups<4, 0>(d, ndm, st, group);
    case 9: return jpass_groups<4, 1>(d, ndm, st, group);
    case 10: return jpass_groups<5, 0>(d, ndm, st, group);
    case 11: return jpass_groups<5, 1>(d, ndm, st, group);
    case 16: return jpass_groups<8, 0>(d, ndm, st, group);
    case 17: return jpass_groups<8, 1>(d, ndm, st, group);
    case 32: return jpass_groups<16, 0>(d, ndm, st, group);
    case 33: return jpass_groups<16, 1>(d, ndm, st, group);
    default: return hipErrorInvalidValue;
  }
}

bool jpass_group_nonempty(const Dev &d, int group) {
  const int La = group == 0 ? 0 : kJSplit + 1, Lb = group == 0 ? kJSplit : 2 * kMaxL;
  for (int L = La; L <= Lb; ++L)
    if (d.L_p1[L] > d.L_p0[L]) return true;
  return false;
}

hipError_t launch_fold_j(const Dev &d, int ndm, hipStream_t st) {
  if (d.nsegJ > 0) {
    dim3 g1((unsigned)((d.nsegJ + 255) / 256), ndm);
    hipLaunchKernelGGL(k_fold_j, g1, dim3(256), 0, st, d.Jblk, d.nelem, d.nsegJ, d.sJ_e0, d.eJ, d.Jfold);
    PWDF_CHECK_LAUNCH();
  }
  return hipSuccess;
}

hipError_t launch_phase_j(const Dev &d, int ndm, double *Jk, double *EJ, hipStream_t st) {
  if (d.ptab_len > kPtabMax) return hipErrorInvalidValue;
  // light path: the support list (support-only or packed J(k)) or every element
  // (zeros off the support); k-planes of nbf^2 elements, or of the support list
  // (light elements, then heavy ones) when packed
  const bool list = d.jk_layout != 0, packed = d.jk_layout == 2;
  const int64_t nn = (int64_t)d.nbf * d.nbf;
  const int64_t nlist = list ? (int64_t)d.nlightJ : nn;
  const int64_t kstride = packed ? (int64_t)d.nlightJ + d.nheavyJ : nn;
  const int nlight = (int)((nlist + 255) / 256);
  const int nheavy_blocks = (d.nheavyJ + 3) / 4;
  if (nlight + nheavy_blocks + (EJ ? 1 : 0) == 0) return hipSuccess;
  dim3 grid((unsigned)(nlight + nheavy_blocks + (EJ ? 1 : 0)), ndm);
  hipLaunchKernelGGL(k_phase_j_all, grid, dim3(256), 0, st, d.Jfold, d.nsegJ, d.sJ_off, d.sJ_code, d.heavyJ,
                     d.nheavyJ, list ? d.lightJ : nullptr, nlist, nlight, d.ptab, d.ptab_len, d.nk, d.kmesh[0],
                     d.kmesh[1], d.kmesh[2], (double2 *)Jk, kstride, packed ? 1 : 0, d.Epart, d.nred_blocks, EJ);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_reduce(const Dev &d, int ndm, double *EJ, hipStream_t st) {
  dim3 g1((unsigned)((d.nslot + 255) / 256), d.ngroups, ndm);
  hipLaunchKernelGGL(k_reduce_rows, g1, dim3(256), 0, st, d.part, d.nrows, d.nslot, d.rows_per_group, d.part2,
                     d.ngroups, d.fp32 ? d.slot_pidx : nullptr, d.parth, d.nrows_h, d.rows_per_group_h, d.npts_head,
                     d.npts - d.npts_head, d.rows_of_block);
  PWDF_CHECK_LAUNCH();
  dim3 g2((unsigned)d.nred_blocks, ndm);
  hipLaunchKernelGGL(k_reduce, g2, dim3(256), 0, st, d.part2, d.ngroups, d.nslot, d.slot_v, d.vol, d.rho, d.Vc,
                     d.Epart);
  PWDF_CHECK_LAUNCH();
  if (EJ == nullptr) return hipSuccess;  // summed by the J(k) launch
  return launch_energy(d, ndm, EJ, st);
}

hipError_t launch_energy(const Dev &d, int ndm, double *EJ, hipStream_t st) {
  hipLaunchKernelGGL(k_energy, dim3(ndm), dim3(256), 0, st, d.Epart, d.nred_blocks, EJ);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// E_J in real space, (1/2) sum over (a, b, L) of D_ab(L) J_ab(L), from the D(L)
// and J(L) blocks of a build: a block with its mirror (b, a, -L) folded in counts
// twice (D and J are real and the mirror's values equal the block's).  A wave per
// block at a time (blocks strided over the kERBlocks x 4 waves), partials per workgroup in
// a fixed order, then one fixed-order sum per density.
// ---------------------------------------------------------------------------
constexpr int kERBlocks = 256;

__global__ __launch_bounds__(256) void k_energy_real_part(const Dev d, double *__restrict__ part) {
  __shared__ double sh[256];
  const int dm = blockIdx.y, lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + (threadIdx.x >> 6), nw = kERBlocks * 4;
  const double *D = d.Dblk + (size_t)dm * d.nelem, *J = d.Jblk + (size_t)dm * d.nelem;
  double acc = 0.0;
  for (int b = gw; b < d.nblocks; b += nw) {
    const BlockRec r = d.blocks[b];
    const int n = ncart(d.sh_l[r.sa]) * ncart(d.sh_l[r.sb]);
    double s = 0.0;
    for (int e = lane; e < n; e += 64) s = fma(D[r.eoff + e], J[r.eoff + e], s);
    acc += r.w2 ? 2.0 * s : s;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)dm * kERBlocks + blockIdx.x] = 0.5 * sh[0];
}

__global__ __launch_bounds__(256) void k_energy_real_sum(const double *__restrict__ part, double *__restrict__ ER) {
  __shared__ double sh[256];
  energy_block(part, kERBlocks, ER, blockIdx.x, sh);
}

__global__ __launch_bounds__(256) void k_gather_rho(const double2 *__restrict__ rho, int nslot,
                                                    const int *__restrict__ slots, int nvalid,
                                                    double2 *__restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x, dm = blockIdx.y;
  if (i < nvalid) out[(size_t)dm * nvalid + i] = rho[(size_t)dm * nslot + slots[i]];
}

hipError_t launch_gather_rho(const Dev &d, int ndm, double2 *out, hipStream_t st) {
  if (d.nvalid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rho, dim3((unsigned)((d.nvalid + 255) / 256), ndm), dim3(256), 0, st, d.rho, d.nslot,
                     d.valid_slots, d.nvalid, out);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

hipError_t launch_energy_real(const Dev &d, int ndm, double *part, double *ER, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_real_part, dim3(kERBlocks, ndm), dim3(256), 0, st, d, part);
  PWDF_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_energy_real_sum, dim3(ndm), dim3(256), 0, st, part, ER);
  PWDF_CHECK_LAUNCH();
  return hipSuccess;
}

}  // namespace pwdf
