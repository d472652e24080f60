// Internal records shared by the host plan and the gfx950 kernels of libpwdf.
//
// Reciprocal space is walked in "lines": fixed relative coordinates (n_v, n_w)
// and a run of consecutive n_u.  Along a line the pair factor
//   S(n) = exp(-|G(n)|^2 / 4p) exp(-2 pi i n.f_P)
// obeys S(n_u + 1) = S(n_u) R(n_u), R(n_u + 1) = q R(n_u) with
//   q = exp(-M_uu / 2p),  M = B^T B the reciprocal metric,
// so a whole segment of a line costs two exponentials and one sincos per pair
// instead of one each per G: the shift-term recurrence of the paper's
// non-separable exponential (eq. "non-separable exponential term").
#pragma once
#include <stdint.h>

namespace pwdf {

constexpr int kMaxL = 3;            // largest shell angular momentum
constexpr int kMaxLsum = 2 * kMaxL + 1;  // class L = la+lb (+1 for force derivatives)

__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
// Hermite / relative-monomial count of total degree <= L.
__host__ __device__ constexpr int nherm(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
// offset of degree d inside a degree-ordered list
__host__ __device__ constexpr int deg_off(int d) { return d * (d + 1) * (d + 2) / 6; }
// offset of the degree-d block inside the block-diagonal transform table
__host__ __device__ constexpr int tblk_off(int d) {
  int o = 0;
  for (int e = 0; e < d; ++e) o += ncart(e) * ncart(e);
  return o;
}
constexpr int kTTableSize = tblk_off(kMaxLsum + 1);

// Phase sums: matrix elements with at most kPhaseLight Born-von Karman classes
// are summed by one thread with the classes in registers; heavier elements by
// one wave.  The phase table e^{2 pi i t/N} lives in LDS (at most kPtabMax).
constexpr int kPhaseLight = 8;
constexpr int kPtabMax = 1024;

// One segment of a G line: cnt <= SEG valid points n_u = nu0 .. nu0+cnt-1.
struct SegDesc {
  int nu0, nv, nw, cnt;
  double gq0;  // |G|^2 at n_u = nu0
  double dg0;  // |G(nu0+1)|^2 - |G(nu0)|^2
  double g2min;  // smallest |G|^2 of the segment's points
  double pad;
};

// One G vector of the half space the kernels walk, for the FP32-MFMA form, which
// evaluates the pair factor at every point directly instead of along lines:
// |G|^2, the relative coordinates (u, v, w) and the slot of the point in the
// segment layout (where rho and V live).
struct GPoint {
  double g2;
  int nu, nv, nw;
  int slot;
};

// Per primitive pair, read by the pair-G kernels (64 bytes).
struct PairHot {
  double inv4p;      // 1/(4p)
  double fu, fv, fw; // fractional coordinates of P in the (u,v,w) axis order, in [-1/2,1/2)
  double cu, su;     // cos(2 pi f_u), -sin(2 pi f_u): the per-step phase e^{-2 pi i f_u}
  double q;          // exp(-M_uu / 2p)
  double gc2;        // squared cut radius: the pair sees the G of the set with |G|^2 <= gc2
};

// Per primitive pair, read by the density / back transforms.
struct PairAux {
  double p;
  double xpa[3], xpb[3];  // P - A, P - (B + L)
  double pref_rho;        // w c_a c_b N_a N_b K (pi/p)^{3/2} / Omega   (w = 1 on the diagonal block, 2 otherwise)
  double pref_j;          // 2 c_a c_b N_a N_b K (pi/p)^{3/2}            (factor 2: G half space)
  double alpha_a, alpha_b;  // primitive exponents (centre derivatives)
  double w;                 // 1 on the diagonal block (s, s, 0), 2 otherwise
  double pad;
};

// A unique (shell a, shell b, image) block with its primitive pairs [p0, p1).
struct BlockRec {
  int sa, sb;
  int img;      // index into the image table
  int p0, p1;   // primitive pairs (global pair index)
  int bfa, bfb; // first basis function of each shell
  int w2;       // 1 if the mirror block (sb, sa, -m) is folded in (weight 2)
  int64_t eoff; // offset of the ncart(la) x ncart(lb) element block
};

// Entry of the J(k) gather list of an ordered shell pair (sa, sb).
struct GatherEnt {
  int blk;  // block index
  int img;  // image index of the block
  int tr;   // 0: block is (sa,sb,m), element (a,b);  1: block is (sb,sa,m), element (b,a), image -m
  int pad;
};

}  // namespace pwdf
