// Host-side plan of libpwdf: everything that depends on the geometry, the basis
// and the k-mesh but not on the density.
#pragma once
#include <array>
#include <string>
#include <vector>

#include "pwdf_internal.h"

namespace pwdf {

struct PlanInput {
  double lattice[9];
  int natm;
  std::vector<double> xyz;
  int nshell;
  std::vector<int> sh_atom, sh_l, sh_nprim;
  std::vector<double> exps, coefs;
  int kmesh[3];
  double omega, eps_pair, eps_G, r_max;
  int pair_gcut = 0;  // 1: every pair block gets its own cut radius (section "Integral screening")
  // > 0: compact/diffuse classification (section "Density classification:
  // compact and diffuse"): pairs of two primitives with exponents below it are
  // DD pairs, taken with the full-range kernel against everything
  double alpha_cut = 0.0;
  // 1: the DD pairs' density and J go through a real-space grid (GPW, appendix
  // "Evaluation of density on real space grid (GPW)") instead of their analytic
  // transforms
  int dd_gpw = 0;
};

// Default relative Coulomb weight that bounds the head of the G set (see
// Plan::npts_head): with 2^-20 the FP32 tail carries a small enough share of the
// energy and of J that its rounding stays near 1e-9 Eh in E_J and 2e-10 in J on
// the rock-salt slab (E_J ~3.4e3 Eh, max|J| ~29), against targets of 1e-7 Eh and
// 1e-8 (2^-16: 6e-8 Eh and up to 1.2e-8 in J over the tuner's shapes).
constexpr double kHeadWeight = 1.0 / 1048576.0;

struct Plan {
  PlanInput in;
  // geometry: A[c][i] = component c of a_i; B = 2 pi A^-T; M = B^T B
  double A[3][3], B[3][3], M[3][3], vol;
  int ax[3];  // relative axes in (u, v, w) order: u is the line axis
  // basis
  std::vector<int> sh_bf, sh_pr;
  int nbf = 0, nk = 0;
  std::vector<int> bf_shell, bf_comp;
  // reciprocal space: segments of lines, padded to seg_len slots each
  int seg_len = 8;
  std::vector<SegDesc> segs;
  std::vector<double> slot_v;       // v(G) per slot, 0 on padding
  std::vector<int> slot_miller;     // [nslot][3] in the original axis order (padding: 0,0,0)
  std::vector<int> valid_slots;     // slots holding a G, in walk order
  std::vector<GPoint> pts;          // the same G vectors as a compact point list, by |G|^2
  // The head of the G set: the vectors whose Coulomb weight v(G) is at least
  // head_weight times the largest one (the shortest |G|).  The FP32-MFMA form
  // evaluates them with FP64 tiles; pts[0, npts_head) are the head.
  double head_weight = kHeadWeight;
  int npts_head = 0;
  double head_g2 = 0.0;             // largest |G|^2 of the head
  double pairG_head = 0.0;          // sum over pairs of the head G within their cut (per pass)
  double pairG_head_L[kMaxLsum + 1];  // per class L
  int64_t nG_full = 0;              // |G set| including -G
  double pairG_cut = 0.0;           // sum over pairs of the half-space G within their cut (per pass)
  std::vector<double> pairG_of;     // per pair: half-space G within its cut
  double pairG_L[kMaxLsum + 1];     // per class L: sum of pairG_of
  // lattice images of the pair list
  std::vector<std::array<int, 3>> imgs;
  // unique blocks and primitive pairs, sorted by (L = la+lb, la, sa, sb, m)
  std::vector<BlockRec> blocks;
  std::vector<PairHot> hot;
  std::vector<PairAux> aux;
  int cls_b0[16], cls_b1[16];  // block range of class (la, lb), index la*4 + lb
  int L_p0[kMaxLsum + 1], L_p1[kMaxLsum + 1];  // pair range of class L
  // The rho pass walks each class range [L_p0, L_p1) in its own order: sorted by
  // p (stable) for L <= 2, so that consecutive pairs mostly share e^{-|G|^2/4p},
  // storage order for L >= 3.  rho_rank[pair] is the pair's position in that walk
  // (the density transform writes its coefficients there), hot_rho the pair
  // records in walk order.
  std::vector<int> rho_rank;
  std::vector<PairHot> hot_rho;
  // The J pass (both forms) and the FP32-MFMA rho pass walk each class by cut
  // radius, largest first, so that the pairs of a wave or a tile share similar
  // cuts and skip the same G: cut_rank[pair] is the position in that walk (of the
  // J moments and the FP32-MFMA coefficient rows), hot_cut the records in it.
  std::vector<int> cut_rank;
  std::vector<PairHot> hot_cut;
  std::vector<int> blk_cut;  // blocks of each (la, lb) class in that walk (back transform)
  int64_t dhat_off[kMaxLsum + 1];             // offset of class L in a per-density coefficient array
  int64_t dhat_size = 0;
  int64_t nelem = 0;                          // sum over blocks of ncart(la) ncart(lb)
  std::vector<int> elem_blk;                  // element -> block
  // phase tables [nimg][nk] complex: w_k e^{ik.L} and e^{ik.L}
  std::vector<double> phD, phJ;
  // J(k) gather lists per ordered shell pair
  std::vector<int> sp_off;
  std::vector<GatherEnt> sp_ent;
  // Phase sums by Born-von Karman class.  e^{ik.L} depends on the image m only
  // through c_i = (m_i mod n_i) N / n_i (N = lcm(n1, n2, n3)): for the k-point
  // (k1, k2, k3), k.L / 2 pi = (k1 c1 + k2 c2 + k3 c3) / N.  The block entries of
  // every matrix element (mu, nu) are grouped into segments of equal class
  // (code = c1 | c2 << 10 | c3 << 20), at most Nk per element:
  //   J side: all entries (mirror entries carry the class of -m and the
  //           transposed element offset), segments ordered by element;
  //   D side: direct entries only (each block element once).
  std::vector<int> sJ_off;          // [nbf*nbf + 1] first J segment of each element
  std::vector<int> sJ_code, sJ_e0;  // per J segment: class code; first entry ([nsegJ + 1])
  std::vector<int> eJ;              // per J entry: element offset in Jblk
  std::vector<int> sD_el, sD_code, sD_e0;  // per D segment: element, class code, first entry
  int64_t nD_support = 0;                  // elements with at least one D segment
  // D side for a packed D(k) (the J(k) support in the packed element order):
  // the same entries, each read at (mu, nu) with shell(mu) <= shell(nu) so that
  // the values read from a row are one run at its end; element = packed index
  std::vector<int> sDp_el, sDp_code, sDp_e0, eDp;
  int64_t nDp_support = 0;  // packed elements read
  // elements with more than kPhaseLight J classes, summed one wave per element
  // (the others one thread per element)
  std::vector<int> heavyJ;
  // the other elements of the J(k) support (1 .. kPhaseLight classes), ascending:
  // the light path of a support-only J(k) launch walks this list instead of every
  // element of the matrix
  std::vector<int> lightJ;
  // largest |G|^2 / 4p and |G(n+1)|^2 - |G(n)|^2 over 4p of any pair and G line
  // point: the segment-start exponentials are evaluated without range handling
  double max_start_arg = 0.0;
  std::vector<int> eD;                      // per D entry: element offset in Dblk
  int phN = 1;                        // N
  std::vector<double> ptab;           // e^{2 pi i t / N}, t = 0 .. (n1+n2+n3) N - 1
  // block-diagonal Hermite -> relative-monomial transform (degree blocks), and
  // the sign of (-i)^{|k|} folded into the rho coefficients / J moments
  std::vector<double> ttab;

  // DD pairs (both exponents below alpha_cut): their gc2 is -1, so the pair-G
  // passes of the compact pairs skip them; dd_q lists them (global pair index),
  // dd_L their class L, dd_of[pair] their index in that list or -1.  slot_vf is
  // the full-range kernel 4 pi/|G|^2 per slot (0 on padding).
  std::vector<int> dd_q, dd_L, dd_of;
  std::vector<double> slot_vf;
  // GPW route of the DD pairs (in.dd_gpw): a grid of gN[i] points along a_i
  // (original axis order), gN[i] = 2 ceil(1.25 gM[i]) + 1 with gM[i] the largest
  // |n_i| of the G set, so that every G of the set aliases only onto |G'| beyond
  // the cutoff sphere.  Per DD pair: its block, centre P and squared cut radius
  // (gP: x, y, z, rc^2); its lattice images whose ball reaches the cell (gimg:
  // dd index, m0, m1, m2; gimg_box: grid index box lo0 hi0 lo1 hi1 lo2 hi2 inside
  // the cell; gimg_off[dd] first entry), and per tile of 8^3 grid points the image
  // entries whose box meets it (gtile_off, gtile_ent).  The collocation's work
  // items cut each tile's list into runs of at most glen entries (gitem: tile,
  // first entry, end entry; gitem_off[tile] its first item), so that a small grid
  // still spreads over enough workgroups.
  int gN[3] = {0, 0, 0}, gM[3] = {0, 0, 0};
  int gtiles[3] = {0, 0, 0};
  int glen = 0;
  std::vector<int> dd_blk;
  std::vector<double> gP;
  std::vector<int> gimg, gimg_box, gimg_off, gtile_off, gtile_ent, gitem, gitem_off;

  // the pair-G kernels must honour gc2 (per-pair cuts, or DD pairs to skip)
  bool cut_on() const { return in.pair_gcut != 0 || !dd_q.empty(); }

  int nseg() const { return (int)segs.size(); }
  int nslot() const { return (int)segs.size() * seg_len; }
  int npairs() const { return (int)hot.size(); }
  int nimg() const { return (int)imgs.size(); }
};

// Validates and builds; returns an empty string on success, else the reason.
std::string build_plan(const PlanInput &in, int seg_len, Plan &out);

// Rebuild only the reciprocal-space segments for another segment length.
void build_segments(Plan &p, int seg_len);

// Set the relative weight that bounds the head of the G set (0 < weight <= 1)
// and recount the head's points and pair-G work.
void set_head_weight(Plan &p, double weight);

}  // namespace pwdf
