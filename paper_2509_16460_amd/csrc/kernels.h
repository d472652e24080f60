// Device-side view of a plan and the kernel launchers of libpwdf.
#pragma once
#include <hip/hip_runtime.h>

#include "pwdf_internal.h"

namespace pwdf {

// Plain struct of device pointers and launch shapes (copied by value into launchers).
struct Dev {
  // sizes
  int nk, nbf, nshell, natm;
  int nseg, nslot, seg_len;
  int64_t nelem;
  double vol;
  // static plan data (device)
  const SegDesc *segs;
  const GPoint *pts;             // the half-space G vectors as a compact list (FP32-MFMA form)
  int npts;
  const double *slot_v;
  const PairHot *hot;
  const PairHot *hot_rho;        // pair records in the rho pass's order (sorted by p for L <= 2)
  const int *rho_rank;           // pair -> position in that order (where its coefficients go)
  const PairHot *hot_cut;        // pair records by cut radius per class (J pass, FP32-MFMA rho pass)
  const int *cut_rank;           // pair -> position in that order (J moments, FP32-MFMA coefficient rows)
  const int *blk_cut;            // blocks of each (la, lb) class in that order: neighbouring lanes / waves
                                 // of the back transform read neighbouring moments
  const PairAux *aux;
  const BlockRec *blocks;
  const int *elem_blk;
  const int *sh_l;
  const int *sh_atom;
  const double2 *phD, *phJ;
  const int *sp_off;
  const GatherEnt *sp_ent;
  const int *bf_shell, *bf_comp;
  // phase sums by Born-von Karman class (see plan.h)
  int nsegJ, nsegD, nsegDp;
  const int *sJ_off, *sJ_code, *sJ_e0, *eJ;
  const int *sD_el, *sD_code, *sD_e0, *eD;
  const int *sDp_el, *sDp_code, *sDp_e0, *eDp;  // the same for a packed D(k)
  const int *heavyJ;             // elements with more than kPhaseLight J classes
  int nheavyJ;
  const int *lightJ;             // the other support elements (1 .. kPhaseLight classes), ascending
  int nlightJ;
  int jk_layout;                 // pwdf_jk_layout: 0 every element, 1 the support in place, 2 packed
  int dk_layout;                 // pwdf_dk_layout: 0 dense D(k), 1 packed on the J(k) support
  int pair_gcut;                 // 1: pairs carry their own cut radius (PairHot::gc2)
  double muu;                    // M_uu = |b_u|^2: |G|^2 along a line grows by steps of 2 M_uu
  int *nonfinite;                // set to 1 by phase_d when a D(L) phase sum is not finite
  double *Jfold;                 // [ndm][nsegJ]
  const double2 *ptab;           // e^{2 pi i t / N}
  int ptab_len;
  int kmesh[3];                  // k-point k = (k1 n2 + k2) n3 + k3
  const double *ttab;
  const double *start_tab;       // 2^(j/32) (32), then (cos, sin)(2 pi j/64), j = -32..32
  int cls_b0[16], cls_b1[16];
  int L_p0[kMaxLsum + 1], L_p1[kMaxLsum + 1];
  int64_t dhat_off[kMaxLsum + 1];
  int64_t dhat_size;
  // workspaces (device), sized for max_ndm densities
  double *Dblk, *Jblk;     // [ndm][nelem]
  double *dhat;            // [ndm][dhat_size]
  double *yhat;            // [ndm][yhat_size]
  double2 *part;           // [ndm][nrows][nslot] (FP64), [ndm][nrows][tail points] (FP32-MFMA)
  double2 *part2;          // [ndm][ngroups][nslot]
  double2 *rho, *Vc;       // [ndm][nslot]
  double *Epart;           // [ndm][nred_blocks]
  // FP32-MFMA form: operands [pair][k * ndmp + dm] per class (columns padded to
  // 16), W'[slot][k * ndmp + dm] for the J pass; ndmp = densities padded to a
  // power of two (<= 16)
  int fp32;
  int ndmp;
  float *dh32;
  int64_t d32_off[kMaxLsum + 1];
  int64_t d32_size;  // floats of all classes
  int ncols32[kMaxLsum + 1];
  float *wre, *wim;
  double *wre64, *wim64;  // W' of the head points in FP64, [head point][k * ndmp + dm]
  int ncolsW;
  // The FP32-MFMA form splits the G set into its head, pts[0, npts_head) (FP64
  // tiles on FP64 MFMA), and the tail (FP32 tiles), both in order of |G|^2, and
  // runs both passes as lists of work items (int4 per item):
  //   rho over the tail: (point block b of 64, pair range [q0, q1) of the class
  //     in cut order, row): the pairs whose cut reaches the block's shortest G;
  //     partial rows [ndm][nrows][tail point], block b using rows [0,
  //     rows_of_block[b]);
  //   J over the tail: (pair block B of 64 in cut order, point range [s0, s1),
  //     chunk c): the points inside the block's largest cut; the moments of
  //     chunk c go to yhat chunk jh_chunks[L] + c, the head's chunks come first,
  //     and a pair's back transform sums jn_of[cut rank] chunks;
  //   rho over the head: chunks of pairs x N-tile groups, partial rows
  //     [ndm][nrows_h][head point].
  // slot_pidx maps a slot to its point (-1 for padding slots).
  int npts_head;
  const int *slot_pidx;
  const int4 *rho_items, *j_items;
  int rho_item0[kMaxLsum + 1], rho_nitems[kMaxLsum + 1];
  // rho over the tail: N-tile groups per slice of grid z (each slice with a
  // partial row of its own: rows [row, row + slices) of an item) and slices
  int rho_gps[kMaxLsum + 1], rho_zs[kMaxLsum + 1];
  int j_item0[kMaxLsum + 1], j_nitems[kMaxLsum + 1];
  const int *rows_of_block;
  // FP32-MFMA form: the relative monomials n_u^a n_v^b n_w^c of every point of
  // pts, [point][kMonoStride] in the order of Monos
  const double *ptmono;
  // the slots holding a G of the half space, in walk order (pwdf_get_rhoG)
  const int *valid_slots;
  int nvalid;
  const int *jn_of;
  double2 *parth;
  int nrows_h, rows_per_group_h;
  int rho_h_chunks[kMaxLsum + 1], rho_h_ppc[kMaxLsum + 1], rho_h_row0[kMaxLsum + 1];  // rows: chunk x tile group
  // J over the head: jh_chunks[L] chunks of jh_ppc[L] head points each, yhat
  // chunks [0, jh_chunks[L]) of the class; the tail's chunks follow them
  int jh_chunks[kMaxLsum + 1], jh_ppc[kMaxLsum + 1];
  // gradient: moments of degree L+1 per class, per-block centre gradients,
  // per-atom lists of (block, 0 = shell a / 3 = shell b)
  double *yF;
  int64_t yF_off[kMaxLsum + 1];
  int64_t yF_size;
  double *gblk;              // [ndm][nblocks][6]
  int nblocks;
  const int *atom_off, *atom_ent;
  // compact/diffuse classification (ndd > 0): the DD pairs (global pair index,
  // class L), pair -> DD index or -1 (null without DD pairs), the full-range
  // kernel per slot; rho_D and conj V_D per slot [ndm][nslot]; the DD pairs' J
  // moments and force moments [ndm][ndd][kDDStride] (raw moments as the J pass
  // writes them, read by the back transform and the force contraction instead of
  // the pair's chunks)
  int ndd;
  int dd_chunks, dd_ppc;  // rho_D: chunks of dd_ppc DD pairs, partial rows rhoDp [ndm][dd_chunks][nslot]
  double2 *rhoDp;
  const int *dd_q, *dd_L, *dd_of;
  const double *slot_vf;
  double2 *rhoD, *VDc;
  double *ydd, *yddF;
  // GPW route of the DD pairs (gpw = 1; see Plan::gN): grid sizes, the DD pairs'
  // blocks, centres and cut radii, image entries and their grid boxes, tile
  // lists; the lattice (lat[c * 3 + i] = component c of a_i); the slot Miller
  // indices; workspaces: a real grid [ndm][gpts] (density, then V(r)), complex
  // intermediates of the separable transforms ([ndm][N2][N1][K0],
  // [ndm][N2][K1][K0], [ndm][K2][K1][K0], K_i = 2 gM_i + 1) and the DD pairs'
  // J partials [ndm][ndd][kGpwEl]; the collocation's work items (gitem,
  // gitem_off) and their partial tiles grid_p [ndm][ngitems][512]
  int gpw;
  int gN[3], gM[3], gtiles[3];
  int64_t gpts;
  double lat[9];
  const int *dd_blk;
  const double *gP;
  const int *gimg, *gimg_box, *gimg_off, *gtile_ent, *gitem, *gitem_off;
  int ngitems;
  double *grid_p;
  const int *slot_miller;
  double *grid_r;
  double2 *grid_a, *grid_b, *grid_c;
  double *gpw_part;
  // launch shapes
  int ndb;  // densities per block of the low-L pair-G launches (1, 2 or 4)
  int rho_bs;
  int rho_chunks[kMaxLsum + 1], rho_ppc[kMaxLsum + 1], rho_row0[kMaxLsum + 1];
  int nrows;
  int ngroups, rows_per_group;  // first stage of the row reduction
  int j_chunks[kMaxLsum + 1], j_spc[kMaxLsum + 1];
  int64_t yhat_off[kMaxLsum + 1];
  int64_t yhat_size;
  int nred_blocks;
};

// moments per DD pair and density: every degree up to the force moments of L = 6
constexpr int kDDStride = nherm(kMaxLsum);
// Cartesian elements of a pair block, at most (3,3)
constexpr int kGpwEl = 100;

// Allocation-free J build: the per-call workspaces are carved out of a static
// device array of this many bytes (one per device, held for the process's life).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
// device address of that array on `device` (looked up once per device)
hipError_t static_scratch(int device, void **ptr);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t st);

// MFMA-tile kernels: N-tiles (16 columns of (k, dm)) per S evaluation; ntiles
// are split into ceil(ntiles / 8) groups of equal size (at most 8 tiles each),
// the last group's missing tiles being zero columns
// monomials per point in Dev::ptmono (every degree up to 2 kMaxL)
constexpr int kMonoStride = nherm(2 * kMaxL);

inline int group_tiles(int ntiles) {
  const int ng = (ntiles + 7) / 8;
  return (ntiles + ng - 1) / ng;
}
inline int tile_groups(int ntiles) {
  const int g = group_tiles(ntiles);
  return (ntiles + g - 1) / g;
}

// FP32-MFMA form (per class L)
hipError_t launch_rho_mfma_L(const Dev &d, int L, int ndm, hipStream_t st);
hipError_t launch_wprep(const Dev &d, int ndm, hipStream_t st);
hipError_t launch_jpass_mfma_L(const Dev &d, int L, int ndm, hipStream_t st);
// the head of the FP32-MFMA form (FP64 MFMA, per class L)
hipError_t launch_rho_head_L(const Dev &d, int L, int ndm, hipStream_t st);
hipError_t launch_jpass_head_L(const Dev &d, int L, int ndm, hipStream_t st);
// FP64 path: one launch per pass over all classes
hipError_t launch_phase_d(const Dev &d, const double *Dk, int ndm, hipStream_t st);
hipError_t launch_transform_all(const Dev &d, int ndm, hipStream_t st);
hipError_t launch_back_all(const Dev &d, int ndm, hipStream_t st);
// rho of the class group 0 (L <= 2) or 1 (L >= 3)
hipError_t launch_rho_group(const Dev &d, int group, int ndm, hipStream_t st);
// EJ null: leave the energy partials for the J(k) launch to sum
hipError_t launch_reduce(const Dev &d, int ndm, double *EJ, hipStream_t st);
// J moments (force = false) or force moments of degree L+1 (force = true) of the
// class group 0 (L <= 2) or 1 (L >= 3)
hipError_t launch_jpass_group(const Dev &d, int group, bool force, int ndm, hipStream_t st);
bool jpass_group_nonempty(const Dev &d, int group);
hipError_t launch_fold_j(const Dev &d, int ndm, hipStream_t st);
// EJ non-null: one more block per density sums the energy partials into EJ
hipError_t launch_phase_j(const Dev &d, int ndm, double *Jk, double *EJ, hipStream_t st);
// compact/diffuse classification: rho_D of the DD pairs, then V_C, V_D, rho =
// rho_C + rho_D and the energy partials from rho_C (the reduce's rho) and rho_D;
// the DD pairs' moments from V_D (force = true: degree L+1); E_J from the
// energy partials
hipError_t launch_rho_dd(const Dev &d, int ndm, hipStream_t st);
hipError_t launch_combine_dd(const Dev &d, int ndm, hipStream_t st);
hipError_t launch_jpass_dd(const Dev &d, bool force, int ndm, hipStream_t st);
hipError_t launch_energy(const Dev &d, int ndm, double *EJ, hipStream_t st);
// E_J from the D(L) and J(L) blocks; part holds 256 doubles per density
hipError_t launch_energy_real(const Dev &d, int ndm, double *part, double *ER, hipStream_t st);
// rho of the valid slots, [ndm][nvalid], gathered from Dev::rho
hipError_t launch_gather_rho(const Dev &d, int ndm, double2 *out, hipStream_t st);
// GPW route: rho_D from the DD pairs' density on the grid (collocation and a
// separable transform onto the G set); V_D onto the grid and the DD pairs' J
// blocks by integration, added to J(L) after the back transform
hipError_t launch_gpw_rho(const Dev &d, int ndm, hipStream_t st);
hipError_t launch_gpw_j(const Dev &d, int ndm, hipStream_t st);
hipError_t launch_gpw_add(const Dev &d, int ndm, hipStream_t st);
// gradient
hipError_t launch_force_back_cls(const Dev &d, int la, int lb, int ndm, hipStream_t st);
hipError_t launch_force_atoms(const Dev &d, int ndm, double *dEdR, hipStream_t st);

}  // namespace pwdf
